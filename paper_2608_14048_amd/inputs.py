"""Seeded synthetic initial states in the canonical layout.

This module builds inputs only: it holds none of the Godunov step's arithmetic and is
the one module that both the HIP library's callers and the CPU oracle's tests use.

Canonical state (FP64, one flat array):
  cell fields [nvar][nz][ny][nx], x fastest --
      adiabatic MHD     : rho, M1, M2, M3, E, then face fields b1, b2, b3
      isothermal + dust : rho, M1, M2, M3, then per species rho_k, M_k1, M_k2, M_k3
  b1[k][j][i] is B_x on the face x_{i-1/2}; b2, b3 likewise on y_{j-1/2}, z_{k-1/2}.

The magnetic field of every MHD state is the discrete curl of an edge-centred vector
potential, so div B = 0 to round-off on the faces, as in the paper's problem set-up
interface (Sec. "User Interface, Problem Setup, and Execution Modes": primitive
functions plus a vector potential).  A_x lives on the edges (i, j-1/2, k-1/2), A_y on
(i-1/2, j, k-1/2), A_z on (i-1/2, j-1/2, k).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    """A synthetic workload: grid, physics, scheme and its initial canonical state."""
    name: str
    shape: tuple            # (nx, ny, nz)
    length: tuple           # box edges (Lx, Ly, Lz); origin irrelevant (periodic)
    state: np.ndarray       # canonical FP64 state
    physics: dict = field(default_factory=dict)
    scheme: dict = field(default_factory=dict)
    nsteps: int = 1


# ---------------------------------------------------------------------------------
# assembling a state from primitives and a vector potential
# ---------------------------------------------------------------------------------

def faces_from_potential(ax, ay, az, dx, dy, dz):
    """Face fields b = curl A from edge potentials (arrays [nz][ny][nx], periodic)."""
    def up(a, axis):  # value at index + 1 along a numpy axis (0 = z, 1 = y, 2 = x)
        return np.roll(a, -1, axis=axis)
    b1 = (up(az, 1) - az) / dy - (up(ay, 0) - ay) / dz
    b2 = (up(ax, 0) - ax) / dz - (up(az, 2) - az) / dx
    b3 = (up(ay, 2) - ay) / dx - (up(ax, 1) - ax) / dy
    return b1, b2, b3


def cell_centred_field(b1, b2, b3):
    """Mean of the two bounding faces per component."""
    bx = 0.5 * (b1 + np.roll(b1, -1, axis=2))
    by = 0.5 * (b2 + np.roll(b2, -1, axis=1))
    bz = 0.5 * (b3 + np.roll(b3, -1, axis=0))
    return bx, by, bz


def mhd_state(rho, vx, vy, vz, eint, b1, b2, b3):
    """Canonical adiabatic-MHD state from cell primitives (internal energy density
    eint = rho e, as the paper's set-up functions return it) and face fields."""
    bx, by, bz = cell_centred_field(b1, b2, b3)
    E = eint + 0.5 * rho * ((vx * vx + vy * vy) + vz * vz) + 0.5 * ((bx * bx + by * by) + bz * bz)
    parts = [rho, rho * vx, rho * vy, rho * vz, E, b1, b2, b3]
    return np.concatenate([np.ascontiguousarray(p, dtype=np.float64).ravel() for p in parts])


def dust_state(fluids):
    """Canonical isothermal-gas + dust state; fluids = [(rho, vx, vy, vz), ...], gas first."""
    parts = []
    for rho, vx, vy, vz in fluids:
        parts += [rho, rho * vx, rho * vy, rho * vz]
    return np.concatenate([np.ascontiguousarray(p, dtype=np.float64).ravel() for p in parts])


def cell_centres(shape, length, origin=(0.0, 0.0, 0.0)):
    """Cell-centre coordinates as [nz][ny][nx] arrays (x, y, z)."""
    nx, ny, nz = shape
    xs = origin[0] + (np.arange(nx) + 0.5) * length[0] / nx
    ys = origin[1] + (np.arange(ny) + 0.5) * length[1] / ny
    zs = origin[2] + (np.arange(nz) + 0.5) * length[2] / nz
    z, y, x = np.meshgrid(zs, ys, xs, indexing="ij")
    return x, y, z


def edge_coords(shape, length, axis):
    """Coordinates of the edges that carry A_axis (centred along axis, at the lower
    faces in the two other directions)."""
    nx, ny, nz = shape
    dx, dy, dz = (length[a] / shape[a] for a in range(3))
    x = np.arange(nx) * dx + (0.5 * dx if axis == 0 else 0.0)
    y = np.arange(ny) * dy + (0.5 * dy if axis == 1 else 0.0)
    z = np.arange(nz) * dz + (0.5 * dz if axis == 2 else 0.0)
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    return X, Y, Z


# ---------------------------------------------------------------------------------
# 3D linear fast magnetosonic wave along the grid diagonal
# ---------------------------------------------------------------------------------

WAVE_FRAME = (
    np.array([1.0, 1.0, 1.0]) / math.sqrt(3.0),
    np.array([-1.0, 1.0, 0.0]) / math.sqrt(2.0),
    np.array([-1.0, -1.0, 2.0]) / math.sqrt(6.0),
)


def mhd_primitive_jacobian(rho, p, bn, bt1, bt2, gamma, u=0.0):
    """7x7 matrix A of the 1D primitive system dW/dt + A dW/dx = 0 for
    W = (rho, u, v, w, p, B_t1, B_t2) with constant normal field bn."""
    A = np.zeros((7, 7))
    A[0, 0] = u; A[0, 1] = rho
    A[1, 1] = u; A[1, 4] = 1.0 / rho; A[1, 5] = bt1 / rho; A[1, 6] = bt2 / rho
    A[2, 2] = u; A[2, 5] = -bn / rho
    A[3, 3] = u; A[3, 6] = -bn / rho
    A[4, 1] = gamma * p; A[4, 4] = u
    A[5, 1] = bt1; A[5, 2] = -bn; A[5, 5] = u
    A[6, 1] = bt2; A[6, 3] = -bn; A[6, 6] = u
    return A


def fast_eigenmode(rho=1.0, p=None, b0=(1.0, math.sqrt(2.0), 0.5), gamma=5.0 / 3.0):
    """Right-going fast eigenpair (speed, eigenvector normalised to drho = 1)."""
    if p is None:
        p = 1.0 / gamma
    A = mhd_primitive_jacobian(rho, p, b0[0], b0[1], b0[2], gamma)
    vals, vecs = np.linalg.eig(A)
    i = int(np.argmax(vals.real))
    r = vecs[:, i].real
    return float(vals[i].real), r / r[0]


def box_wave_frame(length):
    """Wave frame of the oblique wave with one wavelength across each side of a box:
    k = 2 pi (1/Lx, 1/Ly, 1/Lz), e1 = k/|k|, e2 = z^ x e1 normalised, e3 = e1 x e2."""
    kvec = 2.0 * math.pi / np.asarray(length, dtype=np.float64)
    e1 = kvec / np.linalg.norm(kvec)
    e2 = np.array([-e1[1], e1[0], 0.0])
    e2 /= np.linalg.norm(e2)
    return kvec, (e1, e2, np.cross(e1, e2))


def linear_wave(n=32, amp=1e-6, gamma=5.0 / 3.0, b0=(1.0, math.sqrt(2.0), 0.5), t=0.0,
                along="diagonal", shape=None):
    """Fast wave of amplitude amp at time t (the exact linear solution).

    along="diagonal": [0,1]^3, n^3 cells, k = 2 pi (1,1,1), period (1/sqrt 3)/c_f.
    along="x": n x 1 x 1 cells, k = 2 pi x^.
    along="box": shape = (nx, ny, nz) cells of equal spacing 1/nz, box
    [0, nx/nz) x [0, ny/nz) x [0, 1), one wavelength across each side (the oblique
    wave of a 512 x 512 x 256 benchmark box is shape=(512, 512, 256)).
    Returns (state, period)."""
    if along == "diagonal":
        shape = (n, n, n)
        e1, e2, e3 = WAVE_FRAME
        kvec = 2.0 * math.pi * np.array([1.0, 1.0, 1.0])
        length = (1.0, 1.0, 1.0)
    elif along == "x":
        shape = (n, 1, 1)
        e1, e2, e3 = np.eye(3)
        kvec = 2.0 * math.pi * np.array([1.0, 0.0, 0.0])
        length = (1.0, 1.0 / n, 1.0 / n)
    else:
        shape = tuple(int(s) for s in shape)
        n = shape[2]
        length = (shape[0] / n, shape[1] / n, 1.0)
        kvec, (e1, e2, e3) = box_wave_frame(length)
    rho0, p0 = 1.0, 1.0 / gamma
    cf, r = fast_eigenmode(rho0, p0, b0, gamma)
    kmag = float(np.linalg.norm(kvec))
    omega = cf * kmag
    x, y, z = cell_centres(shape, length)
    ph = kvec[0] * x + kvec[1] * y + kvec[2] * z - omega * t
    s = amp * np.sin(ph)
    rho = rho0 + r[0] * s
    vel = [(r[1] * e1[a] + r[2] * e2[a] + r[3] * e3[a]) * s for a in range(3)]
    p = p0 + r[4] * s
    # magnetic perturbation R_B sin(k.x - wt) from A = amp (k x R_B) cos(k.x - wt) / |k|^2
    rb = r[5] * e2 + r[6] * e3
    avec = amp * np.cross(kvec, rb) / kmag ** 2
    bmean = b0[0] * e1 + b0[1] * e2 + b0[2] * e3
    dx = 1.0 / n
    pots = []
    for a in range(3):
        X, Y, Z = edge_coords(shape, length, a)
        pots.append(avec[a] * np.cos(kvec[0] * X + kvec[1] * Y + kvec[2] * Z - omega * t))
    b1, b2, b3 = faces_from_potential(*pots, dx, dx, dx)
    b1 = b1 + bmean[0]; b2 = b2 + bmean[1]; b3 = b3 + bmean[2]
    state = mhd_state(rho, vel[0], vel[1], vel[2], p / (gamma - 1.0), b1, b2, b3)
    period = (2.0 * math.pi / kmag) / cf
    return state, period


# ---------------------------------------------------------------------------------
# decaying MHD turbulence
# ---------------------------------------------------------------------------------

def _random_field(rng, n, kmin, kmax, slope_amp, shift):
    """Real Gaussian random field on an n^3 periodic grid sampled at offset `shift`
    (fractions of a cell per axis x,y,z): Fourier amplitudes ~ |k|^slope_amp on
    kmin <= |k| <= kmax (integer wavenumbers), zero elsewhere."""
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    kr = np.fft.rfftfreq(n, d=1.0 / n)
    KZ, KY, KX = np.meshgrid(k1, k1, kr, indexing="ij")
    kk = np.sqrt(KX * KX + KY * KY + KZ * KZ)
    band = (kk >= kmin) & (kk <= kmax)
    amp = np.zeros_like(kk)
    amp[band] = kk[band] ** slope_amp
    spec = (rng.standard_normal(kk.shape) + 1j * rng.standard_normal(kk.shape)) * amp
    phase = np.exp(2j * math.pi * (KX * shift[0] + KY * shift[1] + KZ * shift[2]) / n)
    return np.fft.irfftn(spec * phase, s=(n, n, n), axes=(0, 1, 2))


def turbulence(n=256, seed=0, gamma=5.0 / 3.0, sigma_lnrho=0.1, mach=1.0, beta=1.0,
               kmin=2.0, kmax=8.0):
    """Decaying MHD turbulence on [0,1]^3: rho = exp(sigma xi) per cell, a Gaussian
    velocity field with E(k) ~ k^-2 on kmin..kmax at rms Mach `mach` (c_s = 1 at
    rho = 1, p = 1/gamma), B = curl of a random edge potential with E_B(k) ~ k^-2,
    scaled to plasma beta `beta` (<|B_cc|^2> = 2 p / beta), no mean field."""
    rng = np.random.default_rng(seed)
    shape = (n, n, n)
    p0 = 1.0 / gamma
    rho = np.exp(sigma_lnrho * rng.standard_normal((n, n, n)))
    vel = [_random_field(rng, n, kmin, kmax, -2.0, (0.0, 0.0, 0.0)) for _ in range(3)]
    vel = [v - v.mean() for v in vel]
    vrms = math.sqrt(float(np.mean(vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)))
    vel = [v * (mach / vrms) for v in vel]
    # edge-staggered potential: A_x at (i, j-1/2, k-1/2) -> shift (0, -1/2, -1/2) etc.
    shifts = [(0.0, -0.5, -0.5), (-0.5, 0.0, -0.5), (-0.5, -0.5, 0.0)]
    pots = [_random_field(rng, n, kmin, kmax, -3.0, shifts[a]) for a in range(3)]
    dx = 1.0 / n
    b1, b2, b3 = faces_from_potential(*pots, dx, dx, dx)
    bx, by, bz = cell_centred_field(b1, b2, b3)
    b2mean = float(np.mean(bx * bx + by * by + bz * bz))
    scale = math.sqrt(2.0 * p0 / beta / b2mean)
    b1, b2, b3 = b1 * scale, b2 * scale, b3 * scale
    eint = np.full((n, n, n), p0 / (gamma - 1.0))
    state = mhd_state(rho, vel[0], vel[1], vel[2], eint, b1, b2, b3)
    return state


def _random_field_box(rng, shape, length, kmin, kmax, slope_amp, shift):
    """Real Gaussian random field on an nx x ny x nz periodic box of side lengths
    `length`, sampled at offset `shift` (fractions of a cell per axis x,y,z): Fourier
    amplitudes ~ |k|^slope_amp for kmin <= |k| <= kmax, |k| in units of 2 pi."""
    nx, ny, nz = shape
    fx = np.fft.rfftfreq(nx, d=1.0 / nx)
    fy = np.fft.fftfreq(ny, d=1.0 / ny)
    fz = np.fft.fftfreq(nz, d=1.0 / nz)
    MZ, MY, MX = np.meshgrid(fz, fy, fx, indexing="ij")  # integer mode numbers
    kk = np.sqrt((MX / length[0]) ** 2 + (MY / length[1]) ** 2 + (MZ / length[2]) ** 2)
    band = (kk >= kmin) & (kk <= kmax)
    amp = np.zeros_like(kk)
    amp[band] = kk[band] ** slope_amp
    spec = (rng.standard_normal(kk.shape) + 1j * rng.standard_normal(kk.shape)) * amp
    phase = np.exp(2j * math.pi * (MX * shift[0] / nx + MY * shift[1] / ny + MZ * shift[2] / nz))
    return np.fft.irfftn(spec * phase, s=(nz, ny, nx), axes=(0, 1, 2))


def turbulence_block(shape, seed=0, gamma=5.0 / 3.0, sigma_lnrho=0.1, mach=1.0, beta=1.0,
                     kmin=2.0, kmax=8.0):
    """The turbulence recipe on one self-periodic block of nx x ny x nz cells with equal
    spacing, box lengths n_a / max(n) (the longest side is 1).  Returns (state, length)."""
    nx, ny, nz = (int(v) for v in shape)
    nmax = max(nx, ny, nz)
    length = (nx / nmax, ny / nmax, nz / nmax)
    rng = np.random.default_rng(seed)
    full = (nz, ny, nx)
    p0 = 1.0 / gamma
    rho = np.exp(sigma_lnrho * rng.standard_normal(full))
    vel = [_random_field_box(rng, (nx, ny, nz), length, kmin, kmax, -2.0, (0.0, 0.0, 0.0))
           for _ in range(3)]
    vel = [v - v.mean() for v in vel]
    vrms = math.sqrt(float(np.mean(vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)))
    vel = [v * (mach / vrms) for v in vel]
    shifts = [(0.0, -0.5, -0.5), (-0.5, 0.0, -0.5), (-0.5, -0.5, 0.0)]
    pots = [_random_field_box(rng, (nx, ny, nz), length, kmin, kmax, -3.0, shifts[a])
            for a in range(3)]
    h = 1.0 / nmax
    b1, b2, b3 = faces_from_potential(*pots, h, h, h)
    bx, by, bz = cell_centred_field(b1, b2, b3)
    b2mean = float(np.mean(bx * bx + by * by + bz * bz))
    scale = math.sqrt(2.0 * p0 / beta / b2mean)
    b1, b2, b3 = b1 * scale, b2 * scale, b3 * scale
    eint = np.full(full, p0 / (gamma - 1.0))
    return mhd_state(rho, vel[0], vel[1], vel[2], eint, b1, b2, b3), length


BLOCK_EDGES = (16, 24, 32, 48, 64)


def meshblock_shapes(nblocks=512, seed=0, edges=BLOCK_EDGES):
    """Block shapes of the batched workload: each edge drawn independently and
    uniformly from `edges` (numpy PCG64 `seed`)."""
    rng = np.random.default_rng(seed)
    return [tuple(int(e) for e in rng.choice(edges, size=3)) for _ in range(nblocks)]


# ---------------------------------------------------------------------------------
# gas + dust under a gas-only acceleration (terminal drift + noise)
# ---------------------------------------------------------------------------------

def dust_stopping_times(nd=8, lo=1e-3, hi=10.0):
    """Log-spaced stopping times lo .. hi."""
    if nd == 1:
        return np.array([lo])
    return lo * (hi / lo) ** (np.arange(nd) / (nd - 1))


def dust_drift(n=192, seed=0, nd=8, eps=0.01, g=0.05, noise=1e-3, shape=None):
    """Isothermal gas (rho = 1) with nd dust species of density eps each, in the exact
    terminal-drift state of a gas-only acceleration g along x, centre-of-mass frame,
    plus i.i.d. N(0, noise^2) on every velocity component of every fluid.
    Returns (state, stopping times)."""
    if shape is None:
        shape = (n, n, n)
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    ts = dust_stopping_times(nd)
    rho_g = 1.0
    rho_tot = rho_g + nd * eps
    abar = g * rho_g / rho_tot
    vg = abar * float(np.sum(eps * ts)) / rho_tot
    fluids = []
    full = (nz, ny, nx)
    vels = [vg] + [vg - abar * t for t in ts]
    rhos = [rho_g] + [eps] * nd
    for r, v in zip(rhos, vels):
        fluids.append((np.full(full, r),
                       v + noise * rng.standard_normal(full),
                       noise * rng.standard_normal(full),
                       noise * rng.standard_normal(full)))
    return dust_state(fluids), ts


# ---------------------------------------------------------------------------------
# one-dimensional problems run on thin 3D grids
# ---------------------------------------------------------------------------------

def sod_doubled(n=1024, gamma=1.4, axis=0):
    """Sod's shock tube on the doubled periodic domain [-1, 1): (rho, p) = (1, 1) for
    |x| < 1/2, (0.125, 0.1) elsewhere, at rest, B = 0.  The Riemann problem at x = 1/2
    is the classical one; the domain is long enough that the two problems do not meet
    by t = 0.25.  `axis` picks the grid direction."""
    shape = [1, 1, 1]
    shape[axis] = n
    length = [2.0 / n, 2.0 / n, 2.0 / n]
    length[axis] = 2.0
    x = -1.0 + (np.arange(n) + 0.5) * 2.0 / n
    inside = np.abs(x) < 0.5
    rho1 = np.where(inside, 1.0, 0.125)
    p1 = np.where(inside, 1.0, 0.1)
    full = (shape[2], shape[1], shape[0])
    rho = rho1.reshape(full)
    p = p1.reshape(full)
    z = np.zeros(full)
    state = mhd_state(rho, z, z, z, p / (gamma - 1.0), z, z, z)
    return state, tuple(shape), tuple(length), x


def dusty_wave_matrix(eps, ts, k=2.0 * math.pi, cs=1.0, rho_g=1.0):
    """Linear system d/dt X = M X of the isothermal gas + dust equations about rest,
    X = (drho_g, dv_g, drho_1, dv_1, ...), perturbations ~ exp(i k x)."""
    nd = len(eps)
    m = 2 + 2 * nd
    M = np.zeros((m, m), dtype=complex)
    M[0, 1] = -1j * k * rho_g
    M[1, 0] = -1j * k * cs * cs / rho_g
    for s in range(nd):
        r, v = 2 + 2 * s, 3 + 2 * s
        M[1, 1] -= eps[s] / ts[s]
        M[1, v] += eps[s] / ts[s]
        M[r, v] = -1j * k * eps[s] * rho_g
        M[v, 1] = 1.0 / ts[s]
        M[v, v] = -1.0 / ts[s]
    return M


def dusty_wave_mode(eps, ts, k=2.0 * math.pi, cs=1.0):
    """Least-damped oscillatory eigenpair (lambda with Im > 0, eigenvector with
    drho_g = 1)."""
    vals, vecs = np.linalg.eig(dusty_wave_matrix(eps, ts, k, cs))
    osc = [i for i in range(len(vals)) if vals[i].imag > 1e-8]
    i = max(osc, key=lambda q: vals[q].real)
    v = vecs[:, i] / vecs[0, i]
    return vals[i], v


def dusty_wave(n=128, amp=1e-4, eps=(0.100, 0.233, 0.367, 0.500), ts=None, k=2.0 * math.pi):
    """Damped dusty sound wave on [0,1) (along x, thin 3D grid), from the eigenvector.
    Returns (state, lambda, eigenvector, cell centres)."""
    if ts is None:
        ts = 10.0 ** (-1.0 + np.arange(4) / 3.0)
    lam, vec = dusty_wave_mode(np.asarray(eps), np.asarray(ts), k)
    x = (np.arange(n) + 0.5) / n
    ph = np.exp(1j * k * x)
    full = (1, 1, n)
    zeros = np.zeros(full)
    fluids = []
    rho0 = [1.0] + list(eps)
    for s in range(len(rho0)):
        drho = (amp * vec[2 * s] * ph).real
        dv = (amp * vec[2 * s + 1] * ph).real
        fluids.append(((rho0[s] + drho).reshape(full), dv.reshape(full), zeros, zeros))
    return dust_state(fluids), lam, vec, x
