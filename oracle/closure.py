"""FP64 reference of the learned subgrid flux-correction closure -- TEST INFRASTRUCTURE
ONLY (imported by tests/, never by the library or its binding).

The closure is an extension of this project, not part of the paper's method: the paper
only remarks that a neural surrogate could stand in for an expensive cell-local solve
such as astrochemistry (Sec. "Discussion and Summary").  What is fixed here is the
construction around the network, which the method dictates:

* input: the 8 primitive channels of the coarse state at the start of a step
  (rho, v_x, v_y, v_z, p, B_x, B_y, B_z at cell centres; B_cc the mean of the two
  bounding faces, p from E as in Sec. "Newtonian Magnetohydrodynamics"), each
  normalised as (w - mu_c) / sd_c;
* network: 4 periodic 3x3x3 convolutions, widths 8 -> 32 -> 32 -> 32 -> 18, ReLU after
  the first three;
* output: 15 face-flux corrections (5 cell fields x 3 directions, on the low face of
  each cell) and 3 edge-EMF corrections (E_x on edge (i, j-1/2, k-1/2), E_y on
  (i-1/2, j, k-1/2), E_z on (i-1/2, j-1/2, k)), scaled by sF[f] and sE;
* closure: added to the plain coarse step in flux form, U_f -= dt sum_d
  (dF_fd[c + e_d] - dF_fd[c]) / dx_d, and in constrained-transport form for the faces,
  b -= dt curl(dE) (eq. (ct)), so mass, momentum and energy stay conservative and
  div B stays what the plain step leaves;
* loss: sum over cells of sum_f wU_f (P_f - T_f)^2 + sum_a wB (b'_a - Tb_a)^2, divided
  by the cell count, against the filtered fine state T.

Conventions shared with the HIP path (each side implements them independently):
tap t = (dz+1)*9 + (dy+1)*3 + (dx+1) with offsets in {-1, 0, 1};
conv: y[co, v] = b[co] + sum_{t, ci} W[t, ci, co] x[ci, v + off(t)] (periodic);
parameters, in order, for each layer l: W_l [27][cin_l][cout_l], then b_l [cout_l].
Arrays are [channel][z][y][x].
"""
from __future__ import annotations

import numpy as np

TAPS = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
WIDTHS = (8, 32, 32, 32, 18)
NLAYER = 4


def param_shapes(widths=WIDTHS):
    out = []
    for l in range(len(widths) - 1):
        out.append(((27, widths[l], widths[l + 1]), (widths[l + 1],)))
    return out


def param_count(widths=WIDTHS):
    return sum(int(np.prod(w)) + int(np.prod(b)) for w, b in param_shapes(widths))


def unpack(flat, widths=WIDTHS):
    """Flat parameter vector -> [(W_l, b_l)]."""
    out, at = [], 0
    for w, b in param_shapes(widths):
        nw, nb = int(np.prod(w)), int(np.prod(b))
        out.append((flat[at:at + nw].reshape(w), flat[at + nw:at + nw + nb].reshape(b)))
        at += nw + nb
    return out


def pack(params):
    return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in params])


def shift(a, off):
    """a[..., z, y, x] read at v + off (periodic)."""
    dx, dy, dz = off
    return np.roll(a, shift=(-dz, -dy, -dx), axis=(-3, -2, -1))


# ---------------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------------

def conv(x, W, b):
    y = np.zeros((W.shape[2],) + x.shape[1:]) + b[:, None, None, None]
    for t, off in enumerate(TAPS):
        y += np.einsum("czyx,cd->dzyx", shift(x, off), W[t])
    return y


def conv_grad_input(dy, W):
    """Adjoint of conv in its input: dx[ci, v] = sum_{t,co} W[t,ci,co] dy[co, v - off(t)]."""
    dx = np.zeros((W.shape[1],) + dy.shape[1:])
    for t, off in enumerate(TAPS):
        dx += shift(np.einsum("dzyx,cd->czyx", dy, W[t]), tuple(-o for o in off))
    return dx


def conv_grad_weight(x, dy):
    """dW[t, ci, co] = sum_v x[ci, v + off(t)] dy[co, v]; db[co] = sum_v dy[co, v]."""
    dW = np.stack([np.einsum("czyx,dzyx->cd", shift(x, off), dy) for off in TAPS])
    return dW, dy.sum(axis=(1, 2, 3))


def forward(params, x):
    """Returns the 18 output channels and the activations for the backward pass."""
    acts = [x]
    h = x
    for l, (W, b) in enumerate(params):
        z = conv(h, W, b)
        h = np.maximum(z, 0.0) if l < len(params) - 1 else z
        acts.append(h)
    return h, acts


def backward(params, acts, dout):
    """Gradients of every parameter from d(loss)/d(output)."""
    grads = [None] * len(params)
    g = dout
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        grads[l] = conv_grad_weight(acts[l], g)
        if l > 0:
            g = conv_grad_input(g, W) * (acts[l] > 0.0)
    return grads


# ---------------------------------------------------------------------------------
# network input: primitives of a canonical MHD state
# ---------------------------------------------------------------------------------

def primitives(state, shape, gamma=5.0 / 3.0):
    """8 primitive channels [8, nz, ny, nx] of a canonical state (rho, M, E, b1..3)."""
    nx, ny, nz = shape
    u = state.reshape(8, nz, ny, nx)
    rho = u[0]
    v = u[1:4] / rho
    bcc = np.stack([0.5 * (u[5] + shift(u[5], (1, 0, 0))), 0.5 * (u[6] + shift(u[6], (0, 1, 0))),
                    0.5 * (u[7] + shift(u[7], (0, 0, 1)))])
    ke = 0.5 * rho * (v ** 2).sum(axis=0)
    p = (gamma - 1.0) * (u[4] - ke - 0.5 * (bcc ** 2).sum(axis=0))
    return np.concatenate([rho[None], v, p[None], bcc])


def normalised_input(state, shape, mu, sd, gamma=5.0 / 3.0):
    w = primitives(state, shape, gamma)
    return (w - np.asarray(mu)[:, None, None, None]) / np.asarray(sd)[:, None, None, None]


# ---------------------------------------------------------------------------------
# closure in flux and constrained-transport form, loss and its gradient
# ---------------------------------------------------------------------------------

def corrections(out, sF, sE):
    """dF[f, d] (5 x 3 face fields) and dE[a] (3 edge fields) from the 18 channels."""
    dF = np.stack([[sF[f] * out[3 * f + d] for d in range(3)] for f in range(5)])
    dE = np.stack([sE * out[15 + a] for a in range(3)])
    return dF, dE


E = ((1, 0, 0), (0, 1, 0), (0, 0, 1))  # unit offsets e_x, e_y, e_z as (dx, dy, dz)


def apply_closure(state, shape, out, sF, sE, dt, dx):
    """The corrected state: cell fields by the divergence of dF, faces by -curl dE."""
    nx, ny, nz = shape
    u = state.reshape(8, nz, ny, nx).copy()
    dF, dE = corrections(out, sF, sE)
    for f in range(5):
        for d in range(3):
            u[f] -= dt * (shift(dF[f, d], E[d]) - dF[f, d]) / dx[d]
    Ex, Ey, Ez = dE
    u[5] -= dt * ((shift(Ez, E[1]) - Ez) / dx[1] - (shift(Ey, E[2]) - Ey) / dx[2])
    u[6] -= dt * ((shift(Ex, E[2]) - Ex) / dx[2] - (shift(Ez, E[0]) - Ez) / dx[0])
    u[7] -= dt * ((shift(Ey, E[0]) - Ey) / dx[0] - (shift(Ex, E[1]) - Ex) / dx[1])
    return u.reshape(-1)


def loss(pred, target, shape, wU, wB):
    nx, ny, nz = shape
    n = nx * ny * nz
    r = (pred - target).reshape(8, n)
    w = np.concatenate([np.asarray(wU, dtype=np.float64), [wB] * 3])
    return float((w[:, None] * r ** 2).sum() / n)


def loss_grad_out(pred, target, shape, sF, sE, dt, dx, wU, wB):
    """d(loss)/d(out) for the 18 channels, through the adjoints of apply_closure."""
    nx, ny, nz = shape
    n = nx * ny * nz
    w = np.concatenate([np.asarray(wU, dtype=np.float64), [wB] * 3])
    g = 2.0 * w[:, None, None, None] * (pred - target).reshape(8, nz, ny, nx) / n  # dL/dpred
    out = np.zeros((18, nz, ny, nx))
    # u_f[c] -= dt (dF[c + e_d] - dF[c]) / dx_d : dF[c] enters u_f[c] with +dt/dx_d and
    # u_f[c - e_d] with -dt/dx_d
    for f in range(5):
        for d in range(3):
            back = tuple(-o for o in E[d])
            out[3 * f + d] = sF[f] * dt / dx[d] * (g[f] - shift(g[f], back))
    gx, gy, gz = g[5], g[6], g[7]
    m = lambda a, d: shift(a, tuple(-o for o in E[d]))  # a[c - e_d]
    # b_y -= dt (Ex[c+e_z] - Ex[c]) / dz, b_z += dt (Ex[c+e_y] - Ex[c]) / dy
    out[15] = sE * (dt / dx[2] * (gy - m(gy, 2)) - dt / dx[1] * (gz - m(gz, 1)))
    # b_z -= dt (Ey[c+e_x] - Ey[c]) / dx, b_x += dt (Ey[c+e_z] - Ey[c]) / dz
    out[16] = sE * (dt / dx[0] * (gz - m(gz, 0)) - dt / dx[2] * (gx - m(gx, 2)))
    # b_x -= dt (Ez[c+e_y] - Ez[c]) / dy, b_y += dt (Ez[c+e_x] - Ez[c]) / dx
    out[17] = sE * (dt / dx[1] * (gx - m(gx, 1)) - dt / dx[0] * (gy - m(gy, 0)))
    return out


# ---------------------------------------------------------------------------------
# box filter of a fine state onto a coarse grid
# ---------------------------------------------------------------------------------

def box_filter(state, fine_shape, r):
    """Cell fields: mean over r^3 fine cells; face fields: mean over the r^2 fine faces
    that tile each coarse face (so the coarse discrete div B is the mean of the fine
    one)."""
    nx, ny, nz = fine_shape
    u = state.reshape(8, nz, ny, nx)
    cx, cy, cz = nx // r, ny // r, nz // r
    out = np.empty((8, cz, cy, cx))
    for f in range(5):
        out[f] = u[f].reshape(cz, r, cy, r, cx, r).mean(axis=(1, 3, 5))
    out[5] = u[5][:, :, ::r].reshape(cz, r, cy, r, cx).mean(axis=(1, 3))
    out[6] = u[6][:, ::r, :].reshape(cz, r, cy, cx, r).mean(axis=(1, 4))
    out[7] = u[7][::r, :, :].reshape(cz, cy, r, cx, r).mean(axis=(2, 4))
    return out.reshape(-1)
