"""Plain FP64 CPU oracle of the Godunov step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library in
``paper_2608_14048_amd``; the two meet only through the seeded input generators and
the canonical state layout documented in ``oracle.h``.

Every function here is a thin ctypes marshaller around ``oracle.c``, which follows the
paper's Sec. "Numerical Methods" step by step (see the header of that file).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAX_DUST = 16
EOS = {"adiabatic_mhd": 0, "isothermal_hydro": 1}
RECON = {"dc": 0, "plm": 1, "ppm": 2}
RIEMANN = {"hlle": 0, "hlld": 1}
INTEG = {"vl2": 0, "rk2": 1, "imex2p": 2, "euler1": 3}


class OrcCfg(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("eos", ctypes.c_int),
        ("gamma", ctypes.c_double), ("cs", ctypes.c_double),
        ("rho_floor", ctypes.c_double), ("p_floor", ctypes.c_double),
        ("dust_rho_floor", ctypes.c_double),
        ("ndust", ctypes.c_int),
        ("tstop", ctypes.c_double * MAX_DUST),
        ("gacc", ctypes.c_double * 3),
        ("recon", ctypes.c_int), ("riemann", ctypes.c_int), ("integ", ctypes.c_int),
        ("courant", ctypes.c_double),
        ("hlld_eps", ctypes.c_double),
    ]


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (no FMA contraction, OpenMP over k-planes)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-std=c99", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        cp = ctypes.POINTER(OrcCfg)
        L.orc_num_threads.argtypes = []; L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]; L.orc_set_num_threads.restype = None
        L.orc_state_len.argtypes = [cp]; L.orc_state_len.restype = ctypes.c_long
        L.orc_step.argtypes = [cp, dp, ctypes.c_double]; L.orc_step.restype = ctypes.c_int
        L.orc_dt_cfl.argtypes = [cp, dp]; L.orc_dt_cfl.restype = ctypes.c_double
        L.orc_diagnostics.argtypes = [cp, dp, dp]; L.orc_diagnostics.restype = ctypes.c_int
        L.orc_recon_line.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp]
        L.orc_recon_line.restype = None
        L.orc_riemann_mhd.argtypes = [cp, dp, dp, ctypes.c_double, dp]
        L.orc_riemann_mhd.restype = None
        L.orc_riemann_iso_hlle.argtypes = [ctypes.c_double, dp, dp, dp]
        L.orc_riemann_iso_hlle.restype = None
        L.orc_riemann_dust_rusanov.argtypes = [dp, dp, dp]
        L.orc_riemann_dust_rusanov.restype = None
        L.orc_drag_solve.argtypes = [ctypes.c_int, dp, dp, dp, ctypes.c_double, dp]
        L.orc_drag_solve.restype = None
        L.orc_rhs_mhd_debug.argtypes = [cp, ctypes.c_int, dp, dp, dp, dp]
        L.orc_rhs_mhd_debug.restype = None
        L.orc_mhd_prims.argtypes = [cp, dp, dp]
        L.orc_mhd_prims.restype = None
        _lib_handle = L
    return _lib_handle


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def make_cfg(shape, length=(1.0, 1.0, 1.0), eos="adiabatic_mhd", gamma=5.0 / 3.0, cs=1.0,
             rho_floor=1e-12, p_floor=1e-10, dust_rho_floor=1e-12, tstop=(), gacc=(0, 0, 0),
             recon="plm", riemann="hlld", integ="vl2", courant=0.3, hlld_eps=1e-12) -> OrcCfg:
    """Build the oracle's configuration; shape = (nx, ny, nz), length = box edges."""
    c = OrcCfg()
    c.nx, c.ny, c.nz = (int(s) for s in shape)
    c.dx, c.dy, c.dz = (float(length[a]) / shape[a] for a in range(3))
    c.eos = EOS[eos]
    c.gamma, c.cs = gamma, cs
    c.rho_floor, c.p_floor, c.dust_rho_floor = rho_floor, p_floor, dust_rho_floor
    c.ndust = len(tstop)
    for k, t in enumerate(tstop):
        c.tstop[k] = float(t)
    for a in range(3):
        c.gacc[a] = float(gacc[a])
    c.recon, c.riemann, c.integ = RECON[recon], RIEMANN[riemann], INTEG[integ]
    c.courant, c.hlld_eps = courant, hlld_eps
    return c


def num_threads() -> int:
    return int(_lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (results do not depend on it)."""
    _lib().orc_set_num_threads(int(n))


def state_len(cfg: OrcCfg) -> int:
    return int(_lib().orc_state_len(ctypes.byref(cfg)))


def step(cfg: OrcCfg, state: np.ndarray, dt: float) -> np.ndarray:
    """Return the state advanced by one step of size dt (input untouched)."""
    out = np.ascontiguousarray(state, dtype=np.float64).copy()
    assert out.size == state_len(cfg)
    rc = _lib().orc_step(ctypes.byref(cfg), _ptr(out), float(dt))
    if rc != 0:
        raise ValueError("oracle does not implement this configuration")
    return out


def dt_cfl(cfg: OrcCfg, state: np.ndarray) -> float:
    s = np.ascontiguousarray(state, dtype=np.float64)
    return float(_lib().orc_dt_cfl(ctypes.byref(cfg), _ptr(s)))


def diagnostics(cfg: OrcCfg, state: np.ndarray) -> np.ndarray:
    s = np.ascontiguousarray(state, dtype=np.float64)
    out = np.zeros(9 + cfg.ndust + 3)
    n = _lib().orc_diagnostics(ctypes.byref(cfg), _ptr(s), _ptr(out))
    return out[:n]


def run(cfg: OrcCfg, state: np.ndarray, nsteps: int, dts=None):
    """Advance nsteps with the oracle's own CFL step (or the given dt sequence).
    Returns (state, list of dt used)."""
    s = np.ascontiguousarray(state, dtype=np.float64).copy()
    used = []
    for n in range(nsteps):
        dt = dt_cfl(cfg, s) if dts is None else float(dts[n])
        s = step(cfg, s, dt)
        used.append(dt)
    return s, used


def recon_line(recon: str, a: np.ndarray):
    a = np.ascontiguousarray(a, dtype=np.float64)
    aL = np.zeros_like(a)
    aR = np.zeros_like(a)
    _lib().orc_recon_line(RECON[recon], a.size, _ptr(a), _ptr(aL), _ptr(aR))
    return aL, aR


def riemann_mhd(cfg: OrcCfg, wl, wr, bn: float) -> np.ndarray:
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    f = np.zeros(7)
    _lib().orc_riemann_mhd(ctypes.byref(cfg), _ptr(wl), _ptr(wr), float(bn), _ptr(f))
    return f


def riemann_iso_hlle(cs: float, wl, wr) -> np.ndarray:
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    f = np.zeros(4)
    _lib().orc_riemann_iso_hlle(float(cs), _ptr(wl), _ptr(wr), _ptr(f))
    return f


def riemann_dust_rusanov(wl, wr) -> np.ndarray:
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    f = np.zeros(4)
    _lib().orc_riemann_dust_rusanov(_ptr(wl), _ptr(wr), _ptr(f))
    return f


def drag_solve(rho, p, ts, h: float) -> np.ndarray:
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    ts = np.ascontiguousarray(ts, dtype=np.float64)
    out = np.zeros_like(p)
    _lib().orc_drag_solve(len(ts), _ptr(rho), _ptr(p), _ptr(ts), float(h), _ptr(out))
    return out


def mhd_prims(cfg: OrcCfg, state: np.ndarray) -> np.ndarray:
    """The 8 cell primitives of an MHD state as a stage computes them, [8][nz][ny][nx]."""
    s = np.ascontiguousarray(state, dtype=np.float64)
    nc = cfg.nx * cfg.ny * cfg.nz
    out = np.zeros(8 * nc)
    _lib().orc_mhd_prims(ctypes.byref(cfg), _ptr(s), _ptr(out))
    return out.reshape(8, cfg.nz, cfg.ny, cfg.nx)


def rhs_mhd_debug(cfg: OrcCfg, recon: str, state: np.ndarray):
    """One stage's right-hand side with its edge and face electric fields."""
    s = np.ascontiguousarray(state, dtype=np.float64)
    nc = cfg.nx * cfg.ny * cfg.nz
    dudt = np.zeros(8 * nc)
    emf = np.zeros(3 * nc)
    facee = np.zeros(6 * nc)
    _lib().orc_rhs_mhd_debug(ctypes.byref(cfg), RECON[recon], _ptr(s), _ptr(dudt), _ptr(emf),
                             _ptr(facee))
    return dudt, emf, facee
