"""Thin ctypes binding of the C ABI in include/mhd950.h.

The module-level functions carry the C names and only marshal arguments; every step
of the update runs in the HIP kernels of libmhd950.so.  PyTorch provides the device
workspace and the stream.  There is no fallback: if the library is missing or the
device is unavailable, the calls raise.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmhd950.so")
MAX_DUST = 16

EOS = {"adiabatic_mhd": 0, "isothermal_hydro": 1}
RECON = {"dc": 0, "plm": 1, "ppm": 2}
RIEMANN = {"hlle": 0, "hlld": 1}
INTEG = {"vl2": 0, "rk2": 1, "imex2p": 2, "euler1": 3}
PREC = {"fp64": 0, "fp32_bulk": 1}

STATUS = {0: "MHD_OK", -1: "MHD_E_INVAL", -2: "MHD_E_UNSUPPORTED", -3: "MHD_E_NOMEM",
          -4: "MHD_E_DEVICE", -5: "MHD_E_NONFINITE", -6: "MHD_E_TOOBIG"}
NOALLOC_MAX_CELLS = 1 << 27


class MhdError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {STATUS.get(code, code)} ({_strerror(code)})")


class MhdGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("length", ctypes.c_double * 3)]


class MhdPhysics(ctypes.Structure):
    _fields_ = [("eos", ctypes.c_int), ("gamma", ctypes.c_double), ("cs_iso", ctypes.c_double),
                ("rho_floor", ctypes.c_double), ("p_floor", ctypes.c_double),
                ("ndust", ctypes.c_int), ("t_stop", ctypes.c_double * MAX_DUST),
                ("dust_rho_floor", ctypes.c_double), ("gas_accel", ctypes.c_double * 3)]


class MhdScheme(ctypes.Structure):
    _fields_ = [("recon", ctypes.c_int), ("riemann", ctypes.c_int), ("integ", ctypes.c_int),
                ("courant", ctypes.c_double), ("prec", ctypes.c_int), ("hlld_eps", ctypes.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libmhd950.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run __graft_entry__.build() or python paper_2608_14048_amd/build.py)")
    L = ctypes.CDLL(path)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    dp = ctypes.POINTER(ctypes.c_double)
    L.mhd_workspace_bytes.argtypes = [ctypes.POINTER(MhdGrid), ctypes.POINTER(MhdPhysics),
                                      ctypes.POINTER(MhdScheme), ctypes.POINTER(sz)]
    L.mhd_create.argtypes = [ctypes.POINTER(MhdGrid), ctypes.POINTER(MhdPhysics),
                             ctypes.POINTER(MhdScheme), vp, sz, vp, ctypes.POINTER(vp)]
    L.mhd_state_len.argtypes = [vp, ctypes.POINTER(sz)]
    L.mhd_set_state.argtypes = [vp, vp, ctypes.c_int]
    L.mhd_get_state.argtypes = [vp, vp, ctypes.c_int]
    L.mhd_step.argtypes = [vp, ctypes.c_double]
    L.mhd_dt_cfl.argtypes = [vp, dp]
    L.mhd_dt_cfl_noalloc.argtypes = [ctypes.POINTER(MhdGrid), ctypes.POINTER(MhdPhysics),
                                     ctypes.POINTER(MhdScheme), vp, vp, vp]
    L.mhd_diagnostics.argtypes = [vp, dp, ctypes.c_int]
    L.mhd_destroy.argtypes = [vp]
    L.mhd_destroy.restype = None
    L.mhd_strerror.argtypes = [ctypes.c_int]
    L.mhd_strerror.restype = ctypes.c_char_p
    L.mhd_timing_enable.argtypes = [vp, ctypes.c_int]
    L.mhd_timing_read.argtypes = [vp, dp, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
    L.mhd_timing_name.argtypes = [ctypes.c_int]
    L.mhd_timing_name.restype = ctypes.c_char_p
    ip = ctypes.POINTER(ctypes.c_int)
    L.mhd_batch_workspace_bytes.argtypes = [ctypes.c_int, ctypes.POINTER(MhdGrid), ctypes.POINTER(MhdPhysics),
                                            ctypes.POINTER(MhdScheme), ctypes.POINTER(sz)]
    L.mhd_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(MhdGrid), ctypes.POINTER(MhdPhysics),
                                   ctypes.POINTER(MhdScheme), vp, sz, vp, ctypes.POINTER(vp)]
    L.mhd_batch_state_len.argtypes = [vp, ctypes.POINTER(sz)]
    L.mhd_batch_set_state.argtypes = [vp, vp, ctypes.c_int]
    L.mhd_batch_get_state.argtypes = [vp, vp, ctypes.c_int]
    L.mhd_batch_step.argtypes = [vp, dp]
    L.mhd_batch_dt_cfl.argtypes = [vp, dp]
    L.mhd_batch_set_shapes.argtypes = [vp, ip, ctypes.c_int]
    L.mhd_batch_get_shapes.argtypes = [vp, ip, ctypes.c_int]
    L.mhd_batch_tune.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_float), ctypes.c_int]
    L.mhd_batch_couple.argtypes = [vp, ip, ctypes.c_int, dp]
    L.mhd_batch_set_domain_state.argtypes = [vp, vp, ctypes.c_int]
    L.mhd_batch_get_domain_state.argtypes = [vp, vp, ctypes.c_int]
    L.mhd_batch_destroy.argtypes = [vp]
    L.mhd_batch_destroy.restype = None
    fp = ctypes.POINTER(ctypes.c_float)
    L.mhd_cnn_param_count.argtypes = [ctypes.POINTER(sz)]
    L.mhd_cnn_workspace_bytes.argtypes = [ctypes.POINTER(MhdGrid), ctypes.POINTER(MhdPhysics), ctypes.POINTER(sz)]
    L.mhd_cnn_create.argtypes = [ctypes.POINTER(MhdGrid), ctypes.POINTER(MhdPhysics), vp, sz, vp, ctypes.POINTER(vp)]
    L.mhd_cnn_set_params.argtypes = [vp, fp]
    L.mhd_cnn_get_params.argtypes = [vp, fp]
    L.mhd_cnn_get_grads.argtypes = [vp, fp]
    L.mhd_cnn_set_scales.argtypes = [vp, fp, fp, fp, ctypes.c_float, fp, ctypes.c_float]
    L.mhd_cnn_forward.argtypes = [vp, vp]
    L.mhd_cnn_output.argtypes = [vp, vp, ctypes.c_int]
    L.mhd_closure_apply.argtypes = [vp, ctypes.c_double, vp]
    L.mhd_cnn_zero_grad.argtypes = [vp]
    L.mhd_cnn_accumulate.argtypes = [vp, vp, vp, vp, ctypes.c_double, dp]
    L.mhd_cnn_adam.argtypes = [vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int,
                               ctypes.c_float]
    L.mhd_step_closure.argtypes = [vp, vp, ctypes.c_double, ctypes.POINTER(ctypes.c_int)]
    L.mhd_box_filter.argtypes = [ctypes.POINTER(MhdGrid), ctypes.c_int, vp, vp, vp]
    L.mhd_cnn_destroy.argtypes = [vp]
    L.mhd_cnn_destroy.restype = None
    for name in ("mhd_workspace_bytes", "mhd_create", "mhd_state_len", "mhd_set_state",
                 "mhd_get_state", "mhd_step", "mhd_dt_cfl", "mhd_dt_cfl_noalloc", "mhd_diagnostics",
                 "mhd_timing_enable", "mhd_timing_read", "mhd_batch_workspace_bytes",
                 "mhd_batch_create", "mhd_batch_state_len", "mhd_batch_set_state",
                 "mhd_batch_get_state", "mhd_batch_step", "mhd_batch_dt_cfl",
                 "mhd_batch_set_shapes", "mhd_batch_get_shapes", "mhd_batch_tune",
                 "mhd_batch_couple", "mhd_batch_set_domain_state", "mhd_batch_get_domain_state",
                 "mhd_cnn_param_count", "mhd_cnn_workspace_bytes", "mhd_cnn_create", "mhd_cnn_set_params",
                 "mhd_cnn_get_params", "mhd_cnn_get_grads", "mhd_cnn_set_scales", "mhd_cnn_forward",
                 "mhd_cnn_output", "mhd_closure_apply", "mhd_cnn_zero_grad", "mhd_cnn_accumulate",
                 "mhd_cnn_adam", "mhd_step_closure", "mhd_box_filter"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _strerror(code: int) -> str:
    try:
        return load_library().mhd_strerror(code).decode()
    except Exception:  # the library itself may be what is missing
        return "?"


def _check(code: int, where: str):
    if code != 0:
        raise MhdError(code, where)


# ---------------------------------------------------------------------------------
# structures from Python values
# ---------------------------------------------------------------------------------

def make_grid(shape, length=(1.0, 1.0, 1.0)) -> MhdGrid:
    g = MhdGrid()
    g.nx, g.ny, g.nz = (int(s) for s in shape)
    for a in range(3):
        g.length[a] = float(length[a])
    return g


def make_physics(eos="adiabatic_mhd", gamma=5.0 / 3.0, cs=1.0, rho_floor=1e-12, p_floor=1e-10,
                 tstop=(), dust_rho_floor=1e-12, gacc=(0.0, 0.0, 0.0)) -> MhdPhysics:
    p = MhdPhysics()
    p.eos = EOS[eos]
    p.gamma, p.cs_iso, p.rho_floor, p.p_floor = gamma, cs, rho_floor, p_floor
    p.ndust = len(tstop)
    for k, t in enumerate(tstop):
        p.t_stop[k] = float(t)
    p.dust_rho_floor = dust_rho_floor
    for a in range(3):
        p.gas_accel[a] = float(gacc[a])
    return p


def make_scheme(recon="plm", riemann="hlld", integ="vl2", courant=0.3, prec="fp64",
                hlld_eps=1e-12) -> MhdScheme:
    s = MhdScheme()
    s.recon, s.riemann, s.integ = RECON[recon], RIEMANN[riemann], INTEG[integ]
    s.courant, s.prec, s.hlld_eps = courant, PREC[prec], hlld_eps
    return s


# ---------------------------------------------------------------------------------
# the C calls under their own names
# ---------------------------------------------------------------------------------

def mhd_workspace_bytes(grid: MhdGrid, phys: MhdPhysics, scheme: MhdScheme) -> int:
    n = ctypes.c_size_t(0)
    _check(load_library().mhd_workspace_bytes(ctypes.byref(grid), ctypes.byref(phys),
                                              ctypes.byref(scheme), ctypes.byref(n)),
           "mhd_workspace_bytes")
    return n.value


def mhd_create(grid, phys, scheme, workspace_ptr: int, nbytes: int, stream_ptr: int) -> int:
    out = ctypes.c_void_p(0)
    _check(load_library().mhd_create(ctypes.byref(grid), ctypes.byref(phys), ctypes.byref(scheme),
                                     ctypes.c_void_p(workspace_ptr), ctypes.c_size_t(nbytes),
                                     ctypes.c_void_p(stream_ptr), ctypes.byref(out)), "mhd_create")
    return out.value


def mhd_state_len(ctx: int) -> int:
    n = ctypes.c_size_t(0)
    _check(load_library().mhd_state_len(ctypes.c_void_p(ctx), ctypes.byref(n)), "mhd_state_len")
    return n.value


def mhd_set_state(ctx: int, ptr: int, is_device: bool):
    _check(load_library().mhd_set_state(ctypes.c_void_p(ctx), ctypes.c_void_p(ptr), int(is_device)),
           "mhd_set_state")


def mhd_get_state(ctx: int, ptr: int, is_device: bool):
    _check(load_library().mhd_get_state(ctypes.c_void_p(ctx), ctypes.c_void_p(ptr), int(is_device)),
           "mhd_get_state")


def mhd_step(ctx: int, dt: float):
    _check(load_library().mhd_step(ctypes.c_void_p(ctx), ctypes.c_double(dt)), "mhd_step")


def mhd_dt_cfl(ctx: int) -> float:
    out = ctypes.c_double(0.0)
    _check(load_library().mhd_dt_cfl(ctypes.c_void_p(ctx), ctypes.byref(out)), "mhd_dt_cfl")
    return out.value


def mhd_dt_cfl_noalloc(grid: MhdGrid, phys: MhdPhysics, scheme: MhdScheme, state_ptr: int,
                       dt_ptr: int, stream: int) -> None:
    """Asynchronous CFL step of a device state into one device double (no workspace)."""
    _check(load_library().mhd_dt_cfl_noalloc(ctypes.byref(grid), ctypes.byref(phys), ctypes.byref(scheme),
                                             ctypes.c_void_p(state_ptr), ctypes.c_void_p(dt_ptr),
                                             ctypes.c_void_p(stream)), "mhd_dt_cfl_noalloc")


def mhd_diagnostics(ctx: int, n: int) -> np.ndarray:
    out = np.zeros(n)
    _check(load_library().mhd_diagnostics(ctypes.c_void_p(ctx),
                                          out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), n),
           "mhd_diagnostics")
    return out


def mhd_destroy(ctx: int):
    if ctx:
        load_library().mhd_destroy(ctypes.c_void_p(ctx))


def mhd_strerror(code: int) -> str:
    return load_library().mhd_strerror(code).decode()


def mhd_timing_name(q: int):
    r = load_library().mhd_timing_name(q)
    return None if r is None else r.decode()


def mhd_timing_enable(ctx: int, capacity: int):
    _check(load_library().mhd_timing_enable(ctypes.c_void_p(ctx), int(capacity)), "mhd_timing_enable")


def mhd_timing_read(ctx: int) -> dict:
    """{kernel class: (summed ms, launches)} since the previous read."""
    names = []
    while mhd_timing_name(len(names)) is not None:
        names.append(mhd_timing_name(len(names)))
    ms = np.zeros(len(names))
    cnt = (ctypes.c_int * len(names))()
    _check(load_library().mhd_timing_read(ctypes.c_void_p(ctx),
                                          ms.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                          cnt, len(names)), "mhd_timing_read")
    return {names[q]: (float(ms[q]), int(cnt[q])) for q in range(len(names)) if cnt[q] > 0}


def _grids(shapes, lengths):
    arr = (MhdGrid * len(shapes))()
    for b, sh in enumerate(shapes):
        arr[b] = make_grid(sh, lengths[b])
    return arr


def mhd_batch_workspace_bytes(grids, phys: MhdPhysics, scheme: MhdScheme) -> int:
    n = ctypes.c_size_t(0)
    _check(load_library().mhd_batch_workspace_bytes(len(grids), grids, ctypes.byref(phys),
                                                    ctypes.byref(scheme), ctypes.byref(n)),
           "mhd_batch_workspace_bytes")
    return n.value


def mhd_batch_create(grids, phys, scheme, workspace_ptr: int, nbytes: int, stream_ptr: int) -> int:
    out = ctypes.c_void_p(0)
    _check(load_library().mhd_batch_create(len(grids), grids, ctypes.byref(phys), ctypes.byref(scheme),
                                           ctypes.c_void_p(workspace_ptr), ctypes.c_size_t(nbytes),
                                           ctypes.c_void_p(stream_ptr), ctypes.byref(out)),
           "mhd_batch_create")
    return out.value


def mhd_batch_state_len(b: int) -> int:
    n = ctypes.c_size_t(0)
    _check(load_library().mhd_batch_state_len(ctypes.c_void_p(b), ctypes.byref(n)), "mhd_batch_state_len")
    return n.value


def mhd_batch_set_state(b: int, ptr: int, is_device: bool):
    _check(load_library().mhd_batch_set_state(ctypes.c_void_p(b), ctypes.c_void_p(ptr), int(is_device)),
           "mhd_batch_set_state")


def mhd_batch_get_state(b: int, ptr: int, is_device: bool):
    _check(load_library().mhd_batch_get_state(ctypes.c_void_p(b), ctypes.c_void_p(ptr), int(is_device)),
           "mhd_batch_get_state")


def mhd_batch_step(b: int, dts=None):
    """dts: nblocks time steps, or None for each block's own CFL step (device-resident)."""
    if dts is None:
        _check(load_library().mhd_batch_step(ctypes.c_void_p(b), None), "mhd_batch_step")
        return
    a = np.ascontiguousarray(np.asarray(dts, dtype=np.float64))
    _check(load_library().mhd_batch_step(ctypes.c_void_p(b), a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "mhd_batch_step")


def mhd_batch_dt_cfl(b: int, nblocks: int) -> np.ndarray:
    out = np.zeros(nblocks)
    _check(load_library().mhd_batch_dt_cfl(ctypes.c_void_p(b), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
           "mhd_batch_dt_cfl")
    return out


def mhd_batch_set_shapes(b: int, shapes):
    a = (ctypes.c_int * len(shapes))(*[int(v) for v in shapes])
    _check(load_library().mhd_batch_set_shapes(ctypes.c_void_p(b), a, len(shapes)), "mhd_batch_set_shapes")


def mhd_batch_get_shapes(b: int, nblocks: int):
    a = (ctypes.c_int * nblocks)()
    _check(load_library().mhd_batch_get_shapes(ctypes.c_void_p(b), a, nblocks), "mhd_batch_get_shapes")
    return list(a)


def mhd_batch_tune(b: int, reps: int, nclasses: int) -> np.ndarray:
    """Autotune; returns the measured ms per pass, [class][shape]."""
    out = (ctypes.c_float * (3 * nclasses))()
    _check(load_library().mhd_batch_tune(ctypes.c_void_p(b), int(reps), out, 3 * nclasses), "mhd_batch_tune")
    return np.array(list(out), dtype=np.float64).reshape(nclasses, 3)


def mhd_batch_couple(b: int, nblocks_xyz, ghost: int, length):
    nb = (ctypes.c_int * 3)(*[int(v) for v in nblocks_xyz])
    L = (ctypes.c_double * 3)(*[float(v) for v in length])
    _check(load_library().mhd_batch_couple(ctypes.c_void_p(b), nb, int(ghost), L), "mhd_batch_couple")


def mhd_batch_set_domain_state(b: int, ptr: int, is_device: bool):
    _check(load_library().mhd_batch_set_domain_state(ctypes.c_void_p(b), ctypes.c_void_p(ptr), int(is_device)),
           "mhd_batch_set_domain_state")


def mhd_batch_get_domain_state(b: int, ptr: int, is_device: bool):
    _check(load_library().mhd_batch_get_domain_state(ctypes.c_void_p(b), ctypes.c_void_p(ptr), int(is_device)),
           "mhd_batch_get_domain_state")


def mhd_batch_destroy(b: int):
    if b:
        load_library().mhd_batch_destroy(ctypes.c_void_p(b))


def _fptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def mhd_cnn_param_count() -> int:
    n = ctypes.c_size_t(0)
    _check(load_library().mhd_cnn_param_count(ctypes.byref(n)), "mhd_cnn_param_count")
    return n.value


def mhd_cnn_workspace_bytes(grid: MhdGrid, phys: MhdPhysics) -> int:
    n = ctypes.c_size_t(0)
    _check(load_library().mhd_cnn_workspace_bytes(ctypes.byref(grid), ctypes.byref(phys), ctypes.byref(n)),
           "mhd_cnn_workspace_bytes")
    return n.value


def mhd_cnn_create(grid, phys, workspace_ptr: int, nbytes: int, stream_ptr: int) -> int:
    out = ctypes.c_void_p(0)
    _check(load_library().mhd_cnn_create(ctypes.byref(grid), ctypes.byref(phys), ctypes.c_void_p(workspace_ptr),
                                         ctypes.c_size_t(nbytes), ctypes.c_void_p(stream_ptr), ctypes.byref(out)),
           "mhd_cnn_create")
    return out.value


def mhd_cnn_set_params(cnn: int, params):
    a = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
    _check(load_library().mhd_cnn_set_params(ctypes.c_void_p(cnn), _fptr(a)), "mhd_cnn_set_params")


def mhd_cnn_get_params(cnn: int) -> np.ndarray:
    a = np.zeros(mhd_cnn_param_count(), dtype=np.float32)
    _check(load_library().mhd_cnn_get_params(ctypes.c_void_p(cnn), _fptr(a)), "mhd_cnn_get_params")
    return a


def mhd_cnn_get_grads(cnn: int) -> np.ndarray:
    a = np.zeros(mhd_cnn_param_count(), dtype=np.float32)
    _check(load_library().mhd_cnn_get_grads(ctypes.c_void_p(cnn), _fptr(a)), "mhd_cnn_get_grads")
    return a


def mhd_cnn_set_scales(cnn: int, mu, sd, sF, sE: float, wU, wB: float):
    f = lambda v: np.ascontiguousarray(np.asarray(v, dtype=np.float32))
    mu, sd, sF, wU = f(mu), f(sd), f(sF), f(wU)
    _check(load_library().mhd_cnn_set_scales(ctypes.c_void_p(cnn), _fptr(mu), _fptr(sd), _fptr(sF), float(sE),
                                             _fptr(wU), float(wB)), "mhd_cnn_set_scales")


def mhd_cnn_forward(cnn: int, state_ptr: int):
    _check(load_library().mhd_cnn_forward(ctypes.c_void_p(cnn), ctypes.c_void_p(state_ptr)), "mhd_cnn_forward")


def mhd_cnn_output(cnn: int, ptr: int, is_device: bool):
    _check(load_library().mhd_cnn_output(ctypes.c_void_p(cnn), ctypes.c_void_p(ptr), int(is_device)),
           "mhd_cnn_output")


def mhd_closure_apply(cnn: int, dt: float, state_ptr: int):
    _check(load_library().mhd_closure_apply(ctypes.c_void_p(cnn), ctypes.c_double(dt), ctypes.c_void_p(state_ptr)),
           "mhd_closure_apply")


def mhd_cnn_zero_grad(cnn: int):
    _check(load_library().mhd_cnn_zero_grad(ctypes.c_void_p(cnn)), "mhd_cnn_zero_grad")


def mhd_cnn_accumulate(cnn: int, state_ptr: int, coarse_ptr: int, target_ptr: int, dt: float) -> float:
    loss = ctypes.c_double(0.0)
    _check(load_library().mhd_cnn_accumulate(ctypes.c_void_p(cnn), ctypes.c_void_p(state_ptr),
                                             ctypes.c_void_p(coarse_ptr), ctypes.c_void_p(target_ptr),
                                             ctypes.c_double(dt), ctypes.byref(loss)), "mhd_cnn_accumulate")
    return loss.value


def mhd_cnn_adam(cnn: int, lr: float, beta1: float, beta2: float, eps: float, step: int, grad_scale: float):
    _check(load_library().mhd_cnn_adam(ctypes.c_void_p(cnn), float(lr), float(beta1), float(beta2), float(eps),
                                       int(step), float(grad_scale)), "mhd_cnn_adam")


def mhd_step_closure(ctx: int, cnn: int, dt: float, report: bool = False):
    """One closure step; with report, returns whether the corrections were applied (1)
    or the plain step was kept (0) (reading it synchronises)."""
    flag = ctypes.c_int(-1)
    _check(load_library().mhd_step_closure(ctypes.c_void_p(ctx), ctypes.c_void_p(cnn), ctypes.c_double(dt),
                                           ctypes.byref(flag) if report else None),
           "mhd_step_closure")
    return flag.value if report else None


def mhd_box_filter(fine_grid: MhdGrid, r: int, fine_ptr: int, coarse_ptr: int, stream_ptr: int):
    _check(load_library().mhd_box_filter(ctypes.byref(fine_grid), int(r), ctypes.c_void_p(fine_ptr),
                                         ctypes.c_void_p(coarse_ptr), ctypes.c_void_p(stream_ptr)),
           "mhd_box_filter")


def mhd_cnn_destroy(cnn: int):
    if cnn:
        load_library().mhd_cnn_destroy(ctypes.c_void_p(cnn))


# ---------------------------------------------------------------------------------
# convenience object: Mesh + Simulation in one (cf. the paper's user interface)
# ---------------------------------------------------------------------------------

class Sim:
    """A context on one device with its torch-owned workspace and stream.

    Sim((nx, ny, nz), length, physics=dict(...), scheme=dict(...)) then set_state,
    step / run, state, dt_cfl, diagnostics."""

    def __init__(self, shape, length=(1.0, 1.0, 1.0), physics=None, scheme=None,
                 device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the MI355X path has no CPU fallback")
        load_library()
        self.device = torch.device(device)
        self.grid = make_grid(shape, length)
        self.phys = make_physics(**(physics or {}))
        self.scheme = make_scheme(**(scheme or {}))
        self.shape = tuple(int(s) for s in shape)
        self.nbytes = mhd_workspace_bytes(self.grid, self.phys, self.scheme)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = mhd_create(self.grid, self.phys, self.scheme, self.workspace.data_ptr(),
                              self.nbytes, self.stream.cuda_stream)
        self.n = mhd_state_len(self.ctx)
        self.nq = 12 + self.phys.ndust

    # state ------------------------------------------------------------------
    def set_state(self, state):
        import torch
        if isinstance(state, torch.Tensor) and state.is_cuda:
            t = state.detach().to(torch.float64).contiguous().reshape(-1)
            assert t.numel() == self.n, (t.numel(), self.n)
            mhd_set_state(self.ctx, t.data_ptr(), True)
            self._keep = t  # the device copy is ordered on the stream
        else:
            a = np.ascontiguousarray(np.asarray(state, dtype=np.float64).reshape(-1))
            assert a.size == self.n, (a.size, self.n)
            mhd_set_state(self.ctx, a.ctypes.data, False)

    def state(self, device: bool = False):
        import torch
        if device:
            out = torch.empty(self.n, dtype=torch.float64, device=self.device)
            mhd_get_state(self.ctx, out.data_ptr(), True)
            return out
        a = np.empty(self.n, dtype=np.float64)
        mhd_get_state(self.ctx, a.ctypes.data, False)
        return a

    # stepping ---------------------------------------------------------------
    def step(self, dt: float):
        mhd_step(self.ctx, float(dt))

    def dt_cfl(self) -> float:
        return mhd_dt_cfl(self.ctx)

    def run(self, nsteps: int, dts=None):
        """Advance nsteps with the device CFL step (or a given dt sequence); returns the
        list of dt taken."""
        used = []
        for k in range(nsteps):
            dt = self.dt_cfl() if dts is None else float(dts[k])
            self.step(dt)
            used.append(dt)
        return used

    def diagnostics(self) -> np.ndarray:
        return mhd_diagnostics(self.ctx, self.nq)

    def timing(self, capacity: int):
        """Record HIP events around up to `capacity` kernel launches (0 = off)."""
        mhd_timing_enable(self.ctx, capacity)

    def timing_read(self) -> dict:
        return mhd_timing_read(self.ctx)

    def close(self):
        if getattr(self, "ctx", 0):
            mhd_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent self-periodic MHD blocks of uneven sizes advanced together (one
    persistent launch per stage kernel and tile shape in use).

    Batch(shapes, lengths, physics=dict(...), scheme=dict(...)); the state is the blocks'
    canonical states concatenated in block order."""

    def __init__(self, shapes, lengths=None, physics=None, scheme=None, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the MI355X path has no CPU fallback")
        load_library()
        self.shapes = [tuple(int(v) for v in sh) for sh in shapes]
        if lengths is None:
            lengths = [tuple(v / max(sh) for v in sh) for sh in self.shapes]
        self.lengths = [tuple(float(v) for v in L) for L in lengths]
        self.nb = len(self.shapes)
        self.device = torch.device(device)
        self.grids = _grids(self.shapes, self.lengths)
        self.phys = make_physics(**(physics or {}))
        self.scheme = make_scheme(**(scheme or {}))
        self.nbytes = mhd_batch_workspace_bytes(self.grids, self.phys, self.scheme)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = mhd_batch_create(self.grids, self.phys, self.scheme, self.workspace.data_ptr(),
                                    self.nbytes, self.stream.cuda_stream)
        self.n = mhd_batch_state_len(self.ctx)
        self.classes = sorted(set(sh[0] for sh in self.shapes))

    def block_slices(self):
        """Slices of the concatenated state holding each block's canonical state."""
        out, at = [], 0
        for sh in self.shapes:
            m = 8 * sh[0] * sh[1] * sh[2]
            out.append(slice(at, at + m))
            at += m
        return out

    def set_state(self, state):
        import torch
        if isinstance(state, (list, tuple)):
            state = np.concatenate([np.asarray(s, dtype=np.float64).reshape(-1) for s in state])
        if isinstance(state, torch.Tensor) and state.is_cuda:
            t = state.detach().to(torch.float64).contiguous().reshape(-1)
            assert t.numel() == self.n, (t.numel(), self.n)
            mhd_batch_set_state(self.ctx, t.data_ptr(), True)
            self._keep = t
        else:
            a = np.ascontiguousarray(np.asarray(state, dtype=np.float64).reshape(-1))
            assert a.size == self.n, (a.size, self.n)
            mhd_batch_set_state(self.ctx, a.ctypes.data, False)

    def state(self, device: bool = False):
        import torch
        if device:
            out = torch.empty(self.n, dtype=torch.float64, device=self.device)
            mhd_batch_get_state(self.ctx, out.data_ptr(), True)
            return out
        a = np.empty(self.n, dtype=np.float64)
        mhd_batch_get_state(self.ctx, a.ctypes.data, False)
        return a

    def step(self, dts=None):
        mhd_batch_step(self.ctx, dts)

    def dt_cfl(self) -> np.ndarray:
        return mhd_batch_dt_cfl(self.ctx, self.nb)

    def set_tile_shapes(self, shapes):
        mhd_batch_set_shapes(self.ctx, shapes)

    def tile_shapes(self):
        return mhd_batch_get_shapes(self.ctx, self.nb)

    def tune(self, reps: int = 3) -> np.ndarray:
        return mhd_batch_tune(self.ctx, reps, len(self.classes))

    def close(self):
        if getattr(self, "ctx", 0):
            mhd_batch_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Domain:
    """One periodic domain of `shape` cells advanced as coupled meshblocks of `block`
    cells, each stored with `ghost` layers of ghost cells that a device exchange refills
    after every stage (a coupled Batch).  The state is the domain's canonical FP64 state;
    every block advances by the domain's one CFL step."""

    def __init__(self, shape, block, length=(1.0, 1.0, 1.0), ghost=None, physics=None, scheme=None,
                 device="cuda:0", stream=None):
        shape = tuple(int(v) for v in shape)
        block = tuple(int(v) for v in block)
        if any(s % b for s, b in zip(shape, block)):
            raise ValueError(f"block {block} does not tile the domain {shape}")
        scheme = dict(scheme or {})
        if ghost is None:
            ghost = {"dc": 2, "plm": 3, "ppm": 4}[scheme.get("recon", "plm")]
        self.shape, self.block, self.ghost = shape, block, int(ghost)
        self.nblocks_xyz = tuple(s // b for s, b in zip(shape, block))
        nb = self.nblocks_xyz[0] * self.nblocks_xyz[1] * self.nblocks_xyz[2]
        padded = tuple(b + 2 * self.ghost for b in block)
        h = tuple(float(L) / s for L, s in zip(length, shape))
        self.length = tuple(float(v) for v in length)
        # the spacing is set exactly by couple(); these lengths only have to be valid
        self.batch = Batch([padded] * nb, [tuple(p * hh for p, hh in zip(padded, h))] * nb, physics=physics,
                           scheme=scheme, device=device, stream=stream)
        mhd_batch_couple(self.batch.ctx, self.nblocks_xyz, self.ghost, self.length)
        self.n = 8 * shape[0] * shape[1] * shape[2]

    def set_state(self, state):
        import torch
        if isinstance(state, torch.Tensor) and state.is_cuda:
            t = state.detach().to(torch.float64).contiguous().reshape(-1)
            assert t.numel() == self.n, (t.numel(), self.n)
            mhd_batch_set_domain_state(self.batch.ctx, t.data_ptr(), True)
            torch.cuda.current_stream(t.device).synchronize()
        else:
            a = np.ascontiguousarray(np.asarray(state, dtype=np.float64).reshape(-1))
            assert a.size == self.n, (a.size, self.n)
            mhd_batch_set_domain_state(self.batch.ctx, a.ctypes.data, False)

    def state(self, device: bool = False):
        import torch
        if device:
            out = torch.empty(self.n, dtype=torch.float64, device=self.batch.device)
            mhd_batch_get_domain_state(self.batch.ctx, out.data_ptr(), True)
            return out
        a = np.empty(self.n, dtype=np.float64)
        mhd_batch_get_domain_state(self.batch.ctx, a.ctypes.data, False)
        return a

    def step(self, dt=None):
        """Advance by dt (every block alike) or, with None, by the domain's CFL step
        already on the device."""
        self.batch.step(None if dt is None else [float(dt)] * self.batch.nb)

    def dt_cfl(self) -> float:
        return float(self.batch.dt_cfl()[0])

    def close(self):
        self.batch.close()


class Closure:
    """The learned flux-correction network on one coarse grid (device workspace owned
    here); state arguments are device tensors of the canonical FP64 layout."""

    def __init__(self, shape, length=(1.0, 1.0, 1.0), physics=None, device="cuda:0", stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible: the MI355X path has no CPU fallback")
        load_library()
        self.shape = tuple(int(v) for v in shape)
        self.grid = make_grid(shape, length)
        self.phys = make_physics(**(physics or {}))
        self.device = torch.device(device)
        self.nbytes = mhd_cnn_workspace_bytes(self.grid, self.phys)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.ctx = mhd_cnn_create(self.grid, self.phys, self.workspace.data_ptr(), self.nbytes,
                                  self.stream.cuda_stream)
        self.nparams = mhd_cnn_param_count()
        self.step_count = 0

    def set_params(self, p):
        mhd_cnn_set_params(self.ctx, p)

    def params(self):
        return mhd_cnn_get_params(self.ctx)

    def grads(self):
        return mhd_cnn_get_grads(self.ctx)

    def set_scales(self, mu, sd, sF, sE, wU, wB):
        mhd_cnn_set_scales(self.ctx, mu, sd, sF, sE, wU, wB)

    def forward(self, state):
        import torch
        mhd_cnn_forward(self.ctx, state.data_ptr())
        n = int(np.prod(self.shape))
        out = torch.empty(18 * n, dtype=torch.float32, device=self.device)
        mhd_cnn_output(self.ctx, out.data_ptr(), True)
        return out

    def apply(self, dt, state):
        mhd_closure_apply(self.ctx, dt, state.data_ptr())

    def zero_grad(self):
        mhd_cnn_zero_grad(self.ctx)

    def accumulate(self, state_t, coarse_next, target, dt) -> float:
        return mhd_cnn_accumulate(self.ctx, state_t.data_ptr(), coarse_next.data_ptr(), target.data_ptr(), dt)

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, grad_scale=1.0):
        self.step_count += 1
        mhd_cnn_adam(self.ctx, lr, beta1, beta2, eps, self.step_count, grad_scale)

    def step(self, sim, dt, report: bool = False):
        """One closure step of a Sim on the same grid and stream; with report, returns 1
        if the corrections were applied, 0 if the plain step was kept."""
        return mhd_step_closure(sim.ctx, self.ctx, dt, report)

    def close(self):
        if getattr(self, "ctx", 0):
            mhd_cnn_destroy(self.ctx)
            self.ctx = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def box_filter(fine_shape, r, fine_state, coarse_state, stream=None):
    """Device box filter of a fine canonical state into a coarse one (torch tensors)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(fine_state.device)
    mhd_box_filter(make_grid(fine_shape), r, fine_state.data_ptr(), coarse_state.data_ptr(), st.cuda_stream)
