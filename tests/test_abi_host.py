"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
function the header declares, and rejects bad configurations before any launch."""
import ctypes
import os
import re

import pytest

from paper_2608_14048_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mhd950.h")

pytestmark = pytest.mark.skipif(not os.path.exists(B.LIB_PATH),
                                reason="libmhd950.so not built (run __graft_entry__.build())")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mhd_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(B.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name


def _ws(shape=(8, 8, 8), **kw):
    phys = {k: kw.pop(k) for k in list(kw) if k in ("eos", "tstop", "cs", "gamma", "gacc")}
    return B.make_grid(shape), B.make_physics(**phys), B.make_scheme(**kw)


def test_workspace_and_validation():
    g, p, s = _ws()
    nb = B.mhd_workspace_bytes(g, p, s)
    assert nb >= 2 * 8 * 512 * 8  # two FP64 registers of 8 fields at least
    # bigger grid, bigger workspace; the FP32-bulk form needs less
    g2, p2, s2 = _ws((16, 8, 8))
    assert B.mhd_workspace_bytes(g2, p2, s2) > nb
    assert B.mhd_workspace_bytes(*_ws(prec="fp32_bulk")) < nb
    # the FP32 dust form: two FP32 registers plus an FP64 staging state of 4(1+N) fields
    dust = dict(eos="isothermal_hydro", tstop=(1.0, 0.1), integ="imex2p", riemann="hlle")
    nd64 = B.mhd_workspace_bytes(*_ws(**dust))
    nd32 = B.mhd_workspace_bytes(*_ws(prec="fp32_bulk", **dust))
    assert nd64 >= 2 * 12 * 512 * 8
    assert nd32 >= 2 * 12 * 512 * 4 + 12 * 512 * 8
    bad = [
        dict(shape=(0, 8, 8)),
        dict(courant=0.0),
        dict(courant=float("nan")),
    ]
    for kw in bad:
        with pytest.raises(B.MhdError) as e:
            B.mhd_workspace_bytes(*_ws(**kw))
        assert e.value.code == -1
    unsupported = [
        dict(integ="imex2p"),                                    # IMEX2P without dust
        dict(eos="isothermal_hydro", tstop=(1.0,), integ="vl2"),  # dust needs IMEX2P
        dict(eos="isothermal_hydro", tstop=(1.0,), integ="imex2p", riemann="hlld"),
        dict(eos="isothermal_hydro", tstop=(1.0,), integ="imex2p", riemann="hlle", recon="ppm"),
        dict(eos="isothermal_hydro", tstop=(), integ="imex2p", riemann="hlle"),
        dict(eos="isothermal_hydro", tstop=(1.0,) * 17, integ="imex2p", riemann="hlle"),
        dict(shape=(1024, 1024, 512)),                            # 2^29 cells: beyond 32-bit offsets
    ]
    for kw in unsupported:
        shape = kw.pop("shape", (8, 8, 8))
        if len(kw.get("tstop", ())) > 16:
            # more species than the ABI holds is refused by the Python marshaller first
            with pytest.raises(IndexError):
                _ws(shape, **kw)
            continue
        with pytest.raises(B.MhdError) as e:
            B.mhd_workspace_bytes(*_ws(shape, **kw))
        assert e.value.code == -2, kw


def test_create_checks_workspace_before_touching_the_device():
    g, p, s = _ws()
    nb = B.mhd_workspace_bytes(g, p, s)
    fake = 1 << 40  # never dereferenced: create only carves pointers
    with pytest.raises(B.MhdError) as e:
        B.mhd_create(g, p, s, fake, nb - 256, 0)
    assert e.value.code == -3
    with pytest.raises(B.MhdError) as e:
        B.mhd_create(g, p, s, fake + 8, nb, 0)  # misaligned
    assert e.value.code == -1
    ctx = B.mhd_create(g, p, s, fake, nb, 0)
    try:
        assert B.mhd_state_len(ctx) == 8 * 512
        for bad_dt in (0.0, -1.0, float("nan"), float("inf")):
            with pytest.raises(B.MhdError) as e:
                B.mhd_step(ctx, bad_dt)
            assert e.value.code == -1
    finally:
        B.mhd_destroy(ctx)
    assert B.mhd_strerror(-5) == "state holds NaN or Inf"


def test_batch_validation_before_touching_the_device():
    shapes = [(16, 24, 32), (64, 16, 16)]
    grids = B._grids(shapes, [(1.0, 1.0, 1.0)] * 2)
    phys, scheme = B.make_physics(), B.make_scheme(recon="ppm")
    nb = B.mhd_batch_workspace_bytes(grids, phys, scheme)
    cells = sum(a * b * c for a, b, c in shapes)
    assert nb >= 3 * 8 * 8 * cells  # three FP64 registers at least
    assert B.mhd_batch_workspace_bytes(grids, phys, B.make_scheme(recon="ppm", prec="fp32_bulk")) < nb
    with pytest.raises(B.MhdError) as e:  # dust batches do not exist
        B.mhd_batch_workspace_bytes(grids, B.make_physics(eos="isothermal_hydro", tstop=(1.0,)),
                                    B.make_scheme(riemann="hlle", integ="imex2p"))
    assert e.value.code == -2
    with pytest.raises(B.MhdError) as e:
        B.mhd_batch_workspace_bytes(B._grids([(0, 4, 4)], [(1.0, 1.0, 1.0)]), phys, scheme)
    assert e.value.code == -1
    big = B._grids([(1024, 1024, 256), (1024, 1024, 256)], [(1.0, 1.0, 1.0)] * 2)
    with pytest.raises(B.MhdError) as e:  # 2^29 cells in total: beyond 32-bit offsets
        B.mhd_batch_workspace_bytes(big, phys, scheme)
    assert e.value.code == -2
    fake = 1 << 40  # never dereferenced: create rejects before any device call
    with pytest.raises(B.MhdError) as e:
        B.mhd_batch_create(grids, phys, scheme, fake, nb - 256, 0)
    assert e.value.code == -3
    with pytest.raises(B.MhdError) as e:
        B.mhd_batch_create(grids, phys, scheme, fake + 8, nb, 0)
    assert e.value.code == -1


def test_closure_validation_before_touching_the_device():
    from oracle import closure as OC
    # the parameter layout the library takes is the reference's
    assert B.mhd_cnn_param_count() == OC.param_count() == 77874
    phys = B.make_physics()
    nb = B.mhd_cnn_workspace_bytes(B.make_grid((64, 64, 64)), phys)
    # parameters, gradients and two Adam moments in FP32 at least
    assert nb >= 4 * 4 * 77874
    assert B.mhd_cnn_workspace_bytes(B.make_grid((64, 32, 16)), phys) < nb
    cases = [
        (B.make_grid((24, 16, 16)), phys, -2),                         # x not a multiple of 16
        (B.make_grid((8, 16, 16)), phys, -1),                          # narrower than one MFMA block
        (B.make_grid((512, 512, 256)), phys, -2),                      # 2^26 cells
        (B.make_grid((64, 64, 64)), B.make_physics(eos="isothermal_hydro", tstop=(1.0,)), -2),
        (B.make_grid((64, 64, 64)), B.make_physics(gamma=1.0), -2),
    ]
    for grid, ph, code in cases:
        with pytest.raises(B.MhdError) as e:
            B.mhd_cnn_workspace_bytes(grid, ph)
        assert e.value.code == code
    fake = 1 << 40  # never dereferenced: create rejects before any device call
    g64 = B.make_grid((64, 64, 64))
    with pytest.raises(B.MhdError) as e:
        B.mhd_cnn_create(g64, phys, fake, nb - 256, 0)
    assert e.value.code == -3
    with pytest.raises(B.MhdError) as e:
        B.mhd_cnn_create(g64, phys, fake + 8, nb, 0)
    assert e.value.code == -1


def test_noalloc_entry_point_rejects_before_any_launch():
    """mhd_dt_cfl_noalloc validates like mhd_create and refuses grids beyond its static
    scratch before touching the device (the pointers here are never dereferenced)."""
    lib = B.load_library()
    fake = ctypes.c_void_p(0x1000)
    g, p, s = _ws()
    assert lib.mhd_dt_cfl_noalloc(ctypes.byref(g), ctypes.byref(p), ctypes.byref(s), None, fake, None) == -1
    assert lib.mhd_dt_cfl_noalloc(ctypes.byref(g), ctypes.byref(p), ctypes.byref(s), fake, None, None) == -1
    g0, p0, s0 = _ws((0, 8, 8))
    assert lib.mhd_dt_cfl_noalloc(ctypes.byref(g0), ctypes.byref(p0), ctypes.byref(s0), fake, fake, None) == -1
    gd, pd, sd = _ws(eos="isothermal_hydro", tstop=(1.0,), integ="vl2", riemann="hlle")
    assert lib.mhd_dt_cfl_noalloc(ctypes.byref(gd), ctypes.byref(pd), ctypes.byref(sd), fake, fake, None) == -2
    gb, pb, sb = _ws((1024, 1024, 256))
    assert lib.mhd_dt_cfl_noalloc(ctypes.byref(gb), ctypes.byref(pb), ctypes.byref(sb), fake, fake, None) == -6
    assert B.NOALLOC_MAX_CELLS == 1 << 27
