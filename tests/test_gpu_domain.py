"""One periodic domain advanced as coupled meshblocks (Sec. "Mesh, Coordinates, and
Boundary Conditions": identical blocks padded with ghost cells that one exchange per
stage refills from the face, edge and corner neighbours) against the same domain
advanced as one grid.

The blocks' interiors must match the single grid bit for bit after every step, with the
same CFL step: every interior cell sees the same input values (its ghost neighbours are
copies of the owners' cells) and the kernels give the same bits wherever a cell sits in
a tile.  The oracle parity of the single grid is covered elsewhere; this pins the
decomposition and the exchange."""
import numpy as np
import pytest

from paper_2608_14048_amd import inputs as I

pytestmark = pytest.mark.gpu

VL2_PPM_HLLD = dict(recon="ppm", riemann="hlld", integ="vl2", courant=0.3)
RK2_PLM_HLLE = dict(recon="plm", riemann="hlle", integ="rk2", courant=0.3)


def _pair(shape, block, scheme, seed, ghost=None):
    from paper_2608_14048_amd import Domain, Sim
    st, L = I.turbulence_block(shape, seed=seed)
    sim = Sim(shape, L, scheme=scheme)
    sim.set_state(st)
    dom = Domain(shape, block, L, ghost=ghost, scheme=scheme)
    dom.set_state(st)
    return st, sim, dom


@pytest.mark.parametrize("shape,block,scheme,steps", [
    ((32, 24, 16), (16, 8, 8), RK2_PLM_HLLE, 6),     # 2 x 3 x 2 blocks, PLM: 3 ghost layers
    ((32, 32, 32), (16, 16, 16), VL2_PPM_HLLD, 6),   # 2 x 2 x 2 blocks, PPM: 4 ghost layers
    ((48, 16, 16), (16, 16, 16), VL2_PPM_HLLD, 3),   # a row of 3 blocks (neighbours on both sides differ)
    ((16, 16, 16), (16, 16, 16), VL2_PPM_HLLD, 3),   # one block: its ghosts are its own periodic images
    ((30, 20, 12), (10, 10, 6), RK2_PLM_HLLE, 4),    # 3 x 2 x 2 blocks of odd sizes (ragged tiles everywhere)
])
def test_blocks_match_one_grid_bitwise(shape, block, scheme, steps):
    st, sim, dom = _pair(shape, block, scheme, seed=7)
    try:
        # the domain state survives the scatter into padded blocks and the gather back
        assert np.array_equal(dom.state(), np.asarray(st, dtype=np.float64).reshape(-1))
        for k in range(steps):
            dt_one, dt_blk = sim.dt_cfl(), dom.dt_cfl()
            assert dt_blk == dt_one, (k, dt_blk, dt_one)
            sim.step(dt_one)
            dom.step()  # the domain's own step, already on the device
            a, b = sim.state(), dom.state()
            if not np.array_equal(a, b):
                d = np.abs(a - b).reshape(8, -1).max(axis=1)
                raise AssertionError(f"step {k}: blocks differ from the single grid (max |diff| per field {d})")
    finally:
        dom.close()
        sim.close()


def test_host_dt_and_wider_ghosts():
    """Explicit (equal) host steps, and more ghost layers than the stencil needs, give the
    same bits as the device steps with the minimal ghost width."""
    shape, block = (32, 16, 16), (16, 16, 16)
    st, sim, dom = _pair(shape, block, RK2_PLM_HLLE, seed=3, ghost=5)
    try:
        for k in range(3):
            dt = sim.dt_cfl()
            assert dom.dt_cfl() == dt
            sim.step(dt)
            dom.step(dt)
            assert np.array_equal(sim.state(), dom.state()), k
    finally:
        dom.close()
        sim.close()


def test_coupling_errors():
    import torch

    from paper_2608_14048_amd import Batch, Domain, MhdError
    from paper_2608_14048_amd.binding import (mhd_batch_couple, mhd_batch_set_domain_state, mhd_batch_step)
    # too few ghost layers for PPM (needs 4)
    with pytest.raises(MhdError):
        Domain((32, 16, 16), (16, 16, 16), (1.0, 0.5, 0.5), ghost=3, scheme=VL2_PPM_HLLD)
    # blocks of different extents, and a block count that does not match
    b = Batch([(22, 22, 22), (22, 22, 24)], scheme=RK2_PLM_HLLE)
    try:
        with pytest.raises(MhdError):
            mhd_batch_couple(b.ctx, (2, 1, 1), 3, (1.0, 0.5, 0.5))
    finally:
        b.close()
    b = Batch([(22, 22, 22)] * 2, scheme=RK2_PLM_HLLE)
    try:
        with pytest.raises(MhdError):
            mhd_batch_couple(b.ctx, (3, 1, 1), 3, (1.0, 0.5, 0.5))
        # a domain state for a batch that is not coupled
        buf = torch.zeros(8 * 32 * 16 * 16, dtype=torch.float64, device="cuda:0")
        with pytest.raises(MhdError):
            mhd_batch_set_domain_state(b.ctx, buf.data_ptr(), True)
    finally:
        b.close()
    # FP32-bulk blocks are not coupled
    b = Batch([(22, 22, 22)] * 2, scheme=dict(RK2_PLM_HLLE, prec="fp32_bulk"))
    try:
        with pytest.raises(MhdError):
            mhd_batch_couple(b.ctx, (2, 1, 1), 3, (1.0, 0.5, 0.5))
    finally:
        b.close()
    # one domain, one step: unequal host steps are rejected
    d = Domain((32, 16, 16), (16, 16, 16), (1.0, 0.5, 0.5), scheme=RK2_PLM_HLLE)
    try:
        d.set_state(I.turbulence_block((32, 16, 16), seed=1)[0])
        with pytest.raises(MhdError):
            mhd_batch_step(d.batch.ctx, [1e-4, 2e-4])
    finally:
        d.close()
