"""The committed trained closure (paper_2608_14048_amd/data/closure_64.npz, written by
python -m paper_2608_14048_amd.learned) on a held-out seed: the closure run stays
conservative and divergence free, and is compared with the plain coarse run against
the filtered fine run."""
import os

import numpy as np
import pytest
import torch

from paper_2608_14048_amd import binding as B
from paper_2608_14048_amd import learned as LC

pytestmark = pytest.mark.gpu

WEIGHTS = os.path.join(os.path.dirname(LC.__file__), "data", "closure_64.npz")


def test_trained_closure_on_a_held_out_seed():
    cl, meta = LC.load(WEIGHTS)
    try:
        nc, r = meta["nc"], meta["r"]
        res, times = LC.evaluate(cl, [905], nc, r, steps=4)
        last = res[0][-1]
        print(f"  after 4 steps: {last}  ms/step {times}", flush=True)
        for run in ("plain", "closure", "plain_2x"):
            assert all(np.isfinite(v) for v in last[run].values())
        # the closure must cut the plain coarse step's error in every class: on this
        # seed after 4 steps the measured ratios closure / plain are rho 0.889, M 0.909,
        # E 0.682, B 0.944 (seeds 904-906 after 8 steps: 0.886-0.896, 0.910-0.918,
        # 0.713-0.722, 0.949-0.953); the bounds leave about 4 points for rounding-level
        # changes, not for a closure that stops working
        bounds = {"rho": 0.93, "M": 0.95, "E": 0.78, "B": 0.98}
        for k, bnd in bounds.items():
            ratio = last["closure"][k] / last["plain"][k]
            assert ratio <= bnd, (k, ratio, bnd)
        # conservation and div B of a closure step
        f = LC.FineToCoarse(905, nc, r)
        st = f.filtered()
        f.close()
        sim = B.Sim((nc,) * 3, scheme=LC.SCHEME)
        sim.set_state(st)
        d0 = sim.diagnostics()
        cl.step(sim, sim.dt_cfl())
        d1 = sim.diagnostics()
        sim.close()
        print(f"  mass {d0[0]:.15e} -> {d1[0]:.15e}, energy {d0[4]:.15e} -> {d1[4]:.15e}, max|divB| {d1[8]:.2e}", flush=True)
        assert abs(d1[0] - d0[0]) <= 1e-13 * abs(d0[0])
        assert np.all(np.abs(d1[1:4] - d0[1:4]) <= 1e-13 * abs(d0[0]))
        assert abs(d1[4] - d0[4]) <= 1e-13 * abs(d0[4])
        assert d1[8] <= 1e-10 * np.abs(st[5 * nc ** 3:].cpu().numpy()).max() * nc
    finally:
        cl.close()
