"""Write turbulence_sensitivity.txt: how far the FP64 oracle separates from itself on the
64^3 decaying-turbulence recipe (VL2 + PPM + HLLD + CT, Courant 0.3) when its input or
its arithmetic moves by one unit in the last place.

Calls only the oracle and the seeded input generators.  For seeds 1-3 it runs
  base   100 steps from the recipe's state, with the oracle's own time steps;
  init   the same time steps from that state with every total-energy value moved by
         one ulp (alternately up and down);
  every  the same time steps, with every value of the state moved by one ulp in a
         random direction after each step (a stand-in for an implementation whose
         operations round differently in the last bit at every step);
and records, after each step, the largest per-class separation from base: max |d|
over the class divided by the class scale (max rho; max rho(|v| + c_s); max E; max |b|).

Run:  python tests/golden/make_turbulence_sensitivity.py   (about 3 minutes, 8 threads)
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2608_14048_amd import inputs as I  # noqa: E402

N, STEPS, GAMMA = 64, 100, 5.0 / 3.0
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "turbulence_sensitivity.txt")


def class_sep(a, ref):
    n = N ** 3
    g, r = a.reshape(8, n), ref.reshape(8, n)
    rho = r[0]
    bcc2 = r[5] ** 2 + r[6] ** 2 + r[7] ** 2
    ke = 0.5 * (r[1] ** 2 + r[2] ** 2 + r[3] ** 2) / rho
    p = np.maximum((GAMMA - 1) * (r[4] - ke - 0.5 * bcc2), 1e-10)
    speed = np.sqrt(r[1] ** 2 + r[2] ** 2 + r[3] ** 2) / rho + np.sqrt(GAMMA * p / rho)
    scales = [np.abs(rho).max(), (rho * speed).max(), np.abs(r[4]).max(), np.abs(r[5:8]).max()]
    rows = [[0], [1, 2, 3], [4], [5, 6, 7]]
    return max(float(np.abs(g[q] - r[q]).max() / s) for q, s in zip(rows, scales))


def ulp_nudge(a, rng):
    up = rng.random(a.size) < 0.5
    return np.where(up, np.nextafter(a, np.inf), np.nextafter(a, -np.inf))


def main():
    cfg = oracle.make_cfg((N, N, N), recon="ppm", riemann="hlld", integ="vl2", courant=0.3)
    lines = ["# oracle self-separation on decaying turbulence 64^3, VL2+PPM+HLLD+CT, C = 0.3",
             "# written by make_turbulence_sensitivity.py (oracle only); columns:",
             "# seed step init every   (max per-class separation from the unperturbed run)"]
    for seed in (1, 2, 3):
        st = I.turbulence(N, seed=seed)
        nc = N ** 3
        init = st.copy()
        e = init[4 * nc:5 * nc]
        alt = (np.arange(nc) % 2 == 0)
        init[4 * nc:5 * nc] = np.where(alt, np.nextafter(e, np.inf), np.nextafter(e, -np.inf))
        base, a, b = st.copy(), init, st.copy()
        rng = np.random.default_rng(1000 + seed)
        for k in range(1, STEPS + 1):
            dt = oracle.dt_cfl(cfg, base)
            base = oracle.step(cfg, base, dt)
            a = oracle.step(cfg, a, dt)
            b = ulp_nudge(oracle.step(cfg, b, dt), rng)
            lines.append(f"{seed} {k} {class_sep(a, base):.3e} {class_sep(b, base):.3e}")
            print(lines[-1], flush=True)
    with open(OUT, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
