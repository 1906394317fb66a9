"""Training and evaluation of the learned flux-correction closure (driver code only:
every state update, filter, network pass and optimiser step runs in the library's HIP
kernels through the C ABI).

Data (a-priori, from this solver itself): a fine run of the turbulence recipe at
r times the coarse resolution; at each coarse step of size dt (the coarse CFL step of
the filtered state), the sample is (filtered fine state at t, the plain coarse step of
it, filtered fine state at t + dt, dt).  The fine run advances dt in equal substeps
within its own CFL limit.  Evaluation (a-posteriori, held-out seeds): from the filtered
fine initial state, the plain coarse run, the closure run and a plain run at twice the
coarse resolution advance on the same dt sequence; each is compared with the filtered
fine state after every step (relative L1 per conserved class).

    python -m paper_2608_14048_amd.learned --out closure_64.npz      (train, on a GPU)
    python -m paper_2608_14048_amd.learned --eval-sizes paper_2608_14048_amd/data/closure_64.npz
        (the closure at 64^3 against plain runs at 72^3 and 80^3 to the same time)
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from . import binding as B
from . import inputs as I

SCHEME = dict(recon="ppm", riemann="hlld", integ="vl2", courant=0.3)
ROWS = {"rho": [0], "M": [1, 2, 3], "E": [4], "B": [5, 6, 7]}


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


def l1_rel(got, ref, n):
    g = got.reshape(8, n)
    r = ref.reshape(8, n)
    return {k: float((g[v] - r[v]).abs().sum() / r[v].abs().sum()) for k, v in ROWS.items()}


class FineToCoarse:
    """A fine run of one seed with its filtered view on the coarse grid."""

    def __init__(self, seed, nc, r):
        import torch
        self.nc, self.r, self.nf = nc, r, nc * r
        self.fine = B.Sim((self.nf,) * 3, scheme=SCHEME)
        self.fine.set_state(I.turbulence(self.nf, seed=seed))
        self.coarse_buf = torch.empty(8 * nc ** 3, dtype=torch.float64, device="cuda:0")

    def filtered(self):
        import torch
        B.box_filter((self.nf,) * 3, self.r, self.fine.state(device=True), self.coarse_buf)
        torch.cuda.synchronize()
        return self.coarse_buf.clone()

    def advance(self, dt):
        m = max(1, math.ceil(dt / (0.9 * self.fine.dt_cfl())))
        for _ in range(m):
            self.fine.step(dt / m)
        return m

    def close(self):
        self.fine.close()


def make_samples(seeds, nc=64, r=4, steps=6, warm=2):
    """Training samples (state_t, coarse_next, target, dt) on the device."""
    coarse = B.Sim((nc,) * 3, scheme=SCHEME)
    out = []
    for seed in seeds:
        t0 = time.perf_counter()
        f = FineToCoarse(seed, nc, r)
        for k in range(warm + steps):
            st = f.filtered()
            coarse.set_state(st)
            dt = coarse.dt_cfl()
            coarse.step(dt)
            nxt = coarse.state(device=True)
            f.advance(dt)
            if k >= warm:
                out.append((st, nxt, f.filtered(), dt))
        f.close()
        _say(f"[learned] seed {seed}: {len(out)} samples ({time.perf_counter() - t0:.1f} s)")
    coarse.close()
    return out


def _prims_stats(samples, nc, gamma=5.0 / 3.0):
    """Mean and spread of the 8 primitive channels over a few samples (host)."""
    acc = []
    for st, _, _, _ in samples[:: max(1, len(samples) // 8)]:
        u = st.cpu().numpy().reshape(8, nc, nc, nc)
        rho = u[0]
        v = u[1:4] / rho
        b = np.stack([0.5 * (u[5] + np.roll(u[5], -1, 2)), 0.5 * (u[6] + np.roll(u[6], -1, 1)),
                      0.5 * (u[7] + np.roll(u[7], -1, 0))])
        p = (gamma - 1.0) * (u[4] - 0.5 * rho * (v ** 2).sum(0) - 0.5 * (b ** 2).sum(0))
        acc.append(np.concatenate([rho[None], v, p[None], b]).reshape(8, -1))
    w = np.concatenate(acc, axis=1)
    return w.mean(axis=1), w.std(axis=1) + 1e-6


def residual_scales(samples, nc):
    """rms of (target - plain step) per conserved field, and the matching output scales
    (a unit output changes a cell by about that rms in one step)."""
    r2 = np.zeros(8)
    for st, nxt, tgt, dt in samples:
        d = (tgt - nxt).reshape(8, -1)
        r2 += (d * d).mean(dim=1).cpu().numpy()
    rms = np.sqrt(r2 / len(samples))
    dt_mean = float(np.mean([s[3] for s in samples]))
    h = 1.0 / nc
    sF = rms[:5] * h / dt_mean
    sE = float(rms[5:].mean() * h / dt_mean)
    return rms, sF, sE


WIDTHS = (8, 32, 32, 32, 18)


def he_init(seed, last_scale=0.1):
    """He-normal weights for the ReLU layers, a small last layer, zero biases; the
    parameter layout of the C ABI (per layer W [27][cin][cout], then b [cout])."""
    rng = np.random.default_rng(seed)
    parts = []
    for l in range(4):
        cin, cout = WIDTHS[l], WIDTHS[l + 1]
        std = math.sqrt(2.0 / (27 * cin)) * (last_scale if l == 3 else 1.0)
        parts.append((std * rng.standard_normal((27, cin, cout))).reshape(-1))
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32)


def train(samples, nc=64, iters=1500, batch=4, lr=1e-3, seed=0, log_every=100):
    """Adam on the a-priori loss; returns the network state and the loss history."""
    mu, sd = _prims_stats(samples, nc)
    rms, sF, sE = residual_scales(samples, nc)
    wU = 1.0 / rms[:5] ** 2
    wB = float(1.0 / np.mean(rms[5:] ** 2))
    cl = B.Closure((nc,) * 3)
    cl.set_scales(mu, sd, sF, sE, wU, wB)
    cl.set_params(he_init(seed))
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.perf_counter()
    for it in range(iters):
        cl.zero_grad()
        tot = 0.0
        for q in rng.choice(len(samples), batch, replace=False):
            st, nxt, tgt, dt = samples[q]
            tot += cl.accumulate(st, nxt, tgt, dt)
        cl.adam(lr * (0.1 if it > 0.8 * iters else 1.0), grad_scale=1.0 / batch)
        hist.append(tot / batch)
        if it % log_every == 0 or it == iters - 1:
            _say(f"[learned] iter {it}: loss {np.mean(hist[-log_every:]):.4f} ({time.perf_counter() - t0:.1f} s)")
    meta = {"mu": mu.tolist(), "sd": sd.tolist(), "sF": sF.tolist(), "sE": sE, "wU": wU.tolist(), "wB": wB,
            "residual_rms": rms.tolist()}
    return cl, meta, hist


def zero_closure_loss(samples, nc, meta):
    """The a-priori loss of the plain coarse step (a network that outputs zero)."""
    cl = B.Closure((nc,) * 3)
    cl.set_scales(meta["mu"], meta["sd"], meta["sF"], meta["sE"], meta["wU"], meta["wB"])
    cl.set_params(np.zeros(cl.nparams, dtype=np.float32))
    tot = 0.0
    for st, nxt, tgt, dt in samples:
        cl.zero_grad()
        tot += cl.accumulate(st, nxt, tgt, dt)
    cl.close()
    return tot / len(samples)


def apriori_loss(cl, samples):
    tot = 0.0
    for st, nxt, tgt, dt in samples:
        cl.zero_grad()
        tot += cl.accumulate(st, nxt, tgt, dt)
    return tot / len(samples)


def load(path, nc=64):
    z = np.load(path, allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    cl = B.Closure((nc,) * 3)
    cl.set_scales(meta["mu"], meta["sd"], meta["sF"], meta["sE"], meta["wU"], meta["wB"])
    cl.set_params(z["params"])
    return cl, meta


def evaluate(cl, seeds, nc=64, r=4, steps=8):
    """A-posteriori errors against the filtered fine run, and step times."""
    import torch
    res = []
    t_plain = t_clos = t_two = 0.0
    for seed in seeds:
        f = FineToCoarse(seed, nc, r)
        st0 = f.filtered()
        plain = B.Sim((nc,) * 3, scheme=SCHEME)
        clos = B.Sim((nc,) * 3, scheme=SCHEME)
        two = B.Sim((2 * nc,) * 3, scheme=SCHEME)
        plain.set_state(st0)
        clos.set_state(st0)
        # the 2x run starts from the fine state filtered by r/2
        buf2 = torch.empty(8 * (2 * nc) ** 3, dtype=torch.float64, device="cuda:0")
        B.box_filter((nc * r,) * 3, r // 2, f.fine.state(device=True), buf2)
        two.set_state(buf2)
        down = torch.empty(8 * nc ** 3, dtype=torch.float64, device="cuda:0")
        n = nc ** 3
        per = []
        for k in range(steps):
            dt = plain.dt_cfl()
            torch.cuda.synchronize()
            a = time.perf_counter()
            plain.step(dt)
            torch.cuda.synchronize()
            b = time.perf_counter()
            cl.step(clos, dt)
            torch.cuda.synchronize()
            c = time.perf_counter()
            m2 = max(2, math.ceil(dt / (0.9 * two.dt_cfl())))
            for _ in range(m2):
                two.step(dt / m2)
            torch.cuda.synchronize()
            d = time.perf_counter()
            t_plain += b - a
            t_clos += c - b
            t_two += d - c
            f.advance(dt)
            ref = f.filtered()
            B.box_filter((2 * nc,) * 3, 2, two.state(device=True), down)
            torch.cuda.synchronize()
            per.append({"plain": l1_rel(plain.state(device=True), ref, n),
                        "closure": l1_rel(clos.state(device=True), ref, n),
                        "plain_2x": l1_rel(down, ref, n)})
        res.append(per)
        for s in (plain, clos, two):
            s.close()
        f.close()
    cnt = len(seeds) * steps
    return res, {"plain_ms": 1e3 * t_plain / cnt, "closure_ms": 1e3 * t_clos / cnt, "plain_2x_ms": 1e3 * t_two / cnt}


def evaluate_sizes(cl, seeds, sizes=(72, 80), nc=64, r=4, steps=8):
    """Plain runs at other resolutions against the closure at nc^3, to the same time.

    For each seed the plain and the closure run at nc^3 take `steps` CFL steps from the
    fine state filtered to nc^3, reaching time T.  A plain run at n^3 for each n in
    `sizes` starts from the same recipe and seed generated at r*n (its own realisation
    at that resolution) filtered to n^3, and advances to T with its own CFL steps (the
    last one shortened), its fine run alongside.  Every run is compared at T with its
    own filtered fine state.  Returns {run: {"l1": mean relative L1 per class,
    "ms_to_T": mean GPU-synchronised wall time of the coarse steps, "steps": mean
    step count}}."""
    import torch
    out = {}

    def add(name, l1, ms, nsteps):
        e = out.setdefault(name, {"l1": [], "ms_to_T": [], "steps": []})
        e["l1"].append(l1)
        e["ms_to_T"].append(ms)
        e["steps"].append(nsteps)

    for seed in seeds:
        f = FineToCoarse(seed, nc, r)
        st0 = f.filtered()
        plain = B.Sim((nc,) * 3, scheme=SCHEME)
        clos = B.Sim((nc,) * 3, scheme=SCHEME)
        plain.set_state(st0)
        clos.set_state(st0)
        T = t_p = t_c = 0.0
        for k in range(steps):
            dt = plain.dt_cfl()
            torch.cuda.synchronize()
            a = time.perf_counter()
            plain.step(dt)
            torch.cuda.synchronize()
            b = time.perf_counter()
            cl.step(clos, dt)
            torch.cuda.synchronize()
            c = time.perf_counter()
            t_p += b - a
            t_c += c - b
            T += dt
            f.advance(dt)
        ref = f.filtered()
        add(f"plain_{nc}", l1_rel(plain.state(device=True), ref, nc ** 3), 1e3 * t_p, steps)
        add(f"closure_{nc}", l1_rel(clos.state(device=True), ref, nc ** 3), 1e3 * t_c, steps)
        for s_ in (plain, clos):
            s_.close()
        f.close()
        for n in sizes:
            g = FineToCoarse(seed, n, r)
            run = B.Sim((n,) * 3, scheme=SCHEME)
            run.set_state(g.filtered())
            t = el = 0.0
            cnt = 0
            while t < T * (1 - 1e-12):
                dt = min(run.dt_cfl(), T - t)
                torch.cuda.synchronize()
                a = time.perf_counter()
                run.step(dt)
                torch.cuda.synchronize()
                el += time.perf_counter() - a
                g.advance(dt)
                t += dt
                cnt += 1
            add(f"plain_{n}", l1_rel(run.state(device=True), g.filtered(), n ** 3), 1e3 * el, cnt)
            run.close()
            g.close()
        _say(f"seed {seed}: T = {T:.5f}, " + ", ".join(f"{k} E {v['l1'][-1]['E']:.3e} ({v['ms_to_T'][-1]:.2f} ms)"
                                                         for k, v in out.items()))
    return {k: {"l1": {c: float(np.mean([e[c] for e in v["l1"]])) for c in ROWS},
                "ms_to_T": float(np.mean(v["ms_to_T"])), "steps": float(np.mean(v["steps"]))}
            for k, v in out.items()}


def summary(res):
    """Mean over seeds of the relative L1 error after the last step, per run and class."""
    out = {}
    for run in ("plain", "closure", "plain_2x"):
        out[run] = {k: float(np.mean([per[-1][run][k] for per in res])) for k in ROWS}
    return out


def main():
    ap = argparse.ArgumentParser(description="train the learned closure on this solver's own data")
    ap.add_argument("--out", help="train and write the weights and record here")
    ap.add_argument("--eval-sizes", metavar="WEIGHTS",
                    help="instead of training: the closure in WEIGHTS against plain runs at other "
                         "resolutions, to the same time (evaluate_sizes)")
    ap.add_argument("--sizes", type=int, nargs="+", default=[72, 80])
    ap.add_argument("--seeds", type=int, nargs="+", default=[900, 901, 902, 903])
    ap.add_argument("--nc", type=int, default=64)
    ap.add_argument("--r", type=int, default=4)
    ap.add_argument("--train-seeds", type=int, default=128)
    ap.add_argument("--eval-seeds", type=int, default=16)
    ap.add_argument("--iters", type=int, default=12000)
    args = ap.parse_args()
    if args.eval_sizes:
        cl, meta = load(args.eval_sizes)
        res = evaluate_sizes(cl, args.seeds, tuple(args.sizes), meta["nc"], meta["r"])
        cl.close()
        print(json.dumps({"seeds": args.seeds, "runs": res}))
        return
    if not args.out:
        ap.error("--out or --eval-sizes is required")
    train_seeds = list(range(100, 100 + args.train_seeds))
    eval_seeds = list(range(900, 900 + args.eval_seeds))
    samples = make_samples(train_seeds, args.nc, args.r)
    cl, meta, hist = train(samples, args.nc, iters=args.iters)
    meta["zero_closure_loss"] = zero_closure_loss(samples, args.nc, meta)
    meta["trained_loss"] = apriori_loss(cl, samples)
    meta["train_seeds"] = train_seeds
    meta["nc"], meta["r"] = args.nc, args.r
    held = make_samples(eval_seeds, args.nc, args.r, steps=4)
    meta["heldout_zero_loss"] = zero_closure_loss(held, args.nc, meta)
    meta["heldout_trained_loss"] = apriori_loss(cl, held)
    del held
    res, times = evaluate(cl, eval_seeds, args.nc, args.r)
    meta["eval_seeds"] = eval_seeds
    meta["aposteriori_l1_after_8_steps"] = summary(res)
    meta["step_ms"] = times
    params = cl.params()
    np.savez(args.out, params=params, meta=json.dumps(meta), loss=np.array(hist, dtype=np.float32))
    print(json.dumps({k: meta[k] for k in ("zero_closure_loss", "trained_loss", "heldout_zero_loss",
                                           "heldout_trained_loss", "aposteriori_l1_after_8_steps", "step_ms")}))


if __name__ == "__main__":
    main()
