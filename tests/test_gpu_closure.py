"""The learned closure's HIP kernels against the FP64 reference of oracle/closure.py.

The network runs on the matrix cores with BF16 operands and FP32 accumulation, so the
forward pass is compared with the reference evaluated on the same BF16-rounded
operands (input channels, weights, hidden activations), and the gradients in relative
L2 norm; the closure itself (FP64 state update from the FP32 output) and the box filter
are exact up to FP64 rounding."""
import numpy as np
import pytest
import torch

from oracle import closure as C
from paper_2608_14048_amd import binding as B
from paper_2608_14048_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def random_params(rng, scale=(0.25, 0.12, 0.12, 0.12)):
    out = []
    for l, (w, b) in enumerate(C.param_shapes()):
        out.append((scale[l] * rng.standard_normal(w), 0.05 * rng.standard_normal(b)))
    return out


def setup(shape, seed):
    rng = np.random.default_rng(seed)
    st = I.turbulence_block(shape, seed=seed)[0]
    L = tuple(v / max(shape) for v in shape)
    mu = C.primitives(st, shape).reshape(8, -1).mean(axis=1)
    sd = C.primitives(st, shape).reshape(8, -1).std(axis=1) + 1e-3
    params = random_params(rng)
    cl = B.Closure(shape, L)
    cl.set_params(C.pack(params).astype(np.float32))
    sF = np.array([1e-2, 2e-2, 2e-2, 2e-2, 3e-2])
    sE, wU, wB = 1e-2, np.array([1.0, 2.0, 2.0, 2.0, 0.5]), 1.5
    cl.set_scales(mu.astype(np.float32), sd.astype(np.float32), sF.astype(np.float32), sE, wU.astype(np.float32), wB)
    # the reference sees the parameters and scales as the device holds them (FP32)
    params32 = C.unpack(C.pack(params).astype(np.float32).astype(np.float64))
    return st, L, cl, params32, mu.astype(np.float32).astype(np.float64), sd.astype(np.float32).astype(np.float64), \
        sF.astype(np.float32).astype(np.float64), float(np.float32(sE)), wU, wB, rng


def emulated_forward(params, x):
    """The reference forward pass with the device's BF16 rounding points."""
    h = bf16(x)
    for l, (W, b) in enumerate(params):
        z = C.conv(h, bf16(W), b)
        h = bf16(np.maximum(z, 0.0)) if l < len(params) - 1 else z
    return h


def emulated_backward(params, acts, dout):
    """The reference backward pass with the device's BF16 rounding points: BF16 weights
    and activations, the output gradient and every back-propagated gradient rounded to
    BF16 before use, FP64 accumulation."""
    grads = [None] * len(params)
    g = bf16(dout)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        grads[l] = C.conv_grad_weight(acts[l], g)
        if l > 0:
            g = bf16(C.conv_grad_input(g, bf16(W)) * (acts[l] > 0.0))
    return grads


def emulated_acts(params, x):
    acts = [bf16(x)]
    h = acts[0]
    for l, (W, b) in enumerate(params):
        z = C.conv(h, bf16(W), b)
        h = bf16(np.maximum(z, 0.0)) if l < len(params) - 1 else z
        acts.append(h)
    return h, acts


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


# (16, 4, 8) tiles into the LDS-staged 16 x 4 x 8 convolution blocks, (16, 8, 12) into
# 16 x 4 x 4 ones; (32, 6, 5) does neither and takes the per-tap gather kernel
@pytest.mark.parametrize("shape", [(16, 4, 8), (16, 8, 12), (32, 6, 5)])
def test_forward_matches_bf16_reference(shape):
    st, L, cl, params, mu, sd, sF, sE, wU, wB, _ = setup(shape, 1)
    try:
        out = cl.forward(dev(st)).cpu().numpy().reshape(18, shape[2], shape[1], shape[0])
        ref = emulated_forward(params, C.normalised_input(st, shape, mu, sd))
        exact, _ = C.forward(params, C.normalised_input(st, shape, mu, sd))
        scale = np.abs(ref).max()
        e = np.abs(out - ref).max() / scale
        e_exact = np.abs(out - exact).max() / scale
        _say(f"  forward: max error vs BF16-emulated reference {e:.2e}, vs exact FP64 {e_exact:.2e}")
        assert e < 2e-2
        assert np.abs(out - ref).mean() / np.abs(ref).mean() < 2e-3
        assert e_exact < 6e-2
    finally:
        cl.close()


def test_closure_apply_and_box_filter_exact():
    shape = (16, 8, 12)
    st, L, cl, params, mu, sd, sF, sE, wU, wB, rng = setup(shape, 2)
    try:
        out = cl.forward(dev(st)).cpu().numpy().astype(np.float64).reshape(18, shape[2], shape[1], shape[0])
        s = dev(st)
        cl.apply(0.01, s)
        dx = tuple(L[a] / shape[a] for a in range(3))
        ref = C.apply_closure(st, shape, out, sF, sE, 0.01, dx)
        e = np.abs(s.cpu().numpy() - ref).max() / np.abs(st).max()
        _say(f"  closure apply: max error {e:.2e}")
        assert e < 1e-14
        fine = (32, 16, 24)
        fs = I.turbulence_block(fine, seed=3)[0]
        co = torch.empty(fs.size // 8, dtype=torch.float64, device="cuda:0")
        B.box_filter(fine, 2, dev(fs), co)
        torch.cuda.synchronize()
        assert np.abs(co.cpu().numpy() - C.box_filter(fs, fine, 2)).max() <= 1e-15 * np.abs(fs).max()
    finally:
        cl.close()


def test_gradients_match_reference():
    shape = (16, 8, 8)
    st, L, cl, params, mu, sd, sF, sE, wU, wB, rng = setup(shape, 4)
    try:
        dx = tuple(L[a] / shape[a] for a in range(3))
        dt = 2e-3
        coarse = st + 1e-4 * rng.standard_normal(st.shape)
        target = st + 1e-4 * rng.standard_normal(st.shape)
        cl.zero_grad()
        loss = cl.accumulate(dev(st), dev(coarse), dev(target), dt)
        g = cl.grads().astype(np.float64)
        x = C.normalised_input(st, shape, mu, sd)
        out, acts = emulated_acts(params, x)
        pred = C.apply_closure(coarse, shape, out, sF, sE, dt, dx)
        ref_loss = C.loss(pred, target, shape, wU, wB)
        gref = C.pack(emulated_backward(params, acts, C.loss_grad_out(pred, target, shape, sF, sE, dt, dx, wU, wB)))
        # and the exact FP64 gradient, for the record
        out64, acts64 = C.forward(params, x)
        pred64 = C.apply_closure(coarse, shape, out64, sF, sE, dt, dx)
        g64 = C.pack(C.backward(params, acts64, C.loss_grad_out(pred64, target, shape, sF, sE, dt, dx, wU, wB)))
        _say(f"  whole gradient vs exact FP64: relative L2 {np.linalg.norm(g - g64) / np.linalg.norm(g64):.2e}")
        _say(f"  loss {loss:.6e} vs reference {ref_loss:.6e}")
        assert abs(loss - ref_loss) <= 1e-3 * ref_loss
        at = 0
        for l, (w, b) in enumerate(C.param_shapes()):
            for kind, part in (("W", int(np.prod(w))), ("b", int(np.prod(b)))):
                a, r = g[at:at + part], gref[at:at + part]
                if l == len(C.param_shapes()) - 1 and kind == "b":
                    # a uniform face flux or EMF has zero divergence and curl: the output
                    # biases are a null direction of the loss, their gradient is round-off
                    wl = np.linalg.norm(g[at - int(np.prod(w)):at])
                    _say(f"  layer {l} b: |grad| {np.linalg.norm(a):.2e} (reference {np.linalg.norm(r):.2e}; |grad W| {wl:.2e})")
                    assert np.linalg.norm(a) < 1e-3 * wl
                else:
                    rel = np.linalg.norm(a - r) / np.linalg.norm(r)
                    cos = a @ r / (np.linalg.norm(a) * np.linalg.norm(r))
                    _say(f"  layer {l} {kind}: relative L2 {rel:.2e}, cosine {cos:.6f}")
                    assert rel < 1e-2 and cos > 0.9999
                at += part
    finally:
        cl.close()


def test_zero_network_is_the_plain_step_and_training_lowers_the_loss():
    shape = (16, 16, 16)
    st = I.turbulence_block(shape, seed=7)[0]
    scheme = dict(recon="ppm", riemann="hlld", integ="vl2")
    a, b = B.Sim(shape, scheme=scheme), B.Sim(shape, scheme=scheme)
    cl = B.Closure(shape)
    try:
        a.set_state(st)
        b.set_state(st)
        dt = a.dt_cfl()
        a.step(dt)
        cl.step(b, dt)  # zero parameters: exactly the plain step
        assert np.array_equal(a.state(), b.state())
        assert a.dt_cfl() == b.dt_cfl()
        # a teacher network makes the targets; training a differently seeded student must
        # lower the loss
        rng = np.random.default_rng(8)
        teacher = C.pack(random_params(rng, scale=(0.2, 0.1, 0.1, 0.1))).astype(np.float32)
        mu = C.primitives(st, shape).reshape(8, -1).mean(axis=1)
        sd = C.primitives(st, shape).reshape(8, -1).std(axis=1) + 1e-3
        scales = (mu, sd, np.full(5, 1e-2), 1e-2, np.ones(5), 1.0)
        cl.set_scales(*scales)
        cl.set_params(teacher)
        s0 = torch.from_numpy(st).to("cuda:0")
        coarse = a.state(device=True)
        target = coarse.clone()
        cl.forward(s0)
        cl.apply(dt, target)
        cl.set_params(C.pack(random_params(np.random.default_rng(9), scale=(0.2, 0.1, 0.1, 0.1))).astype(np.float32))
        losses = []
        for it in range(60):
            cl.zero_grad()
            losses.append(cl.accumulate(s0, coarse, target, dt))
            cl.adam(2e-3)
        _say(f"  teacher-student loss {losses[0]:.3e} -> {losses[-1]:.3e}")
        assert losses[-1] < 0.5 * losses[0]
    finally:
        a.close()
        b.close()
        cl.close()


def test_closure_step_falls_back_to_the_plain_step():
    """A network scaled so that its corrections would drive the state below the floors
    (or make it non-finite) is rejected: the plain step stands, bit for bit, and the
    step reports the fallback; a zero network is applied (and changes nothing)."""
    shape = (16, 16, 16)
    st = I.turbulence_block(shape, seed=11)[0]
    scheme = dict(recon="ppm", riemann="hlld", integ="vl2")
    a, b = B.Sim(shape, scheme=scheme), B.Sim(shape, scheme=scheme)
    cl = B.Closure(shape)
    try:
        a.set_state(st)
        b.set_state(st)
        dt = a.dt_cfl()
        a.step(dt)
        assert cl.step(b, dt, report=True) == 1          # zero network: applied
        assert np.array_equal(a.state(), b.state())
        assert a.dt_cfl() == b.dt_cfl()
        # a wild network: corrections of order 1e6 of the state
        rng = np.random.default_rng(12)
        cl.set_params(C.pack(random_params(rng, scale=(2.0, 2.0, 2.0, 2.0))).astype(np.float32))
        mu = C.primitives(st, shape).reshape(8, -1).mean(axis=1)
        sd = C.primitives(st, shape).reshape(8, -1).std(axis=1) + 1e-3
        cl.set_scales(mu, sd, np.full(5, 1e3), 1e3, np.ones(5), 1.0)
        a.set_state(st)
        b.set_state(st)
        a.step(dt)
        assert cl.step(b, dt, report=True) == 0          # rejected: the plain step stands
        assert np.array_equal(a.state(), b.state())
        assert a.dt_cfl() == b.dt_cfl()
        # a mild network with small output scales is applied and changes the state
        cl.set_params(C.pack(random_params(rng, scale=(0.2, 0.1, 0.1, 0.1))).astype(np.float32))
        cl.set_scales(mu, sd, np.full(5, 1e-4), 1e-4, np.ones(5), 1.0)
        b.set_state(st)
        assert cl.step(b, dt, report=True) == 1
        d = np.abs(b.state() - a.state()).max()
        assert 0.0 < d < 1e-3, d
    finally:
        a.close()
        b.close()
        cl.close()


def test_closure_step_rejects_other_grids_and_streams():
    shape = (16, 16, 8)
    cl = B.Closure(shape)
    try:
        # the same number of cells on a transposed grid
        other = B.Sim((16, 8, 16), scheme=dict(recon="plm"))
        other.set_state(I.turbulence_block((16, 8, 16), seed=1)[0])
        with pytest.raises(B.MhdError) as e:
            cl.step(other, 1e-3)
        assert e.value.code == -1
        other.close()
        # the same grid on another stream
        s = torch.cuda.Stream()
        sim = B.Sim(shape, scheme=dict(recon="plm"), stream=s)
        sim.set_state(I.turbulence_block(shape, seed=2)[0])
        with pytest.raises(B.MhdError) as e:
            cl.step(sim, 1e-3)
        assert e.value.code == -1
        sim.close()
        # an FP32-bulk context
        sim = B.Sim(shape, scheme=dict(recon="plm", prec="fp32_bulk"))
        sim.set_state(I.turbulence_block(shape, seed=2)[0])
        with pytest.raises(B.MhdError) as e:
            cl.step(sim, 1e-3)
        assert e.value.code == -2
        sim.close()
    finally:
        cl.close()
