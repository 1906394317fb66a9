"""Pins of the closure oracle (CPU): the convolution against a brute-force sum, each
adjoint against its defining identity, the whole gradient against finite differences,
and the closure's conservation and div B properties."""
import numpy as np
import pytest

from oracle import closure as C
from paper_2608_14048_amd import inputs as I


def test_conv_matches_brute_force_sum():
    rng = np.random.default_rng(0)
    nz, ny, nx = 3, 4, 5
    x = rng.standard_normal((2, nz, ny, nx))
    W = rng.standard_normal((27, 2, 3))
    b = rng.standard_normal(3)
    y = C.conv(x, W, b)
    for co in range(3):
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    s = b[co]
                    for t, (dx, dy, dz) in enumerate(C.TAPS):
                        for ci in range(2):
                            s += W[t, ci, co] * x[ci, (k + dz) % nz, (j + dy) % ny, (i + dx) % nx]
                    assert abs(y[co, k, j, i] - s) < 1e-12


def test_conv_adjoints():
    rng = np.random.default_rng(1)
    sh = (4, 3, 5)
    x = rng.standard_normal((3,) + sh)
    dy = rng.standard_normal((2,) + sh)
    W = rng.standard_normal((27, 3, 2))
    zero = np.zeros(2)
    # <conv(x), dy> = <x, conv^T(dy)>
    assert abs(np.sum(C.conv(x, W, zero) * dy) - np.sum(x * C.conv_grad_input(dy, W))) < 1e-10
    # the weight gradient of the bilinear form <conv(x, W, b), dy> is exact for any step
    dW, db = C.conv_grad_weight(x, dy)
    for (t, ci, co) in [(0, 0, 0), (13, 2, 1), (26, 1, 0), (7, 0, 1)]:
        E = np.zeros_like(W)
        E[t, ci, co] = 1.0
        fd = np.sum(C.conv(x, W + E, zero) * dy) - np.sum(C.conv(x, W, zero) * dy)
        assert abs(fd - dW[t, ci, co]) < 1e-10
    assert np.allclose(db, dy.sum(axis=(1, 2, 3)))


def _problem(seed=2, shape=(4, 4, 4), widths=(8, 4, 4, 4, 18)):
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    params = [(0.3 * rng.standard_normal(w), 0.1 * rng.standard_normal(b)) for w, b in C.param_shapes(widths)]
    st = I.turbulence_block(shape, seed=seed)[0]
    target = st + 1e-3 * rng.standard_normal(st.shape)
    coarse = st + 1e-3 * rng.standard_normal(st.shape)
    x = C.normalised_input(st, shape, np.zeros(8), np.ones(8))
    sF = np.array([1e-2, 2e-2, 2e-2, 2e-2, 3e-2])
    return params, x, coarse, target, sF, 2e-2, 0.01, (1 / nx, 1 / ny, 1 / nz), rng


def _total_loss(params, x, coarse, target, sF, sE, dt, dx, shape, wU, wB):
    out, _ = C.forward(params, x)
    pred = C.apply_closure(coarse, shape, out, sF, sE, dt, dx)
    return C.loss(pred, target, shape, wU, wB)


def test_network_gradient_matches_finite_differences():
    shape = (4, 4, 4)
    params, x, coarse, target, sF, sE, dt, dx, rng = _problem(shape=shape)
    wU, wB = [1.0, 0.5, 0.5, 0.5, 2.0], 0.7
    out, acts = C.forward(params, x)
    pred = C.apply_closure(coarse, shape, out, sF, sE, dt, dx)
    g_out = C.loss_grad_out(pred, target, shape, sF, sE, dt, dx, wU, wB)
    grads = C.backward(params, acts, g_out)
    flat = C.pack(params)
    gflat = C.pack(grads)
    widths = (8, 4, 4, 4, 18)
    h = 1e-6
    for q in rng.choice(flat.size, 40, replace=False):
        e = np.zeros_like(flat)
        e[q] = h
        lp = _total_loss(C.unpack(flat + e, widths), x, coarse, target, sF, sE, dt, dx, shape, wU, wB)
        lm = _total_loss(C.unpack(flat - e, widths), x, coarse, target, sF, sE, dt, dx, shape, wU, wB)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gflat[q]) <= 1e-6 * max(1e-8, abs(fd)) + 1e-12, (q, fd, gflat[q])


def test_closure_is_conservative_and_keeps_div_b():
    shape = (6, 5, 4)
    nx, ny, nz = shape
    rng = np.random.default_rng(3)
    st = I.turbulence_block(shape, seed=3)[0]
    L = tuple(v / max(shape) for v in shape)
    dx = tuple(L[a] / shape[a] for a in range(3))
    out = rng.standard_normal((18, nz, ny, nx))
    new = C.apply_closure(st, shape, out, rng.uniform(0.5, 1, 5), 0.3, 0.01, dx)
    u0, u1 = st.reshape(8, nz, ny, nx), new.reshape(8, nz, ny, nx)
    for f in range(5):
        assert abs(u1[f].sum() - u0[f].sum()) < 1e-12 * np.abs(u0[f]).sum() + 1e-12
    div = lambda u: ((C.shift(u[5], (1, 0, 0)) - u[5]) / dx[0] + (C.shift(u[6], (0, 1, 0)) - u[6]) / dx[1]
                     + (C.shift(u[7], (0, 0, 1)) - u[7]) / dx[2])
    assert np.abs(div(u1) - div(u0)).max() < 1e-11 * np.abs(u0[5:]).max() / min(dx)
    assert not np.allclose(u1[5:], u0[5:])
    # zero corrections leave the state alone
    assert np.array_equal(C.apply_closure(st, shape, 0 * out, np.ones(5), 1.0, 0.01, dx), st)


def test_loss_gradient_in_the_output_matches_finite_differences():
    shape = (3, 4, 5)
    nx, ny, nz = shape
    rng = np.random.default_rng(4)
    st = I.turbulence_block(shape, seed=4)[0]
    target = st + 1e-2 * rng.standard_normal(st.shape)
    dx = (0.2, 0.25, 1 / 3)
    sF, sE, dt = rng.uniform(0.5, 2, 5), 0.7, 0.05
    wU, wB = rng.uniform(0.5, 2, 5), 1.3
    out = rng.standard_normal((18, nz, ny, nx))
    pred = C.apply_closure(st, shape, out, sF, sE, dt, dx)
    g = C.loss_grad_out(pred, target, shape, sF, sE, dt, dx, wU, wB)
    for _ in range(30):
        ch, k, j, i = (int(rng.integers(18)), int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx)))
        e = np.zeros_like(out)
        e[ch, k, j, i] = 1e-6
        lp = C.loss(C.apply_closure(st, shape, out + e, sF, sE, dt, dx), target, shape, wU, wB)
        lm = C.loss(C.apply_closure(st, shape, out - e, sF, sE, dt, dx), target, shape, wU, wB)
        fd = (lp - lm) / 2e-6
        assert abs(fd - g[ch, k, j, i]) <= 1e-6 * abs(fd) + 1e-13, (ch, fd, g[ch, k, j, i])


def test_box_filter_keeps_totals_and_div_b():
    fine = (16, 8, 12)
    r = 4
    st = I.turbulence_block(fine, seed=5)[0]
    L = tuple(v / max(fine) for v in fine)
    co = C.box_filter(st, fine, r)
    cs = tuple(v // r for v in fine)
    u0, u1 = st.reshape(8, fine[2], fine[1], fine[0]), co.reshape(8, cs[2], cs[1], cs[0])
    for f in range(5):
        assert abs(u1[f].mean() - u0[f].mean()) < 1e-14 * np.abs(u0[f]).mean() + 1e-15
    dxc = tuple(L[a] / cs[a] for a in range(3))
    div = ((C.shift(u1[5], (1, 0, 0)) - u1[5]) / dxc[0] + (C.shift(u1[6], (0, 1, 0)) - u1[6]) / dxc[1]
           + (C.shift(u1[7], (0, 0, 1)) - u1[7]) / dxc[2])
    assert np.abs(div).max() * min(dxc) < 1e-13 * np.abs(u1[5:]).max()
    const = np.concatenate([np.full(int(np.prod(fine)), v) for v in (1.0, 0.1, 0.2, 0.3, 2.0, 0.5, 0.6, 0.7)])
    assert np.allclose(C.box_filter(const, fine, r).reshape(8, -1), np.array([1.0, 0.1, 0.2, 0.3, 2.0, 0.5, 0.6, 0.7])[:, None])


def test_primitives_of_one_cell():
    shape = (4, 3, 2)
    st = I.turbulence_block(shape, seed=6)[0]
    w = C.primitives(st, shape)
    u = st.reshape(8, 2, 3, 4)
    k, j, i = 1, 2, 3
    rho = u[0, k, j, i]
    v = u[1:4, k, j, i] / rho
    b = np.array([0.5 * (u[5, k, j, i] + u[5, k, j, 0]), 0.5 * (u[6, k, j, i] + u[6, k, 0, i]),
                  0.5 * (u[7, k, j, i] + u[7, 0, j, i])])
    p = (5 / 3 - 1) * (u[4, k, j, i] - 0.5 * rho * v @ v - 0.5 * b @ b)
    assert np.allclose(w[:, k, j, i], np.concatenate([[rho], v, [p], b]), rtol=1e-14, atol=1e-14)
