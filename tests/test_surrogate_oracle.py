"""Pins of the surrogate's FP64 oracle: finite differences for every gradient,
reductions of the 3x3 convolution to a plain matmul, to a pure shift and to
scipy's 2-D correlation, a closed form of the first Adam step, and bfloat16
rounding against torch's conversion."""
import numpy as np
import pytest
import scipy.signal
import torch

from oracle import surrogate_oracle as S


def rand_layer(rng, cin, cout, scale=0.3):
    return rng.standard_normal((cout, 9, cin)) * scale, rng.standard_normal(cout) * 0.1


def test_conv_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 7, 9, 3))
    w, b = rand_layer(rng, 3, 4)
    z = S.conv_forward(x, w, b)
    for bi in range(2):
        for co in range(4):
            ref = np.full((7, 9), b[co])
            for ci in range(3):
                ker = w[co, :, ci].reshape(3, 3)  # [dy + 1][dx + 1]
                ref += scipy.signal.correlate2d(x[bi, :, :, ci], ker, mode="same", boundary="fill")
            assert np.allclose(z[bi, :, :, co], ref, atol=1e-13)


def test_centre_tap_is_matmul_and_delta_tap_is_shift():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 5, 6, 4))
    w = np.zeros((4, 9, 4))
    w[:, 4, :] = rng.standard_normal((4, 4))
    b = rng.standard_normal(4)
    assert np.allclose(S.conv_forward(x, w, b), x @ w[:, 4, :].T + b, atol=1e-14)
    for t, (dy, dx) in enumerate(S.TAPS):
        w = np.zeros((4, 9, 4))
        w[:, t, :] = np.eye(4)
        z = S.conv_forward(x, w, np.zeros(4))
        for y in range(5):
            for xx in range(6):
                yy, xs = y + dy, xx + dx
                want = x[0, yy, xs] if 0 <= yy < 5 and 0 <= xs < 6 else 0.0
                assert np.allclose(z[0, y, xx], want)


def _fd(f, p, eps=1e-6):
    g = np.zeros_like(p)
    it = np.nditer(p, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        old = p[i]
        p[i] = old + eps
        fp = f()
        p[i] = old - eps
        fm = f()
        p[i] = old
        g[i] = (fp - fm) / (2 * eps)
    return g


def test_conv_backward_finite_differences():
    rng = np.random.default_rng(3)
    x = rng.standard_normal((2, 4, 5, 3))
    w, b = rand_layer(rng, 3, 2)
    r = rng.standard_normal((2, 4, 5, 2))
    f = lambda: float(np.sum(r * S.conv_forward(x, w, b)))
    dx, dw, db = S.conv_backward(x, w, r)
    for ana, p in ((dx, x), (dw, w), (db, b)):
        num = _fd(f, p)
        assert np.abs(ana - num).max() / np.abs(num).max() < 1e-7


def test_silu_grad_finite_differences():
    z = np.linspace(-6, 6, 101)
    num = (S.silu(z + 1e-6) - S.silu(z - 1e-6)) / 2e-6
    assert np.abs(S.silu_grad(z) - num).max() < 1e-8


def test_network_gradients_finite_differences():
    rng = np.random.default_rng(4)
    layers = [rand_layer(rng, 3, 5), rand_layer(rng, 5, 4), rand_layer(rng, 4, 4)]
    x = rng.standard_normal((2, 4, 4, 3))
    target = rng.standard_normal((2, 4, 4, 2))

    def f():
        zs, _ = S.forward(layers, x)
        return S.mse(zs[-1][..., :2], target)[0]

    _, grads = S.loss_and_grads(layers, x, target, 2)
    for l, (w, b) in enumerate(layers):
        for ana, p in ((grads[l][0], w), (grads[l][1], b)):
            num = _fd(f, p)
            assert np.abs(ana - num).max() / np.abs(num).max() < 1e-7, l


def test_adam_first_step_closed_form_and_convergence():
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = S.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    # minimise a separable quadratic: converges to its minimiser
    c = np.array([1.0, -3.0, 0.5])
    p, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 3001):
        p, m, v = S.adam_step(p, 2 * (p - c), m, v, t, lr=0.05)
    assert np.abs(p - c).max() < 1e-3


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(5)
    vals = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                           [1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -9, -0.0, 65504.0, 1e-30]])
    want = torch.tensor(vals, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(S.bf16(vals), want)


def test_features_layout():
    f = S.features(np.array([[0.1, 0.2, 0.3, 0.4, 0.5]]), 4, 8)
    assert f.shape == (1, 4, 8, 15)
    assert np.allclose(f[0, :, :, 2], 0.3)
    assert np.allclose(f[0, 0, :, 5], (np.arange(8) + 0.5) / 8)
    assert np.allclose(f[0, :, 0, 6], (np.arange(4) + 0.5) / 4)
    assert np.allclose(f[..., 7] ** 2 + f[..., 8] ** 2, 1.0)
    assert np.allclose(f[0, 1, 3, 13], np.sin(2 * np.pi * 1.5 / 4))


# ---- warm-start preparation: smoothing and staggered-momentum removal ------
def test_smooth_equals_library_correlation():
    from scipy import ndimage

    rng = np.random.default_rng(3)
    a = rng.standard_normal((3, 11, 17))
    k = np.outer([1, 2, 1], [1, 2, 1]) / 16.0
    want = np.stack([ndimage.correlate(x, k, mode="nearest") for x in a])
    assert np.allclose(S.smooth(a), want, rtol=0, atol=1e-14)


def test_smooth_kills_grid_scale_and_keeps_constants():
    H, W = 12, 10
    y, x = np.mgrid[0:H, 0:W]
    assert np.abs(S.smooth(((-1.0) ** x)[None])[0][:, 1:-1]).max() < 1e-15
    assert np.abs(S.smooth(((-1.0) ** y)[None])[0][1:-1, :]).max() < 1e-15
    assert np.allclose(S.smooth(np.full((1, H, W), 2.5)), 2.5, rtol=0, atol=1e-15)
    lin = (0.3 * x + 0.7 * y)[None].astype(float)
    assert np.allclose(S.smooth(lin)[0][1:-1, 1:-1], lin[0][1:-1, 1:-1], rtol=0, atol=1e-13)


def test_destagger_removes_only_the_staggered_sums():
    rng = np.random.default_rng(4)
    n, H, W = 2, 10, 14
    f = rng.standard_normal((n, 4, H, W))
    g = S.destagger(f)
    y, x = np.mgrid[0:H, 0:W]
    sx, sy = (-1.0) ** x, (-1.0) ** y
    for k in range(n):
        assert abs(np.sum(g[k, 0] * sx)) < 1e-12 and abs(np.sum(g[k, 1] * sy)) < 1e-12
        assert np.array_equal(g[k, 2:], f[k, 2:])
        du, dv = f[k, 0] - g[k, 0], f[k, 1] - g[k, 1]
        assert np.allclose(du, du[0, 0] * sx, rtol=0, atol=1e-14)   # a pure (-1)^x pattern
        assert np.allclose(dv, dv[0, 0] * sy, rtol=0, atol=1e-14)
    assert np.allclose(S.destagger(g), g, rtol=0, atol=1e-14)      # idempotent


def test_staggered_momentum_is_a_lattice_invariant(oracle_mod):
    """The reason for the removal, pinned on the LB oracle: without force,
    Q_y = sum (-1)^y j_y and Q_x = sum (-1)^x j_x flip sign every step exactly
    (collision conserves momentum; streaming and bounce-back flip the parity),
    with no-slip walls and with an even periodic axis."""
    from paper_2101_03055_amd import workloads as W

    for fb in (["noslip"] * 4, ["periodic", "periodic", "noslip", "noslip"]):
        sb = [["noflux"] * 2] * 4 if fb[0] == "noslip" else [["periodic"] * 2] * 2 + [["noflux"] * 2] * 2
        wl, phi0, u0, p0 = W.random_case(16, 12, seed=8, fluid_bc=fb, scalar_bc=sb, force=False)
        o = oracle_mod.Oracle(wl, phi0, u0, p0)
        y, x = np.mgrid[0:12, 0:16]
        sx, sy = (-1.0) ** x, (-1.0) ** y
        q = []
        for t in range(6):
            _, u, _ = o.moments()
            q.append((np.sum(u[0] * sx), np.sum(u[1] * sy)))
            o.step(1)
        q = np.array(q)
        assert np.abs(q).min() > 1e-4
        assert np.allclose(q[1:], -q[:-1], rtol=1e-11, atol=0), fb
