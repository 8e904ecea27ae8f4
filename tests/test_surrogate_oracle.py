"""Pins of the surrogate's FP64 oracle (CPU): the convolution against an
explicit-loop evaluation and against special kernels whose result is known,
the backward pass against the adjoint identity and central finite
differences, Adam against its closed-form first step, and the pooling."""
import numpy as np
import pytest

from oracle import surrogate as S


def _rand(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


@pytest.mark.parametrize("s,u,shape", [(1, 1, (5, 4, 3)), (2, 1, (5, 4, 6)), (1, 2, (3, 2, 3)),
                                       (2, 1, (4, 4, 4)), (1, 1, (1, 1, 1))])
def test_conv_matches_explicit_loops(s, u, shape):
    x = _rand((2, 3) + shape, 1)
    w = _rand((4, 3, 3, 3, 3), 2)
    b = _rand((4,), 3)
    y = S.conv3d(x, w, b, s, u)
    assert y.shape == (2, 4) + S.out_shape(*shape, s, u)
    assert np.abs(y - S.conv3d_direct(x, w, b, s, u)).max() < 1e-12


def test_conv_special_kernels():
    x = _rand((1, 2, 6, 4, 8), 4)
    w = np.zeros((2, 2, 3, 3, 3))
    w[0, 0, 1, 1, 1] = 1.0
    w[1, 1, 1, 1, 1] = 1.0
    b = np.zeros(2)
    assert np.array_equal(S.conv3d(x, w, b, 1, 1), x)                       # identity
    assert np.array_equal(S.conv3d(x, w, b, 2, 1), x[:, :, ::2, ::2, ::2])  # subsampling
    up = S.conv3d(x, w, b, 1, 2)                                            # nearest upsampling
    assert np.array_equal(up[:, :, 1::2, 0::2, 1::2], x)
    # a shift kernel: tap (1, 1, 2) reads x[p + 1] along W, zero at the end
    w2 = np.zeros((1, 1, 3, 3, 3))
    w2[0, 0, 1, 1, 2] = 1.0
    y = S.conv3d(x[:, :1], w2, np.zeros(1))
    assert np.array_equal(y[..., :-1], x[:, :1, ..., 1:]) and np.all(y[..., -1] == 0)
    # a constant field and a kernel of ones: 27 in the interior, fewer at faces
    ones = np.ones((1, 1, 4, 4, 4))
    y = S.conv3d(ones, np.ones((1, 1, 3, 3, 3)), np.zeros(1))
    assert y[0, 0, 1, 1, 1] == 27 and y[0, 0, 0, 0, 0] == 8 and y[0, 0, 0, 1, 1] == 18


@pytest.mark.parametrize("s,u", [(1, 1), (2, 1), (1, 2)])
def test_conv_backward_adjoint_and_bias(s, u):
    x = _rand((2, 3, 4, 6, 5), 5)
    w = _rand((4, 3, 3, 3, 3), 6)
    dy = _rand((2, 4) + S.out_shape(4, 6, 5, s, u), 7)
    dx, dw, db = S.conv3d_backward(x, w, dy, s, u)
    # <conv(x), dy> is linear in x and in w: both adjoints give the same number
    lhs = np.sum(S.conv3d(x, w, np.zeros(4), s, u) * dy)
    assert abs(lhs - np.sum(x * dx)) < 1e-10 * abs(lhs)
    assert abs(lhs - np.sum(w * dw)) < 1e-10 * abs(lhs)
    assert np.allclose(db, dy.sum(axis=(0, 2, 3, 4)))


@pytest.mark.parametrize("s,u", [(1, 1), (2, 1), (1, 2)])
def test_conv_backward_finite_differences(s, u):
    x = _rand((1, 2, 3, 4, 3), 8)
    w = _rand((2, 2, 3, 3, 3), 9)
    b = _rand((2,), 10)
    dy = _rand((1, 2) + S.out_shape(3, 4, 3, s, u), 11)
    f = lambda x_, w_, b_: np.sum(S.conv3d(x_, w_, b_, s, u) * dy)  # noqa: E731
    dx, dw, db = S.conv3d_backward(x, w, dy, s, u)
    h = 1e-6
    rng = np.random.default_rng(12)
    for _ in range(12):
        i = tuple(rng.integers(0, n) for n in x.shape)
        e = np.zeros_like(x)
        e[i] = h
        fd = (f(x + e, w, b) - f(x - e, w, b)) / (2 * h)
        assert abs(fd - dx[i]) < 1e-6 * (1 + abs(fd))
        j = tuple(rng.integers(0, n) for n in w.shape)
        e = np.zeros_like(w)
        e[j] = h
        fd = (f(x, w + e, b) - f(x, w - e, b)) / (2 * h)
        assert abs(fd - dw[j]) < 1e-6 * (1 + abs(fd))
    e = np.array([h, 0.0])
    assert abs((f(x, w, b + e) - f(x, w, b - e)) / (2 * h) - db[0]) < 1e-6


@pytest.mark.parametrize("scale", [1.0, 0.05])
def test_network_gradient_finite_differences(scale):
    spec = S.layers(cin=2, c1=2, c2=3, c3=3)
    P = S.init_params(spec, seed=3)
    for k in P:  # non-zero biases so every term is exercised
        if k.endswith(".b"):
            P[k] = np.random.default_rng(len(k)).standard_normal(P[k].shape) * 0.1
    x = _rand((2, 2, 8, 4, 4), 13)
    t = _rand((2, 2, 8, 4, 4), 14)
    L, G = S.loss_and_grad(P, spec, x, t, scale)
    h = 1e-6
    rng = np.random.default_rng(15)
    checked = 0
    for name in ("e1.w", "e2.w", "e4.w", "b2.w", "d1.w", "d3.w", "out.w", "d2.b", "out.b"):
        for _ in range(3):
            j = tuple(rng.integers(0, n) for n in P[name].shape)
            Pp = {k: v.copy() for k, v in P.items()}
            Pm = {k: v.copy() for k, v in P.items()}
            Pp[name][j] += h
            Pm[name][j] -= h
            fd = (S.loss_and_grad(Pp, spec, x, t, scale)[0] - S.loss_and_grad(Pm, spec, x, t, scale)[0]) / (2 * h)
            # central differences of an O(1) loss at h = 1e-6 carry ~1e-10 of rounding
            assert abs(fd - G[name][j]) < 1e-5 * abs(fd) + 1e-9, (name, j, fd, G[name][j])
            checked += 1
    assert checked == 27


def test_input_gradient_includes_residual_path():
    spec = S.layers(cin=1, c1=2, c2=2, c3=2)
    P = S.init_params(spec, seed=4)
    x = _rand((1, 1, 4, 4, 4), 16)
    pred, cache = S.forward(P, spec, x)
    dpred = _rand(pred.shape, 17)
    _, dx = S.backward(P, spec, cache, dpred)
    f = lambda x_: np.sum(S.forward(P, spec, x_)[0] * dpred)  # noqa: E731
    h = 1e-6
    for i in [(0, 0, 0, 0, 0), (0, 0, 2, 1, 3), (0, 0, 3, 3, 3)]:
        e = np.zeros_like(x)
        e[i] = h
        assert abs((f(x + e) - f(x - e)) / (2 * h) - dx[i]) < 1e-6


def test_parameter_count_of_the_production_network():
    spec = S.layers()
    n = S.n_params(spec)
    assert 400_000 <= n <= 600_000, n


def test_adam_first_step_and_convergence():
    P = {"a": np.array([1.0, -2.0, 3.0])}
    G = {"a": np.array([0.5, -4.0, 1e-3])}
    st = {"t": 0, "m": {}, "v": {}}
    S.adam_step(P, G, st, lr=0.1, eps=0.0)
    # bias-corrected first step: m_hat = g, v_hat = g^2 -> move by lr sign(g)
    assert np.allclose(P["a"], [0.9, -1.9, 2.9], atol=1e-15)
    # minimise |P - c|^2
    c = np.array([0.3, 0.7, -0.2])
    P = {"a": np.zeros(3)}
    st = {"t": 0, "m": {}, "v": {}}
    for _ in range(2000):
        S.adam_step(P, {"a": 2 * (P["a"] - c)}, st, lr=1e-2)
    assert np.abs(P["a"] - c).max() < 1e-3


def test_pool2_and_mass_drift():
    z, y, x = np.meshgrid(np.arange(4.0), np.arange(6.0), np.arange(8.0), indexing="ij")
    f = 2 * x + 3 * y - z
    p = S.pool2(f)
    zc, yc, xc = np.meshgrid(np.arange(2) * 2 + 0.5, np.arange(3) * 2 + 0.5, np.arange(4) * 2 + 0.5,
                             indexing="ij")
    assert np.allclose(p, 2 * xc + 3 * yc - zc)
    assert np.isclose(p.sum() * 8, f.sum())
    a = np.ones((2, 3, 3))
    b = a * 1.001
    assert np.allclose(S.relative_mass_drift(b, a), 1e-3)


def test_mass_term_gradient_and_value():
    rng = np.random.default_rng(21)
    pred = rng.standard_normal((3, 5, 4, 3, 2))
    tgt = rng.standard_normal((3, 5, 4, 3, 2))
    mw = 7.0
    L, g = S.mse(pred, tgt, mw)
    d = pred - tgt
    m = d[:, 0].reshape(3, -1).mean(axis=1)
    assert abs(L - (np.mean(d * d) + mw * np.mean(m * m))) < 1e-14
    h = 1e-6
    for idx in [(0, 0, 1, 2, 1), (2, 0, 3, 0, 0), (1, 3, 2, 1, 1)]:
        e = np.zeros_like(pred)
        e[idx] = h
        fd = (S.mse(pred + e, tgt, mw)[0] - S.mse(pred - e, tgt, mw)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-8
    # a uniform shift of the phase field in one sample is penalised beyond the plain MSE
    shifted = tgt.copy()
    shifted[0, 0] += 0.01
    assert S.mse(shifted, tgt, mw)[0] > S.mse(shifted, tgt, 0.0)[0]
