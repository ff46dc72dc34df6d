"""Pins of the oracle's warm-start CNN (forward, input and weight gradients,
loss gradients, BF16 rounding) against facts independent of its code:
scipy's n-D correlation, an impulse response written out by coordinates,
adjointness, linearity in the weights, positive homogeneity, central finite
differences and torch's own float32 -> bfloat16 conversion.  The residual
loss (the network's guess judged as a solver's initial guess) is pinned by
central differences on a nonsymmetric operator (a transposed operand would
fail it), by its reduction to the solution loss with target x when A = I,
and by its value 1 for the zero network."""
import numpy as np
import pytest
import torch
from scipy import ndimage

import oracle


def _vol(a, N):
    """(n,) channel vector -> (z, y, x) array (r = x + N y + N^2 z)."""
    return np.asarray(a).reshape(N, N, N)


def _kernel(w27):
    """27 taps, t = (dz+1)*9 + (dy+1)*3 + (dx+1) -> k[dz+1, dy+1, dx+1]."""
    return np.asarray(w27).reshape(3, 3, 3)


def _scipy_conv(N, W, x):
    """Zero-padded 3x3x3 cross-correlation summed over input channels."""
    cout, cin = W.shape[:2]
    x = x.reshape(N ** 3, cin)
    y = np.zeros((N ** 3, cout))
    for co in range(cout):
        acc = np.zeros((N, N, N))
        for ci in range(cin):
            acc += ndimage.correlate(_vol(x[:, ci], N), _kernel(W[co, ci]), mode="constant",
                                     cval=0.0)
        y[:, co] = acc.reshape(-1)
    return y


@pytest.mark.parametrize("cin,cout", [(1, 3), (4, 2), (16, 16), (16, 1)])
def test_conv_matches_scipy_correlate(cin, cout):
    N = 6
    rng = np.random.default_rng(11 + cin + cout)
    W = rng.standard_normal((cout, cin, 27))
    x = rng.standard_normal((N ** 3, cin))
    y = oracle.conv3d_fwd(N, W, x)
    assert np.allclose(y, _scipy_conv(N, W, x), rtol=1e-12, atol=1e-12)


def test_impulse_response_by_coordinates():
    # out[r, co] = sum_t W[co][0][t] in[r + off(t)]: a unit impulse at
    # (x0, y0, z0) appears at (x0 - dx, y0 - dy, z0 - dz) with weight W[t]
    N = 7
    x0, y0, z0 = 3, 2, 4
    W = np.arange(1, 28, dtype=np.float64).reshape(1, 1, 27) * np.array([1.0, -2.0]).reshape(2, 1, 1)
    x = np.zeros(N ** 3)
    x[x0 + N * y0 + N * N * z0] = 1.0
    y = oracle.conv3d_fwd(N, W, x)
    expect = np.zeros((N ** 3, 2))
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                r = (x0 - dx) + N * (y0 - dy) + N * N * (z0 - dz)
                expect[r] = W[:, 0, t]
    assert np.array_equal(y, expect)


def test_corner_impulse_zero_padding():
    N = 5
    W = np.ones((1, 1, 27))
    x = np.zeros(N ** 3)
    x[0] = 1.0                       # corner voxel
    y = oracle.conv3d_fwd(N, W, x).reshape(-1)
    nz = np.flatnonzero(y)
    # only the 2 x 2 x 2 block of voxels within one step of the corner sees it
    got = sorted((r % N, (r // N) % N, r // (N * N)) for r in nz)
    assert got == sorted((a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1))
    assert np.all(y[nz] == 1.0)


@pytest.mark.parametrize("cin,cout", [(1, 16), (16, 16), (16, 1), (3, 5)])
def test_dgrad_is_adjoint(cin, cout):
    N = 6
    rng = np.random.default_rng(5 * cin + cout)
    W = rng.standard_normal((cout, cin, 27))
    x = rng.standard_normal((N ** 3, cin))
    g = rng.standard_normal((N ** 3, cout))
    lhs = np.sum(oracle.conv3d_fwd(N, W, x) * g)
    rhs = np.sum(x * oracle.conv3d_dgrad(N, W, g))
    assert abs(lhs - rhs) <= 1e-10 * (1 + abs(lhs))


@pytest.mark.parametrize("cin,cout", [(1, 16), (16, 16), (16, 1)])
def test_wgrad_is_derivative_in_weights(cin, cout):
    # the layer is linear in W: <dW, V> = <g, conv_V(x)> for any direction V
    N = 6
    rng = np.random.default_rng(17 * cin + cout)
    x = rng.standard_normal((N ** 3, cin))
    g = rng.standard_normal((N ** 3, cout))
    V = rng.standard_normal((cout, cin, 27))
    dW = oracle.conv3d_wgrad(N, g, x, cin, cout)
    assert dW.shape == (cout, cin, 27)
    lhs = np.sum(dW * V)
    rhs = np.sum(g * oracle.conv3d_fwd(N, V, x))
    assert abs(lhs - rhs) <= 1e-10 * (1 + abs(lhs))


def _rand_weights(rng, scale=1.0):
    return [scale * rng.standard_normal((co, ci, 27)) / np.sqrt(27 * ci)
            for ci, co in oracle.CNN_LAYERS]


def test_forward_matches_scipy_network():
    N = 6
    rng = np.random.default_rng(3)
    Ws = _rand_weights(rng, 2.0)
    x = rng.standard_normal(N ** 3)
    a = x.reshape(-1, 1)
    for l, W in enumerate(Ws):
        a = _scipy_conv(N, W, a)
        if l < 3:
            a = np.maximum(a, 0.0)
    y = oracle.cnn_forward(N, Ws, x)[-1]
    assert np.allclose(y, a, rtol=1e-12, atol=1e-12)


def test_positive_homogeneity():
    # bias-free ReLU network: f(c x) = c f(x) for c > 0
    N = 6
    rng = np.random.default_rng(4)
    Ws = _rand_weights(rng, 2.0)
    x = rng.standard_normal(N ** 3)
    y1 = oracle.cnn_forward(N, Ws, x)[-1]
    y3 = oracle.cnn_forward(N, Ws, 3.0 * x)[-1]
    assert np.allclose(y3, 3.0 * y1, rtol=1e-12, atol=1e-12)
    assert np.abs(y1).max() > 0


def test_zero_network_loss_is_one():
    N = 4
    rng = np.random.default_rng(6)
    Ws = [np.zeros((co, ci, 27)) for ci, co in oracle.CNN_LAYERS]
    xs = [rng.standard_normal(N ** 3) for _ in range(2)]
    ts = [rng.standard_normal(N ** 3) for _ in range(2)]
    loss, grads = oracle.cnn_loss_and_grads(N, Ws, xs, ts)
    assert loss == pytest.approx(1.0, abs=1e-15)


def test_loss_gradient_central_differences():
    N = 4
    rng = np.random.default_rng(8)
    Ws = _rand_weights(rng, 2.0)
    xs = [rng.standard_normal(N ** 3) for _ in range(2)]
    ts = [rng.standard_normal(N ** 3) for _ in range(2)]
    loss, grads = oracle.cnn_loss_and_grads(N, Ws, xs, ts)
    h = 1e-6
    checked = 0
    for l in range(4):
        flat = Ws[l].reshape(-1)
        for k in rng.choice(flat.size, 6, replace=False):
            Wp = [W.copy() for W in Ws]
            Wm = [W.copy() for W in Ws]
            Wp[l].reshape(-1)[k] += h
            Wm[l].reshape(-1)[k] -= h
            lp, _ = oracle.cnn_loss_and_grads(N, Wp, xs, ts)
            lm, _ = oracle.cnn_loss_and_grads(N, Wm, xs, ts)
            fd = (lp - lm) / (2 * h)
            an = grads[l].reshape(-1)[k]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (l, k, fd, an)
            checked += 1
    assert checked == 24


def test_bf16_known_values():
    one = 1.0
    cases = [
        (1.0, 1.0),
        (1.0 + 2.0 ** -8, 1.0),                      # tie, even mantissa below
        (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),      # tie, even mantissa above
        (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),
        (-(1.0 + 2.0 ** -8 + 2.0 ** -20), -(1.0 + 2.0 ** -7)),
        (0.0, 0.0),
        (3.0, 3.0),
    ]
    for v, e in cases:
        assert oracle.bf16(np.array([v]))[0] == e, v
    assert oracle.lib().orc_bf16_round(one + 2.0 ** -8) == 1.0


def test_bf16_matches_torch():
    rng = np.random.default_rng(9)
    a = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        [np.inf, -np.inf, 0.0, -0.0]]).astype(np.float32)
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    got = oracle.bf16(a)
    assert np.array_equal(got, ref)
    got_c = np.array([oracle.lib().orc_bf16_round(float(v)) for v in a[:2000]])
    assert np.array_equal(got_c, ref[:2000])


def test_adam_first_step_closed_form():
    # after one step the bias-corrected moments are g and g^2 exactly:
    # w1 = w0 - lr g / (|g| + eps)
    rng = np.random.default_rng(12)
    w = rng.standard_normal(50)
    g = rng.standard_normal(50) * 10.0 ** rng.integers(-3, 3, 50)
    m = np.zeros(50)
    v = np.zeros(50)
    w1 = oracle.adam_step(w, g, m, v, 1, lr=1e-3)
    assert np.allclose(w1, w - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-13, atol=1e-15)


def test_adam_constant_gradient_limit():
    # with a constant gradient the corrected moments stay g and g^2 at every step
    g = np.array([2.0, -0.5, 1e-3])
    w = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    for t in range(1, 51):
        w = oracle.adam_step(w, g, m, v, t, lr=0.01)
    assert np.allclose(w, -50 * 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-10)


def _nonsym_csr(n, seed):
    """Nonsymmetric diagonally dominant sparse matrix (CSR arrays)."""
    rng = np.random.default_rng(seed)
    A = np.diag(4.0 + rng.uniform(0.0, 1.0, n))
    for i in range(n - 1):
        A[i, i + 1] = -1.0 + 0.6 * rng.uniform(-1.0, 1.0)
        A[i + 1, i] = -1.0 - 0.6 * rng.uniform(-1.0, 1.0)
    for i in range(n - 5):
        A[i, i + 5] = 0.5 * rng.uniform(-1.0, 1.0)
    rows, cols = np.nonzero(A)
    rp = np.searchsorted(rows, np.arange(n + 1)).astype(np.int32)
    return rp, cols.astype(np.int32), A[rows, cols]


def test_residual_loss_gradient_central_differences():
    N = 4
    rng = np.random.default_rng(9)
    Ws = _rand_weights(rng, 2.0)
    A = _nonsym_csr(N ** 3, 10)
    xs = [rng.standard_normal(N ** 3) for _ in range(2)]
    loss, grads = oracle.cnn_residual_loss_and_grads(N, Ws, xs, A)
    h = 1e-6
    for l in range(4):
        flat = Ws[l].reshape(-1)
        for k in rng.choice(flat.size, 6, replace=False):
            Wp = [W.copy() for W in Ws]
            Wm = [W.copy() for W in Ws]
            Wp[l].reshape(-1)[k] += h
            Wm[l].reshape(-1)[k] -= h
            lp, _ = oracle.cnn_residual_loss_and_grads(N, Wp, xs, A)
            lm, _ = oracle.cnn_residual_loss_and_grads(N, Wm, xs, A)
            fd = (lp - lm) / (2 * h)
            an = grads[l].reshape(-1)[k]
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (l, k, fd, an)


def test_residual_loss_with_identity_is_solution_loss():
    # A = I: ||x - f(x)||^2 / ||x||^2 is the solution loss with target t = x
    N = 5
    n = N ** 3
    rng = np.random.default_rng(12)
    Ws = _rand_weights(rng, 2.0)
    I = (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    xs = [rng.standard_normal(n) for _ in range(3)]
    lr, gr = oracle.cnn_residual_loss_and_grads(N, Ws, xs, I)
    ls, gs = oracle.cnn_loss_and_grads(N, Ws, xs, xs)
    assert lr == pytest.approx(ls, rel=1e-13)
    for a, b in zip(gr, gs):
        assert np.allclose(a, b, rtol=1e-12, atol=1e-14 * np.abs(b).max())


def test_residual_loss_of_zero_network_is_one():
    N = 4
    rng = np.random.default_rng(13)
    Ws = [np.zeros((co, ci, 27)) for ci, co in oracle.CNN_LAYERS]
    xs = [rng.standard_normal(N ** 3) for _ in range(2)]
    loss, _ = oracle.cnn_residual_loss_and_grads(N, Ws, xs, _nonsym_csr(N ** 3, 14))
    assert loss == pytest.approx(1.0, abs=1e-15)


def test_output_voxel_depends_only_on_its_9cube():
    # four 3^3 layers without bias: an output voxel sees the inputs within 4
    # cells, so the forward over a 9^3 patch (aligned to the volume's faces
    # within 4 cells of them, where both apply the same zero padding) gives
    # the full volume's output there; the full-size GPU test relies on this
    N = 20
    rng = np.random.default_rng(20)
    Ws = [oracle.bf16(rng.standard_normal((co, ci, 27)) / np.sqrt(27 * ci))
          for ci, co in oracle.CNN_LAYERS]
    x = rng.standard_normal(N ** 3)
    full = oracle.cnn_forward(N, Ws, x, quantize=True)[-1].reshape(N, N, N)
    vol = x.reshape(N, N, N)
    pts = [(0, 0, 0), (19, 19, 19), (0, 10, 19), (3, 4, 16), (10, 10, 10), (4, 15, 2),
           (19, 0, 7), (5, 5, 5), (14, 14, 14)]
    for pt in pts:
        lo = [min(max(c - 4, 0), N - 9) for c in pt]
        patch = vol[lo[0]:lo[0] + 9, lo[1]:lo[1] + 9, lo[2]:lo[2] + 9]
        y = oracle.cnn_forward(9, Ws, np.ascontiguousarray(patch).reshape(-1),
                               quantize=True)[-1].reshape(9, 9, 9)
        got = y[pt[0] - lo[0], pt[1] - lo[1], pt[2] - lo[2]]
        assert got == full[pt], (pt, got, full[pt])
    # a 7^3 patch (too small) does not reproduce an interior voxel
    pt = (10, 10, 10)
    patch = vol[7:14, 7:14, 7:14]
    y = oracle.cnn_forward(7, Ws, np.ascontiguousarray(patch).reshape(-1),
                           quantize=True)[-1].reshape(7, 7, 7)
    assert y[3, 3, 3] != full[pt]
