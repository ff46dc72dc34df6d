"""GPU parity of the warm-start CNN kernels (through the C ABI) against the
CPU oracle on the same BF16-rounded operands.

Bounds: a device layer output is the FP32 sum of the products, rounded to
BF16 where stored.  Against the oracle's exact sum z it therefore differs
by at most half a BF16 unit (<= 2^-8 |z|) plus the FP32 accumulation error
(<= k 2^-24 sum |w x| with k terms; k <= 27 * 16 + 1), so each check uses
|dev - z| <= 2^-8 |z| + 4e-5 sum |w x|, with sum |w x| computed by the
oracle from |W| and |x|.  Weight gradients are FP32 sums over n voxels
(per-block partials summed in block order): |dev - dW| <= 1e-5 sum |g x|.
A full forward/backward pass rounds every stored activation, so a rounding
that goes the other way on one side can move a value by one BF16 unit
downstream: there the check is on norms (loss 1e-5, gradients 2e-3
relative; 2e-3 for the warm-start output), all far below what a wrong tap,
channel or mask would give.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2103_07329_amd import inputs

pytestmark = pytest.mark.gpu

U = 2.0 ** -8


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.fixture(scope="module")
def xm():
    from paper_2103_07329_amd import xamg
    xamg.lib()
    return xamg


def _weights(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return [(scale * rng.standard_normal((co, ci, 27)) / np.sqrt(27 * ci)).astype(np.float32)
            for ci, co in oracle.CNN_LAYERS]


def _bf16_dev(torch, a):
    """BF16-representable float64/32 array -> torch.bfloat16 CUDA tensor (exact)."""
    t = torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()
    return t.to(torch.bfloat16).contiguous()


def _f32_dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


def _host(t):
    return t.float().cpu().numpy().astype(np.float64)


def _act(rng, n, c, zero_frac=0.3):
    a = np.abs(rng.standard_normal((n, c)))
    a[rng.random((n, c)) < zero_frac] = 0.0
    return oracle.bf16(a)


def _check_bound(dev, z, absmag, what):
    err = np.abs(dev - z)
    lim = U * np.abs(z) + 4e-5 * absmag + 1e-30
    worst = float((err / lim).max())
    _say(f"  {what}: max err {err.max():.3e}, worst err/bound {worst:.3f}")
    assert worst <= 1.0, what


@pytest.mark.parametrize("N", [16, 32])
@pytest.mark.parametrize("layer", [1, 2, 3, 4])
def test_layer_forward(torch, xm, N, layer):
    _say(f"[cnn fwd] N={N} layer={layer}")
    n = N ** 3
    Ws = _weights(100 + layer, 2.0)
    net = xm.Cnn(N, xm.join_weights(Ws))
    Wq = oracle.bf16(Ws[layer - 1])
    cin, cout = oracle.CNN_LAYERS[layer - 1]
    rng = np.random.default_rng(7 * N + layer)
    x = oracle.bf16(rng.standard_normal((n, 1))) if layer == 1 else _act(rng, n, cin)
    z = oracle.conv3d_fwd(N, Wq, x)
    absmag = oracle.conv3d_fwd(N, np.abs(Wq), np.abs(x))
    xd = _bf16_dev(torch, x)
    if layer == 4:
        out = torch.full((n,), float("nan"), dtype=torch.float32, device="cuda")
    else:
        out = torch.full((n, cout), float("nan"), dtype=torch.bfloat16, device="cuda")
    net.layer(layer, 0, xd, None, out)
    got = _host(out).reshape(n, cout)
    if layer < 4:
        z = np.maximum(z, 0.0)
    _check_bound(got, z, absmag, f"layer {layer} forward")
    net.close()


@pytest.mark.parametrize("N", [16, 32])
@pytest.mark.parametrize("layer", [2, 3, 4])
def test_layer_input_gradient(torch, xm, N, layer):
    _say(f"[cnn dgrad] N={N} layer={layer}")
    n = N ** 3
    Ws = _weights(200 + layer, 2.0)
    net = xm.Cnn(N, xm.join_weights(Ws))
    Wq = oracle.bf16(Ws[layer - 1])
    cin, cout = oracle.CNN_LAYERS[layer - 1]
    rng = np.random.default_rng(11 * N + layer)
    mask = _act(rng, n, cin, zero_frac=0.4)
    if layer == 4:
        g = rng.standard_normal((n, 1)).astype(np.float32).astype(np.float64)
        gd = _f32_dev(torch, g.reshape(-1))
    else:
        g = oracle.bf16(rng.standard_normal((n, cout)))
        gd = _bf16_dev(torch, g)
    d = oracle.conv3d_dgrad(N, Wq, g) * (mask > 0)
    absmag = oracle.conv3d_dgrad(N, np.abs(Wq), np.abs(g))
    out = torch.full((n, cin), float("nan"), dtype=torch.bfloat16, device="cuda")
    net.layer(layer, 1, gd, _bf16_dev(torch, mask), out)
    got = _host(out)
    assert np.all(got[mask == 0] == 0.0)
    _check_bound(got, d, absmag, f"layer {layer} input gradient")
    net.close()


@pytest.mark.parametrize("N", [16, 32])
@pytest.mark.parametrize("layer", [1, 2, 3, 4])
def test_layer_weight_gradient(torch, xm, N, layer):
    _say(f"[cnn wgrad] N={N} layer={layer}")
    n = N ** 3
    Ws = _weights(300 + layer)
    net = xm.Cnn(N, xm.join_weights(Ws))
    cin, cout = oracle.CNN_LAYERS[layer - 1]
    rng = np.random.default_rng(13 * N + layer)
    x = oracle.bf16(rng.standard_normal((n, 1))) if layer == 1 else _act(rng, n, cin)
    if layer == 4:
        g = rng.standard_normal((n, 1)).astype(np.float32).astype(np.float64)
        gd = _f32_dev(torch, g.reshape(-1))
    else:
        g = oracle.bf16(rng.standard_normal((n, cout)))
        gd = _bf16_dev(torch, g)
    dW = oracle.conv3d_wgrad(N, g, x, cin, cout)
    absmag = oracle.conv3d_wgrad(N, np.abs(g), np.abs(x), cin, cout)
    dummy = torch.empty(1, device="cuda")
    net.layer(layer, 2, gd, _bf16_dev(torch, x), dummy)
    grads = xm.split_weights(net.grads().astype(np.float64))
    for l in range(4):
        if l != layer - 1:
            assert np.all(grads[l] == 0.0)
    err = np.abs(grads[layer - 1] - dW)
    worst = float((err / (1e-5 * absmag + 1e-30)).max())
    _say(f"  max err {err.max():.3e}, worst err/bound {worst:.3f}")
    assert worst <= 1.0
    net.close()


def test_full_pass_loss_and_gradients(torch, xm):
    N, S = 16, 3
    n = N ** 3
    _say(f"[cnn pass] N={N} S={S}")
    Ws = _weights(400, 2.0)
    net = xm.Cnn(N, xm.join_weights(Ws))
    rng = np.random.default_rng(41)
    xs = [rng.standard_normal(n).astype(np.float32) for _ in range(S)]
    ts = [rng.standard_normal(n).astype(np.float32) for _ in range(S)]
    loss_o, grads_o = oracle.cnn_loss_and_grads(N, [oracle.bf16(W) for W in Ws], xs, ts,
                                                quantize=True)
    xd = _f32_dev(torch, np.stack(xs))
    td = _f32_dev(torch, np.stack(ts))
    loss_d = net.loss_and_grads(xd, td)
    grads_d = xm.split_weights(net.grads().astype(np.float64))
    _say(f"  loss dev {loss_d:.8f} oracle {loss_o:.8f}")
    assert abs(loss_d - loss_o) <= 1e-5 * loss_o
    for l in range(4):
        rel = np.linalg.norm(grads_d[l] - grads_o[l]) / np.linalg.norm(grads_o[l])
        _say(f"  layer {l + 1} gradient rel err {rel:.3e}")
        assert rel <= 2e-3
    # forward output of the same pass
    y = net.forward(xd)
    yo = oracle.cnn_forward(N, [oracle.bf16(W) for W in Ws], xs[0], quantize=True)[-1].reshape(-1)
    rel = np.linalg.norm(_host(y)[0] - yo) / np.linalg.norm(yo)
    _say(f"  forward rel err {rel:.3e}")
    assert rel <= 2e-3
    net.close()


def test_residual_pass_loss_and_gradients(torch, xm):
    """The residual loss ||x - A f(x)||^2 / ||x||^2 with A the solver's
    finest operator (7-point Poisson, stored padded to 7 entries a row)
    against the oracle's BF16-rounded network."""
    N, S = 16, 2
    n = N ** 3
    _say(f"[cnn residual pass] N={N} S={S}")
    Ws = _weights(300)
    net = xm.Cnn(N, xm.join_weights(Ws))
    prob = inputs.poisson7(N)
    solver = xm.Solver(xm.HostHierarchy(*prob.csr()))
    rng = np.random.default_rng(43)
    xs = [rng.standard_normal(n).astype(np.float32) for _ in range(S)]
    loss_o, grads_o = oracle.cnn_residual_loss_and_grads(N, [oracle.bf16(W) for W in Ws], xs,
                                                         prob.csr(), quantize=True)
    loss_d = net.residual_loss_and_grads(_f32_dev(torch, np.stack(xs)), solver)
    grads_d = xm.split_weights(net.grads().astype(np.float64))
    _say(f"  loss dev {loss_d:.8f} oracle {loss_o:.8f}")
    assert abs(loss_d - loss_o) <= 1e-5 * loss_o
    for l in range(4):
        rel = np.linalg.norm(grads_d[l] - grads_o[l]) / np.linalg.norm(grads_o[l])
        _say(f"  layer {l + 1} gradient rel err {rel:.3e}")
        assert rel <= 2e-3
    with pytest.raises(xm.XamgError):   # operator of another grid size
        other = xm.Solver(xm.HostHierarchy(*inputs.poisson7(8).csr()))
        try:
            net.residual_loss_and_grads(_f32_dev(torch, np.stack(xs)), other)
        finally:
            other.close()
    solver.close()
    net.close()


def test_adam_matches_oracle(torch, xm):
    # gradient buffer from one weight-gradient call (matches the oracle to
    # FP32 accumulation), then two Adam steps on it
    N = 16
    n = N ** 3
    _say(f"[cnn adam] N={N}")
    Ws = _weights(500)
    w0 = xm.join_weights(Ws).astype(np.float64)
    net = xm.Cnn(N, w0)
    rng = np.random.default_rng(51)
    x = _act(rng, n, 16)
    g = oracle.bf16(rng.standard_normal((n, 16)))
    dummy = torch.empty(1, device="cuda")
    net.layer(3, 2, _bf16_dev(torch, g), _bf16_dev(torch, x), dummy)
    G = np.zeros_like(w0)
    off = 16 * 27 + 16 * 16 * 27
    G[off:off + 16 * 16 * 27] = oracle.conv3d_wgrad(N, g, x, 16, 16).reshape(-1)
    m = np.zeros_like(w0)
    v = np.zeros_like(w0)
    w = w0.copy()
    for t in (1, 2):
        net.adam(1e-3, 0.9, 0.999, 1e-8)
        w = oracle.adam_step(w, G, m, v, t, lr=1e-3)
        got = net.weights().astype(np.float64)
        err = np.abs(got - w)
        _say(f"  step {t}: max err {err.max():.3e}")
        assert np.all(err <= 2e-8 + 2.0 ** -23 * np.abs(w))
        assert np.array_equal(got[:off], w0[:off].astype(np.float32))
    net.close()


def _passthrough_weights(c):
    """f(x) = c x exactly: channel 0 carries relu(x), channel 1 relu(-x)."""
    Ws = [np.zeros((co, ci, 27), np.float32) for ci, co in oracle.CNN_LAYERS]
    ctr = 13
    Ws[0][0, 0, ctr] = 1.0
    Ws[0][1, 0, ctr] = -1.0
    for l in (1, 2):
        Ws[l][0, 0, ctr] = 1.0
        Ws[l][1, 1, ctr] = 1.0
    Ws[3][0, 0, ctr] = c
    Ws[3][0, 1, ctr] = -c
    return Ws


def _oracle_warmstart(N, Ws, B):
    n, m = B.shape
    X0 = np.zeros_like(B)
    for j in range(m):
        s = np.sqrt(B[:, j] @ B[:, j] / n)
        if s == 0:
            continue
        y = oracle.cnn_forward(N, [oracle.bf16(W) for W in Ws], (B[:, j] / s).astype(np.float32),
                               quantize=True)[-1].reshape(-1)
        X0[:, j] = s * y
    return X0


def test_warmstart_fallback_rule(torch, xm, orc):
    N, m = 16, 6
    n = N ** 3
    _say(f"[warmstart fallback] N={N} m={m}")
    p = inputs.poisson7(N)
    H = orc.Hierarchy(*p.csr())
    S = xm.Solver(H.export())
    B = inputs.gaussian_rhs(N, m, 1234)
    B[:, 3] = 0.0
    from scipy.sparse import csr_matrix
    A = csr_matrix((p.val, p.col, p.rowptr), shape=(n, n))
    for c, name in ((1.0 / 6.0, "jacobi-like"), (-1.0 / 6.0, "negated")):
        Ws = _passthrough_weights(c)
        net = xm.Cnn(N, xm.join_weights(Ws))
        Bd = torch.from_numpy(B).cuda()
        X0d = torch.full((n, m), np.nan, dtype=torch.float64, device="cuda")
        fb = net.warmstart(Bd, X0d, S)
        X0 = X0d.cpu().numpy()
        X0o = _oracle_warmstart(N, Ws, B)
        rn = np.linalg.norm(B - A @ X0o, axis=0)
        bn = np.linalg.norm(B, axis=0)
        expect = (~(rn < bn)).astype(np.int32)
        _say(f"  {name}: fallback dev {fb.tolist()} oracle {expect.tolist()}")
        assert np.array_equal(fb, expect)
        for j in range(m):
            if expect[j]:
                assert np.all(X0[:, j] == 0.0)
            else:
                rel = np.abs(X0[:, j] - X0o[:, j]).max() / np.abs(X0o[:, j]).max()
                assert rel <= 1e-6, (j, rel)
        net.close()
    S.close()


def test_warmstart_parity_and_homogeneity(torch, xm):
    N, m = 32, 4
    n = N ** 3
    _say(f"[warmstart parity] N={N} m={m}")
    Ws = _weights(600, 2.0)
    net = xm.Cnn(N, xm.join_weights(Ws))
    B = inputs.gaussian_rhs(N, m, 4321)
    Bd = torch.from_numpy(B).cuda()
    X0d = torch.zeros((n, m), dtype=torch.float64, device="cuda")
    fb = net.warmstart(Bd, X0d, None)
    assert np.all(fb == 0)
    X0 = X0d.cpu().numpy()
    X0o = _oracle_warmstart(N, Ws, B)
    for j in range(m):
        rel = np.linalg.norm(X0[:, j] - X0o[:, j]) / np.linalg.norm(X0o[:, j])
        _say(f"  column {j}: rel err {rel:.3e}")
        assert rel <= 2e-3
    # s(2b) = 2 s(b) and (2b) / s(2b) = b / s(b) exactly, so X0 doubles bit for bit
    X0d2 = torch.zeros_like(X0d)
    net.warmstart(Bd * 2.0, X0d2, None)
    assert torch.equal(X0d2, 2.0 * X0d)
    net.close()


def test_cnn_argument_errors(torch, xm):
    with pytest.raises(xm.XamgError):
        xm.Cnn(20, np.zeros(xm.CNN_PARAMS, np.float32))
    net = xm.Cnn(16, np.zeros(xm.CNN_PARAMS, np.float32))
    x = torch.zeros(16 ** 3, dtype=torch.bfloat16, device="cuda")
    with pytest.raises(xm.XamgError):
        net.layer(1, 1, x, x, x)          # no input gradient for layer 1
    with pytest.raises(xm.XamgError):
        net.layer(5, 0, x, None, x)
    xs = torch.zeros(16 ** 3 * 16 + 8, dtype=torch.bfloat16, device="cuda")[1:]
    with pytest.raises(xm.XamgError):
        net.layer(2, 0, xs, None, xs)     # 2-byte offset: not 16-byte aligned
    net.close()
