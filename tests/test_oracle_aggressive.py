"""Pins of the oracle's aggressive coarsening and multipass interpolation
(the paper's mg_agg_num_levels / mg_num_paths, Section 2.4), CPU only.

* The 1D model problem, worked out by hand from the definitions
  (tests/golden/agg_1d_multipass.txt): the coarse points and every row of P.
* The C/F split against a brute force from the definitions: the first RS
  pass (recomputed weights, tests/test_oracle_pins.py), the distance-two
  strength among its C points by counting paths with dense matrix products,
  and an RS pass on that strength written out the same way.
* Multipass interpolation against a dense brute force of the passes.
* The hierarchy's invariants: R = P^T, A_c = P^T A P, A_c SPD, C rows unit
  rows, and an AMG-preconditioned CG that reaches the dense solution.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2103_07329_amd import inputs
from test_oracle_pins import (_lognormal_graph_laplacian, _random_mixed_sign,
                              _rs_bruteforce, dense, lap1d)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    d = {}
    with open(os.path.join(GOLDEN, "agg_1d_multipass.txt")) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split(":", 1)
                d[k.strip()] = v.split()
    return d


def test_aggressive_multipass_1d_worked_example(orc):
    g = _golden()
    n = int(g["n"][0])
    rp, ci, v = lap1d(n)
    st = orc.agg_split(rp, ci, v)
    assert list(np.nonzero(st == 1)[0]) == [int(x) for x in g["cpoints"]]
    H = orc.Hierarchy(rp, ci, v, max_coarse=4, agg_levels=1)
    assert H.sizes() == [n, len(g["cpoints"])]
    P = dense(*H.P(0)[:3], H.P(0)[3])
    Pg = np.zeros_like(P)
    for i in range(n):
        for ent in g[f"P{i}"]:
            c, w = ent.split(":")
            Pg[i, int(c)] = float(w)
    assert np.array_equal(P, Pg)


def _strength_sets(A, theta=0.25):
    n = A.shape[0]
    S = []
    for i in range(n):
        off = [-A[i, j] for j in range(n) if j != i]
        mx = max(off) if off else 0.0
        S.append({j for j in range(n) if j != i and mx > 0 and -A[i, j] >= theta * mx})
    return S


def _rs_on_sets(S):
    """First RS pass on an explicit strength relation S (list of sets),
    weights |S^T n U| + 2 |S^T n F| recomputed before every pick."""
    n = len(S)
    ST = [{j for j in range(n) if i in S[j]} for i in range(n)]
    state = ["U"] * n
    while "U" in state:
        best, bi = -1, -1
        for i in range(n):
            if state[i] != "U":
                continue
            lam = sum(1 for j in ST[i] if state[j] == "U") + \
                2 * sum(1 for j in ST[i] if state[j] == "F")
            if lam > best:
                best, bi = lam, i
        state[bi] = "C"
        for j in ST[bi]:
            if state[j] == "U":
                state[j] = "F"
    return state


def _agg_bruteforce(A, num_paths):
    S = _strength_sets(A)
    n = A.shape[0]
    Sb = np.zeros((n, n), np.int64)
    for i in range(n):
        for j in S[i]:
            Sb[i, j] = 1
    paths = Sb + Sb @ Sb            # paths of length one and two
    first = _rs_bruteforce(A)
    C1 = np.nonzero(first == 1)[0]
    S2 = [{b for b in range(len(C1)) if b != a and paths[C1[a], C1[b]] >= num_paths}
          for a in range(len(C1))]
    st2 = _rs_on_sets(S2)
    out = first.copy()
    for a, i in enumerate(C1):
        out[i] = 1 if st2[a] == "C" else 2
    return out


def _problem(k):
    """0: jump coefficients; 1: anisotropic; 2: random graph Laplacian;
    3, 5: log-normal weights (strongly asymmetric strength, so C points of
    the first pass depend on each other directly: with one path, and with
    two, the direct path decides some distance-two connections); 4:
    positive off-diagonal couplings."""
    rng = np.random.default_rng(21 + k)
    if k == 3:
        return _lognormal_graph_laplacian(60, 0, 0.06, 2.0)
    if k == 5:
        return _lognormal_graph_laplacian(60, 6, 0.06, 2.0)
    if k == 4:
        return _random_mixed_sign(130, 12)
    if k == 0:
        return inputs.jump7(6, inputs.jump_kappa(6, rng, block=2)).csr()
    if k == 1:
        return inputs.anisotropic7(6).csr()
    n = 140
    W = sp.random(n, n, density=0.05, random_state=rng) * 10
    W = sp.triu(W, 1)
    W = (W + W.T).tocsr()
    L = sp.csr_matrix(sp.diags(np.asarray(W.sum(axis=1)).ravel() + 0.1) - W)
    L.sort_indices()
    return L.indptr.astype(np.int32), L.indices.astype(np.int32), L.data.astype(np.float64)


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4, 5])
@pytest.mark.parametrize("num_paths", [1, 2])
def test_aggressive_split_bruteforce(orc, k, num_paths):
    rp, ci, v = _problem(k)
    A = dense(rp, ci, v)
    st = orc.agg_split(rp, ci, v, num_paths=num_paths)
    assert np.array_equal(st, _agg_bruteforce(A, num_paths))
    # the coarse grid is a subset of the first pass's
    assert np.all(orc.rs_split(rp, ci, v)[st == 1] == 1)


def _multipass_bruteforce(A, state, theta=0.25):
    """Dense multipass interpolation from its definition."""
    n = A.shape[0]
    S = _strength_sets(A, theta)
    C = [i for i in range(n) if state[i] == 1]
    cidx = {c: k for k, c in enumerate(C)}
    P = np.zeros((n, len(C)))
    level = {c: 0 for c in C}
    for c in C:
        P[c, cidx[c]] = 1.0
    p = 0
    while True:
        p += 1
        now = [i for i in range(n) if i not in level and any(level.get(j, p) < p for j in S[i])]
        if not now:
            break
        for i in now:
            level[i] = p
        for i in now:
            Pi = [j for j in S[i] if level.get(j, p) < p]
            off = [j for j in range(n) if j != i and A[i, j] != 0]
            neg_n = sum(A[i, j] for j in off if A[i, j] < 0)
            pos_n = sum(A[i, j] for j in off if A[i, j] > 0)
            neg_p = sum(A[i, j] for j in Pi if A[i, j] < 0)
            pos_p = sum(A[i, j] for j in Pi if A[i, j] > 0)
            d = A[i, i] + (pos_n if pos_p == 0 else 0.0)
            al = neg_n / neg_p if neg_p != 0 else 0.0
            be = pos_n / pos_p if pos_p != 0 else 0.0
            for j in Pi:
                w = -(al if A[i, j] < 0 else be) * A[i, j] / d
                P[i] += w * P[j]
    return P


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
@pytest.mark.parametrize("num_paths", [1, 2])
def test_multipass_bruteforce(orc, k, num_paths):
    rp, ci, v = _problem(k)
    A = dense(rp, ci, v)
    H = orc.Hierarchy(rp, ci, v, max_coarse=10, agg_levels=1, num_paths=num_paths)
    P = dense(*H.P(0)[:3], H.P(0)[3])
    Pb = _multipass_bruteforce(A, H.cf(0))
    assert np.allclose(P, Pb, rtol=0, atol=1e-14 * np.abs(Pb).max())
    # the stored pattern holds exactly the nonzero entries
    assert np.count_nonzero(P) == len(H.P(0)[1])


@pytest.mark.parametrize("k", [0, 1, 2])
@pytest.mark.parametrize("agg,num_paths", [(1, 1), (2, 2)])
def test_aggressive_hierarchy_invariants(orc, k, agg, num_paths):
    rp, ci, v = _problem(k)
    H = orc.Hierarchy(rp, ci, v, max_coarse=8, agg_levels=agg, num_paths=num_paths)
    for l in range(H.nlev - 1):
        A = dense(*H.A(l)[:3])
        P = dense(*H.P(l)[:3], H.P(l)[3])
        R = dense(*H.R(l)[:3], H.R(l)[3])
        Ac = dense(*H.A(l + 1)[:3])
        assert np.array_equal(R, P.T)
        ref = P.T @ A @ P
        assert np.allclose(Ac, ref, rtol=0, atol=1e-13 * np.abs(ref).max())
        assert np.linalg.eigvalsh(0.5 * (Ac + Ac.T)).min() > 0
        cf = H.cf(l)
        cidx = np.cumsum(cf == 1) - 1
        for i in np.nonzero(cf == 1)[0]:
            e = np.zeros(P.shape[1]); e[cidx[i]] = 1.0
            assert np.array_equal(P[i], e)
    A0 = dense(rp, ci, v)
    B = inputs.uniform_rhs(A0.shape[0], 3, 5)
    for smoother in (0, 1, 2):
        X, st, rc = H.solve(B, smoother=smoother, tol=1e-12)
        assert rc == orc.OK
        Xd = np.linalg.solve(A0, B)
        assert np.allclose(X, Xd, rtol=0, atol=1e-9 * np.abs(Xd).max())


def test_aggressive_lowers_complexity(orc):
    p = inputs.poisson7(16)
    std = orc.Hierarchy(*p.csr())
    agg = orc.Hierarchy(*p.csr(), agg_levels=1)
    nnz = lambda H: sum(len(H.A(l)[1]) for l in range(H.nlev))
    assert nnz(agg) < nnz(std) and sum(agg.sizes()) < sum(std.sizes())
    # one path: at least as aggressive as two paths
    two = orc.Hierarchy(*p.csr(), agg_levels=1, num_paths=2)
    assert agg.sizes()[1] <= two.sizes()[1]
