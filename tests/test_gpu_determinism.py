"""GPU: repeated solves are bitwise reproducible.

Every reduction on the device has a fixed order (block-local trees, then the
block partials summed in block order), and no kernel uses atomics on values,
so the same solve on the same handle -- and on a second handle forced to the
same launch shapes -- must give bitwise identical solutions and statistics.
"""
import sys

import numpy as np
import pytest

from paper_2103_07329_amd import inputs

pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def jump24(orc):
    p = inputs.jump7(24, inputs.jump_kappa(24, np.random.default_rng(77)))
    return p, orc.Hierarchy(*p.csr())


def _solve(torch, S, B):
    Bd = torch.from_numpy(B).cuda()
    Xd = torch.zeros_like(Bd)
    rc, st = S.solve(Bd, Xd, tol=1e-9, check=False)
    torch.cuda.synchronize()
    return rc, Xd.cpu().numpy(), st


CASES = [
    dict(method=0, smoother=1, precision=0, m=16),
    dict(method=1, smoother=0, precision=1, index_bits=16, m=8),
    dict(method=2, smoother=2, precision=0, m=4),
    dict(method=0, smoother=2, precision=1, m=5),
    dict(method=3, smoother=1, precision=0, m=16),             # pipelined BiCGStab
    dict(method=0, smoother=1, precision=0, merged=2, m=8),    # CG, p pass in the SpMM
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_repeat_solves_bitwise(torch, xm, jump24, case):
    kw = dict(CASES[case])
    m = kw.pop("m")
    _say(f"[determinism] jump24 {kw} m={m}")
    p, H = jump24
    B = inputs.uniform_rhs(p.n, m, 90 + case)
    S = xm.Solver(H.export(), **kw)
    runs = [_solve(torch, S, B) for _ in range(3)]
    # a second handle with the first one's launch shapes
    S2 = xm.Solver(H.export(), **kw)
    mp = 1 << (m - 1).bit_length()
    S2.autotune(mp, enable=False)
    S2.set_tuning(mp, S.tuning(mp))
    runs.append(_solve(torch, S2, B))
    S.close()
    S2.close()
    rc0, X0, st0 = runs[0]
    for rc, X, st in runs[1:]:
        assert rc == rc0
        assert np.array_equal(X, X0)
        for k in ("iters", "relres", "true_relres", "restarts"):
            assert np.array_equal(st[k], st0[k]), k
