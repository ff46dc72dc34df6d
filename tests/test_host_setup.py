"""The library's host AMG setup against the oracle's (CPU only).

Both follow the same definitions (classical strength, first-pass RS with
lowest-index ties, direct interpolation, Galerkin; on aggressive levels a
second RS pass on the distance-two strength among the C points and
multipass interpolation), written independently:
C/F splits and sparsity patterns must agree exactly, values to rounding.
"""
import numpy as np
import pytest

from paper_2103_07329_amd import inputs


def _problems():
    rng = np.random.default_rng(2)
    return {
        "poisson16": inputs.poisson7(16),
        "aniso12": inputs.anisotropic7(12),
        "jump16": inputs.jump7(16, inputs.jump_kappa(16, rng)),
        "poisson32": inputs.poisson7(32),
    }


@pytest.fixture(scope="module")
def xm():
    from paper_2103_07329_amd import xamg
    try:
        xamg.lib()
    except OSError as e:
        pytest.fail(f"libxamg.so not built: {e}")
    return xamg


@pytest.mark.parametrize("name,agg,paths", [
    ("poisson16", 0, 1), ("aniso12", 0, 1), ("jump16", 0, 1), ("poisson32", 0, 1),
    ("poisson16", 1, 1), ("aniso12", 1, 2), ("jump16", 2, 1), ("poisson32", 2, 2)])
def test_setup_matches_oracle(orc, xm, name, agg, paths):
    """agg > 0: aggressive coarsening with multipass interpolation on the
    first agg levels, num_paths = paths."""
    p = _problems()[name]
    Ho = orc.Hierarchy(*p.csr(), agg_levels=agg, num_paths=paths)
    Hp = xm.HostHierarchy(*p.csr(), agg_levels=agg, num_paths=paths)
    assert Hp.nlev == Ho.nlev
    assert Hp.sizes() == Ho.sizes()
    for l in range(Ho.nlev - 1):
        assert np.array_equal(Hp.cf(l).astype(np.int32), Ho.cf(l))
        for which in ("A", "P", "R"):
            rp_o, ci_o, v_o, sh_o = getattr(Ho, which)(l)
            rp_p, ci_p, v_p, sh_p = getattr(Hp, which)(l)
            assert sh_o == sh_p
            assert np.array_equal(rp_o, rp_p), (which, l)
            assert np.array_equal(ci_o, ci_p), (which, l)
            scale = np.abs(v_o).max()
            assert np.allclose(v_p, v_o, rtol=0, atol=1e-12 * scale), (which, l)
        assert abs(Hp.lmax(l) - Ho.lmax(l)) <= 1e-10 * Ho.lmax(l)
    L = Ho.nlev - 1
    assert np.array_equal(Hp.A(L)[1], Ho.A(L)[1])
    assert np.allclose(Hp.A(L)[2], Ho.A(L)[2], rtol=0, atol=1e-12 * np.abs(Ho.A(L)[2]).max())


def test_setup_rejects_bad_csr(xm):
    p = inputs.poisson7(4)
    rp, ci, v = p.csr()
    bad = ci.copy()
    bad[3] = 10_000
    with pytest.raises(xm.XamgError) as e:
        xm.HostHierarchy(rp, bad, v)
    assert e.value.code == xm.EINVAL
    unsorted = ci.copy()
    unsorted[[0, 1]] = unsorted[[1, 0]]
    with pytest.raises(xm.XamgError):
        xm.HostHierarchy(rp, unsorted, v)
    nodiag = v.copy()
    nodiag[rp[5]:rp[6]][ci[rp[5]:rp[6]] == 5] = 0.0
    with pytest.raises(xm.XamgError):
        xm.HostHierarchy(rp, ci, nodiag)
    with pytest.raises(xm.XamgError) as e:
        xm.HostHierarchy(rp, ci, v, max_levels=2, max_coarse=2)
    assert e.value.code == xm.EBREAKDOWN
