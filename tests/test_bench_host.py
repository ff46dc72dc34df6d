"""Host-side arithmetic of bench.py (CPU only): the algorithmic byte counts
behind the reported rates, the lookup of committed PMC traffic, and the
one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_spmm_bytes_match_the_stated_table():
    # 7-point Poisson 128^3: nnz = 7 N^3 - 6 N^2; FP64 values, int32 indices
    N = 128
    n, nnz = N ** 3, 7 * N ** 3 - 6 * N ** 2
    assert nnz == 14581760
    mb = {m: bench.spmm_bytes(n, nnz, m) / 1e6 for m in (1, 2, 4, 8, 16, 32)}
    for m, want in {1: 216.9, 2: 250.5, 4: 317.6, 8: 451.8, 16: 720.2, 32: 1257.1}.items():
        assert abs(mb[m] - want) < 0.05, (m, mb[m])
    # Chebyshev pre-smoothing pass from zero: + D^-1, b read instead of x
    assert bench.presmooth_bytes(n, nnz, 16) == pytest.approx(
        bench.spmm_bytes(n, nnz, 16) + 8 * n)
    # Jacobi writes r as well
    assert bench.presmooth_bytes(n, nnz, 16, jacobi=True) == pytest.approx(
        bench.presmooth_bytes(n, nnz, 16) + 8 * n * 16)


class _Shape:
    """Level sizes and nonzero counts of a hierarchy (what the byte count reads)."""

    def __init__(self, sizes, nnzA, nnzP):
        self.sizes, self.nnzA, self.nnzP, self.nlev = sizes, nnzA, nnzP, len(sizes)


def test_pcg_iteration_bytes_two_levels_by_hand():
    # level 0: n0 rows, a0 nonzeros; P_0 with p0 nonzeros; level 1 coarsest (n1 rows)
    n0, a0, p0, n1, m = 1000, 6000, 1500, 10, 4
    S = _Shape([n0, n1], [a0, 50], [p0, 0])
    V0, V1 = n0 * m * 8, n1 * m * 8
    MA = a0 * 12 + 4 * (n0 + 1)
    MP = p0 * 12 + 4 * (n0 + 1)
    MR = p0 * 12 + 4 * (n1 + 1)
    d = n0 * 8
    cheb = ((MA + V0 + d + V0) + (MA + V0 + V0 + V0) + (MR + V0 + V1) + (MP + V1 + 2 * V0)
            + (MA + V0 + V0 + d + V0) + (MA + V0 + V0 + d + V0) + V0)      # + (b, z) dot
    coarse = n1 * n1 * 8 + 2 * V1
    # Krylov passes of the default CG form (merged = 1): q = A p; r -= a q
    # (r, q read, r written); x += a p_old with p = z + b p (p, z, x read;
    # p, x written)
    krylov = (a0 * 12 + 4 * (n0 + 1) + 2 * V0) + 3 * V0 + 5 * V0
    got = bench.pcg_iteration_bytes(S, m, chebyshev=True, mixed=False, flexible=False)
    assert got == pytest.approx(cheb + coarse + krylov)
    # standard form: x and r together (6 vectors), then p (3)
    got = bench.pcg_iteration_bytes(S, m, chebyshev=True, mixed=False, flexible=False, merged=0)
    assert got == pytest.approx(cheb + coarse + (a0 * 12 + 4 * (n0 + 1) + 2 * V0) + 9 * V0)
    # p pass inside the SpMM: z, p gathered, p', q written, x read and written
    got = bench.pcg_iteration_bytes(S, m, chebyshev=True, mixed=False, flexible=False, merged=2)
    assert got == pytest.approx(cheb + coarse + (a0 * 12 + 4 * (n0 + 1) + 6 * V0) + 3 * V0)
    jac = ((MA + V0 + d + 2 * V0) + (MR + V0 + V1) + (MP + V1 + 2 * V0)
           + (MA + V0 + V0 + d + V0))
    got = bench.pcg_iteration_bytes(S, m, chebyshev=False, mixed=False, flexible=False)
    assert got == pytest.approx(jac + coarse + krylov)
    # flexible CG also reads q in the last pass of level 0
    got = bench.pcg_iteration_bytes(S, m, chebyshev=False, mixed=False, flexible=True)
    assert got == pytest.approx(jac + coarse + krylov + V0)


def test_pcg_iteration_bytes_mixed_is_smaller():
    S = _Shape([4096, 512, 40], [28000, 9000, 1600], [6000, 900, 0])
    f64 = bench.pcg_iteration_bytes(S, 8, True, mixed=False, flexible=False)
    f32 = bench.pcg_iteration_bytes(S, 8, True, mixed=True, flexible=True)
    f16 = bench.pcg_iteration_bytes(S, 8, True, mixed=True, flexible=True,
                                    idx16=[(1.0, 1.0, 1.0)] * 2)
    assert f16 < f32 < f64


def test_stored_traffic_requires_the_current_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abc123")
    f = prof / "pmc_w_k.txt"
    f.write_text("# comment: ignored\nkernel: k\nkernel_source_sha: abc123\n"
                 "traffic_bytes_per_launch: 1234.5\n")
    assert bench.stored_traffic("w", "k") == 1234.5
    f.write_text("kernel_source_sha: other\ntraffic_bytes_per_launch: 1234.5\n")
    assert bench.stored_traffic("w", "k") is None
    assert bench.stored_traffic("w", "missing") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
