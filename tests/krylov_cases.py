"""Seeded small systems built to drive the Krylov methods into their rarely
taken branches, shared as inputs by the oracle pins and the GPU tests.
Input construction only: nothing here computes any step of a solver.

Every case states the exact arithmetic that makes the branch happen; the
entries are small integers or powers of two, so the quantities that must be
zero are exactly zero in floating point, whatever the summation order.
"""
import numpy as np


def csr(A):
    """Dense square matrix -> sorted CSR arrays with the diagonal stored."""
    A = np.asarray(A, np.float64)
    n = A.shape[0]
    rows, cols = [], []
    for i in range(n):
        js = set(np.nonzero(A[i])[0].tolist()) | {i}
        for j in sorted(js):
            rows.append(i)
            cols.append(j)
    rows = np.array(rows)
    cols = np.array(cols)
    rp = np.zeros(n + 1, np.int32)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp).astype(np.int32)
    return rp, cols.astype(np.int32), A[rows, cols].astype(np.float64)


def nonsymmetric(n, seed):
    """Diagonally dominant nonsymmetric matrix (eigenvalues in the right
    half plane): tridiagonal with unequal off-diagonals plus a third
    superdiagonal."""
    rng = np.random.default_rng(seed)
    A = np.diag(4.0 + rng.uniform(0.0, 1.0, n))
    for i in range(n - 1):
        A[i, i + 1] = -1.0 + 0.6 * rng.uniform(-1.0, 1.0)
        A[i + 1, i] = -1.0 - 0.6 * rng.uniform(-1.0, 1.0)
    for i in range(n - 3):
        A[i, i + 3] = 0.5 * rng.uniform(-1.0, 1.0)
    return A


def rho_breakdown(n=8, seed=1):
    """BiCGStab without preconditioner, b = e_0, first row of A = e_0^T:
    iteration 1 has alpha = 1 exactly, so s, t and the new r vanish in
    component 0; iteration 2 then finds rho' = (rh, r) = (e_0, r) = 0 and
    restarts with rh = r, after which the solve continues in the trailing
    block and converges.  Returns (A, b)."""
    rng = np.random.default_rng(seed)
    A = np.zeros((n, n))
    A[0, 0] = 1.0
    A[1:, 0] = rng.uniform(-1.0, 1.0, n - 1)
    A[1:, 1:] = nonsymmetric(n - 1, seed + 100)
    b = np.zeros(n)
    b[0] = 1.0
    return A, b


def rhv_breakdown(n=8):
    """BiCGStab without preconditioner: the leading block [[1, -2], [0, 1]]
    and b = e_0 + e_1 give v = A p = A b = (-1, 1, 0, ...), so
    (rh, v) = -1 + 1 = 0 on the first iteration and again after the
    restart (rh = r = b): the second breakdown in a row stops the column.
    Returns (A, b)."""
    A = 2.0 * np.eye(n)
    A[0, 0], A[0, 1], A[1, 1] = 1.0, -2.0, 1.0
    b = np.zeros(n)
    b[0] = b[1] = 1.0
    return A, b


def omega_breakdown(n=8):
    """BiCGStab without preconditioner, b = e_0: alpha = 1, s = (0, -1, -1),
    t = A s = (0, 1, -1), (t, s) = 0, so omega = 0 (first breakdown, restart
    with rh = r = s); the next iteration finds (rh, v) = (s, A s) = 0, the
    second breakdown in a row.  Returns (A, b)."""
    A = 2.0 * np.eye(n)
    A[:3, :3] = [[1.0, 0.0, 0.0], [1.0, 1.0, -2.0], [1.0, 0.0, 1.0]]
    b = np.zeros(n)
    b[0] = 1.0
    return A, b


def indefinite(n=8):
    """Symmetric indefinite matrix (two negative eigenvalues) and right-hand
    sides: the eigenvectors of the largest and the smallest eigenvalue and a
    vector of ones.  With the exact one-level preconditioner M = A^-1,
    CG's (p, q) = (A^-1 b, b) is negative for the second column (a
    breakdown) and positive for the others.  Returns (A, B)."""
    A = np.diag([4.0, 3.0, 5.0, 6.0, -3.0, -4.0, 5.0, 2.0][:n])
    for i in range(n - 1):
        A[i, i + 1] = A[i + 1, i] = 0.5
    w, V = np.linalg.eigh(A)
    B = np.stack([V[:, -1], V[:, 0], np.ones(n)], axis=1)
    return A, np.ascontiguousarray(B)
