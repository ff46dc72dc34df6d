"""Seeded synthetic problem generators (inputs only).

This module builds the linear systems A X = B that the solver is run on: the
finite-difference matrices of the model problems of the paper's performance
section (3D Poisson equation with a 7-point stencil in a cube, Section 3) and
the diffusion variants used as further test problems, plus seeded blocks of
right-hand sides.  It holds none of the solver's arithmetic (no coarsening,
smoothing or Krylov steps), so both the CPU oracle and the GPU path may take
their inputs from here.

Conventions (shared by every generator):

* unknowns sit on the grid points (i, j, k) in [0, N)^3 of an N^3 grid with a
  homogeneous Dirichlet boundary eliminated, row index r = i + N*j + N*N*k
  (x fastest, 0-based);
* the operator is the negative discrete Laplacian (or -div(K grad u)) with
  grid step h = 1, so it is symmetric positive definite;
* CSR arrays: ``rowptr`` int32 (n+1), ``col`` int32 (nnz, sorted within a
  row, diagonal present), ``val`` float64;
* a block of m right-hand sides is an (n, m) float64 C-ordered array, i.e.
  the m columns are interleaved: B[i*m + j].
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "poisson7", "anisotropic7", "jump7", "stencil_csr", "uniform_rhs",
    "gaussian_rhs", "jump_kappa", "batched_systems", "Problem",
    "BATCH_SIDES", "BATCH_MS",
]

BATCH_SIDES = (48, 64, 96, 128, 160)
BATCH_MS = (1, 4, 8, 16, 32)


class Problem:
    """A CSR matrix with its grid side (plain container)."""

    def __init__(self, N, rowptr, col, val, name):
        self.N = int(N)
        self.n = int(N) ** 3
        self.rowptr = rowptr
        self.col = col
        self.val = val
        self.name = name

    @property
    def nnz(self):
        return int(self.rowptr[-1])

    def csr(self):
        return self.rowptr, self.col, self.val

    def __repr__(self):
        return f"Problem({self.name}, N={self.N}, n={self.n}, nnz={self.nnz})"


def stencil_csr(N, wxm, wxp, wym, wyp, wzm, wzp, diag):
    """Assemble a 7-point CSR matrix from per-point face weights.

    ``w?m``/``w?p`` are arrays of shape (N, N, N) indexed [k, j, i] giving the
    weight of the face towards the -/+ neighbour along each axis; the matrix
    entry for an in-grid neighbour is -weight, faces on the Dirichlet
    boundary contribute only to ``diag`` (already included by the caller).
    Columns of each row come out sorted: -z, -y, -x, diag, +x, +y, +z.
    """
    n = N ** 3
    kk, jj, ii = np.meshgrid(np.arange(N), np.arange(N), np.arange(N),
                             indexing="ij")
    r = (ii + N * jj + N * N * kk).ravel().astype(np.int64)
    ii = ii.ravel(); jj = jj.ravel(); kk = kk.ravel()
    cols = []
    vals = []
    masks = []
    # order of the seven slots within a row = increasing column index
    slots = [
        (kk > 0, r - N * N, -wzm.ravel()),
        (jj > 0, r - N, -wym.ravel()),
        (ii > 0, r - 1, -wxm.ravel()),
        (np.ones(n, dtype=bool), r, diag.ravel()),
        (ii < N - 1, r + 1, -wxp.ravel()),
        (jj < N - 1, r + N, -wyp.ravel()),
        (kk < N - 1, r + N * N, -wzp.ravel()),
    ]
    for m_, c_, v_ in slots:
        masks.append(m_)
        cols.append(c_)
        vals.append(v_)
    M = np.stack(masks, axis=1)            # (n, 7)
    C = np.stack(cols, axis=1)
    V = np.stack(vals, axis=1)
    counts = M.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = C[M].astype(np.int32)
    val = V[M].astype(np.float64)
    return rowptr.astype(np.int32), col, val


def _const_weights(N, cx, cy, cz):
    shape = (N, N, N)
    ones = np.ones(shape)
    diag = np.full(shape, 2.0 * (cx + cy + cz))
    return (cx * ones, cx * ones, cy * ones, cy * ones, cz * ones, cz * ones,
            diag)


def poisson7(N):
    """-Laplace(u) = f on the unit-step N^3 grid, 7-point stencil, Dirichlet.

    Diagonal 6, off-diagonals -1; nnz = 7 N^3 - 6 N^2.
    """
    wxm, wxp, wym, wyp, wzm, wzp, d = _const_weights(N, 1.0, 1.0, 1.0)
    rp, c, v = stencil_csr(N, wxm, wxp, wym, wyp, wzm, wzp, d)
    return Problem(N, rp, c, v, f"poisson{N}")


def anisotropic7(N, kx=1.0, ky=1.0, kz=0.01):
    """-div(K grad u) with K = diag(kx, ky, kz), 7-point stencil, Dirichlet."""
    wxm, wxp, wym, wyp, wzm, wzp, d = _const_weights(N, kx, ky, kz)
    rp, c, v = stencil_csr(N, wxm, wxp, wym, wyp, wzm, wzp, d)
    return Problem(N, rp, c, v, f"aniso{N}")


def jump_kappa(N, rng, block=8, lo=-3.0, hi=3.0):
    """Piecewise-constant coefficient: one value 10**U(lo, hi) per aligned
    block^3 cube of grid points, returned as an (N, N, N) array [k, j, i]."""
    nb = -(-N // block)
    logk = rng.uniform(lo, hi, size=(nb, nb, nb))
    kap = 10.0 ** logk
    kap = np.repeat(np.repeat(np.repeat(kap, block, 0), block, 1), block, 2)
    return kap[:N, :N, :N].copy()


def jump7(N, kappa):
    """-div(kappa grad u) with the face weight between neighbours p, q equal
    to the harmonic mean 2 k_p k_q / (k_p + k_q); a Dirichlet face weighs
    k_p; the diagonal is the sum of the six face weights."""
    k = kappa

    def hm(a, b):
        return 2.0 * a * b / (a + b)

    wxm = k.copy(); wxp = k.copy(); wym = k.copy(); wyp = k.copy()
    wzm = k.copy(); wzp = k.copy()
    wxp[:, :, :-1] = hm(k[:, :, :-1], k[:, :, 1:])
    wxm[:, :, 1:] = wxp[:, :, :-1]
    wyp[:, :-1, :] = hm(k[:, :-1, :], k[:, 1:, :])
    wym[:, 1:, :] = wyp[:, :-1, :]
    wzp[:-1, :, :] = hm(k[:-1, :, :], k[1:, :, :])
    wzm[1:, :, :] = wzp[:-1, :, :]
    diag = wxm + wxp + wym + wyp + wzm + wzp
    rp, c, v = stencil_csr(N, wxm, wxp, wym, wyp, wzm, wzp, diag)
    return Problem(N, rp, c, v, f"jump{N}")


def uniform_rhs(n, m, seed):
    """(n, m) block, i.i.d. U[-1, 1) from numpy's default_rng(seed)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=(n, m))


def gaussian_params(N, m, seed, nsrc=8, wlo=2.0, whi=8.0):
    """Source parameters of ``gaussian_rhs``: centres (m, nsrc, 3) uniform in
    [0, N)^3, widths (m, nsrc) uniform in [wlo, whi] cells, amplitudes
    (m, nsrc) uniform in [-1, 1], drawn from numpy's default_rng(seed) column
    by column in the order centres, widths, amplitudes."""
    rng = np.random.default_rng(seed)
    c = np.empty((m, nsrc, 3))
    s = np.empty((m, nsrc))
    a = np.empty((m, nsrc))
    for j in range(m):
        c[j] = rng.uniform(0.0, N, size=(nsrc, 3))
        s[j] = rng.uniform(wlo, whi, size=nsrc)
        a[j] = rng.uniform(-1.0, 1.0, size=nsrc)
    return c, s, a


def gaussian_rhs(N, m, seed, nsrc=8, wlo=2.0, whi=8.0):
    """Each column is a sum of ``nsrc`` Gaussian sources
    a * exp(-|x - c|^2 / (2 s^2)) at the cell indices x (lexicographic, x
    fastest), with the parameters of ``gaussian_params``."""
    c, s, a = gaussian_params(N, m, seed, nsrc, wlo, whi)
    n = N ** 3
    ax = np.arange(N, dtype=np.float64)
    B = np.empty((n, m))
    for j in range(m):
        col = np.zeros((N, N, N))
        for t in range(nsrc):
            gx = np.exp(-(ax - c[j, t, 0]) ** 2 / (2 * s[j, t] ** 2))
            gy = np.exp(-(ax - c[j, t, 1]) ** 2 / (2 * s[j, t] ** 2))
            gz = np.exp(-(ax - c[j, t, 2]) ** 2 / (2 * s[j, t] ** 2))
            col += a[j, t] * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
        B[:, j] = col.ravel()
    return B


def gaussian_rhs_torch(N, params, cols, torch, device):
    """Columns ``cols`` of a Gaussian-source block with parameters from
    ``gaussian_params``, evaluated with torch (float64) on ``device``:
    an (n, len(cols)) contiguous tensor.  Same formula as ``gaussian_rhs``
    (values agree to rounding); used to make large training sets in place."""
    c, s, a = (torch.as_tensor(v, dtype=torch.float64, device=device) for v in params)
    ax = torch.arange(N, dtype=torch.float64, device=device)
    out = torch.empty((N ** 3, len(cols)), dtype=torch.float64, device=device)
    for k, j in enumerate(cols):
        col = torch.zeros((N, N, N), dtype=torch.float64, device=device)
        for t in range(c.shape[1]):
            den = 2 * s[j, t] ** 2
            gx = torch.exp(-(ax - c[j, t, 0]) ** 2 / den)
            gy = torch.exp(-(ax - c[j, t, 1]) ** 2 / den)
            gz = torch.exp(-(ax - c[j, t, 2]) ** 2 / den)
            col += a[j, t] * gz[:, None, None] * gy[None, :, None] * gx[None, None, :]
        out[:, k] = col.reshape(-1)
    return out


def batched_systems(seed=1004, count=12, sides=BATCH_SIDES, ms=BATCH_MS,
                    max_side=None):
    """Uneven batch of jump-coefficient systems.

    Draw order from default_rng(seed): the ``count`` grid sides, then the
    ``count`` column counts, then per system its coefficient field and its
    uniform right-hand-side block.  ``max_side`` (optional) clips the sides
    for small test runs, after the draws, so the rest of the stream is the
    same.  Returns a list of (Problem, B).
    """
    rng = np.random.default_rng(seed)
    Ns = rng.choice(np.asarray(sides), size=count)
    Ms = rng.choice(np.asarray(ms), size=count)
    out = []
    for s in range(count):
        N = int(Ns[s]) if max_side is None else min(int(Ns[s]), max_side)
        kap = jump_kappa(N, rng)
        prob = jump7(N, kap)
        B = rng.uniform(-1.0, 1.0, size=(prob.n, int(Ms[s])))
        out.append((prob, B))
    return out
