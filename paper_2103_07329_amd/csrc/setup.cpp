// setup.cpp -- host-side construction of the classical AMG hierarchy.
//
// The paper builds its multigrid hierarchy once, on the host, with the
// classical (Ruge-Stueben) algebraic multigrid of hypre, and optimises only
// the solve phase (Section 2.3, the MultiGrid setup() wrapper; Section 1).
// This file is this library's own setup with the same ingredients:
//   * classical strength of connection, theta = 0.25 by default;
//   * the first Ruge-Stueben coarsening pass (largest weight first, lowest
//     index on ties, no second pass);
//   * direct interpolation; on the first `agg_levels` levels instead
//     aggressive coarsening (a second RS pass over the C points on their
//     distance-two strength with `num_paths` paths) and multipass
//     interpolation -- the paper's mg_agg_num_levels / mg_num_paths
//     parameters (Section 2.4, its example configuration);
//   * Galerkin coarse operators A_{l+1} = R_l A_l P_l with R_l = P_l^T;
//   * stop when a level has at most `max_coarse` rows;
//   * per level a Lanczos estimate of lambda_max(D^-1 A_l) for Chebyshev.
// The result is plain CSR arrays (int32 indices, float64 values) that the
// device setup (xamg_setup) uploads.  Nothing here touches the GPU.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "xamg.h"
#include "internal.h"

namespace xamg {

namespace {

struct Csr {
    int nr = 0, nc = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> v;
    int64_t nnz() const { return rp.empty() ? 0 : rp[nr]; }
};

// ---- strength: S_i = { j != i : -a_ij >= theta * max_k(-a_ik) } ------------
void strength(const Csr& a, double theta, std::vector<int32_t>& srp,
              std::vector<int32_t>& sci)
{
    const int n = a.nr;
    srp.assign(n + 1, 0);
    std::vector<double> thr(n);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double mx = 0.0;
        for (int k = a.rp[i]; k < a.rp[i + 1]; ++k)
            if (a.ci[k] != i) mx = std::max(mx, -a.v[k]);
        thr[i] = mx;
        int cnt = 0;
        if (mx > 0.0)
            for (int k = a.rp[i]; k < a.rp[i + 1]; ++k)
                cnt += (a.ci[k] != i && -a.v[k] >= theta * mx);
        srp[i + 1] = cnt;
    }
    for (int i = 0; i < n; ++i) srp[i + 1] += srp[i];
    sci.resize(std::max<int64_t>(srp[n], 1));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        const double mx = thr[i];
        int pos = srp[i];
        if (mx > 0.0)
            for (int k = a.rp[i]; k < a.rp[i + 1]; ++k)
                if (a.ci[k] != i && -a.v[k] >= theta * mx) sci[pos++] = a.ci[k];
    }
}

void transpose_pattern(int n, const std::vector<int32_t>& rp,
                       const std::vector<int32_t>& ci, std::vector<int32_t>& trp,
                       std::vector<int32_t>& tci)
{
    trp.assign(n + 1, 0);
    const int64_t nnz = rp[n];
    for (int64_t k = 0; k < nnz; ++k) trp[ci[k] + 1]++;
    for (int i = 0; i < n; ++i) trp[i + 1] += trp[i];
    tci.resize(std::max<int64_t>(nnz, 1));
    std::vector<int32_t> pos(trp.begin(), trp.end() - 1);
    for (int i = 0; i < n; ++i)
        for (int k = rp[i]; k < rp[i + 1]; ++k) tci[pos[ci[k]]++] = i;
}

// ---- first-pass RS split ----------------------------------------------------
// A max segment tree over the points holds the weight of every undecided
// point (decided points hold -1); the root yields the undecided point of
// largest weight, the leftmost one among equals.
class ArgmaxTree {
  public:
    explicit ArgmaxTree(const std::vector<int>& w) : n_(int(w.size()))
    {
        size_ = 1;
        while (size_ < n_) size_ <<= 1;
        val_.assign(2 * size_, -1);
        idx_.assign(2 * size_, 0);
        for (int i = 0; i < size_; ++i) {
            val_[size_ + i] = i < n_ ? w[i] : -1;
            idx_[size_ + i] = i;
        }
        for (int p = size_ - 1; p >= 1; --p) pull(p);
    }
    void set(int i, int w)
    {
        int p = size_ + i;
        val_[p] = w;
        for (p >>= 1; p >= 1; p >>= 1) pull(p);
    }
    int top_value() const { return val_[1]; }
    int top_index() const { return idx_[1]; }

  private:
    void pull(int p)
    {
        const int l = 2 * p, r = l + 1;
        if (val_[r] > val_[l]) { val_[p] = val_[r]; idx_[p] = idx_[r]; }
        else { val_[p] = val_[l]; idx_[p] = idx_[l]; }   // ties: left = lower index
    }
    int n_, size_;
    std::vector<int> val_, idx_;
};

enum : int8_t { U = 0, C = 1, F = 2 };

void rs_split(int n, const std::vector<int32_t>& srp, const std::vector<int32_t>& sci,
              const std::vector<int32_t>& trp, const std::vector<int32_t>& tci,
              std::vector<int8_t>& state)
{
    std::vector<int> lam(n);
    for (int i = 0; i < n; ++i) lam[i] = trp[i + 1] - trp[i];
    state.assign(n, U);
    ArgmaxTree tree(lam);
    while (tree.top_value() >= 0) {
        const int i = tree.top_index();
        state[i] = C;
        tree.set(i, -1);
        for (int k = trp[i]; k < trp[i + 1]; ++k) {   // points depending on i
            const int j = tci[k];
            if (state[j] != U) continue;
            state[j] = F;
            tree.set(j, -1);
            for (int kk = srp[j]; kk < srp[j + 1]; ++kk) {
                const int l = sci[kk];
                if (state[l] == U) tree.set(l, ++lam[l]);
            }
        }
        for (int k = srp[i]; k < srp[i + 1]; ++k) {   // points i depends on
            const int j = sci[k];
            if (state[j] == U) tree.set(j, --lam[j]);
        }
    }
}

// ---- direct interpolation ---------------------------------------------------
void direct_interpolation(const Csr& a, const std::vector<int32_t>& srp,
                          const std::vector<int32_t>& sci,
                          const std::vector<int8_t>& state, Csr& P)
{
    const int n = a.nr;
    std::vector<int32_t> cidx(n, -1);
    int nc = 0;
    for (int i = 0; i < n; ++i)
        if (state[i] == C) cidx[i] = nc++;
    // strong-C membership by a per-row merge of the sorted strength list
    P.nr = n;
    P.nc = nc;
    P.rp.assign(n + 1, 0);
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        if (state[i] == C) { P.rp[i + 1] = 1; continue; }
        int cnt = 0;
        for (int s = srp[i]; s < srp[i + 1]; ++s) cnt += (state[sci[s]] == C);
        P.rp[i + 1] = cnt;
    }
    for (int i = 0; i < n; ++i) P.rp[i + 1] += P.rp[i];
    P.ci.resize(std::max<int64_t>(P.rp[n], 1));
    P.v.resize(std::max<int64_t>(P.rp[n], 1));
#pragma omp parallel for schedule(dynamic, 4096)
    for (int i = 0; i < n; ++i) {
        int pos = P.rp[i];
        if (state[i] == C) { P.ci[pos] = cidx[i]; P.v[pos] = 1.0; continue; }
        double diag = 0.0, neg_all = 0.0, pos_all = 0.0, neg_c = 0.0, pos_c = 0.0;
        int s = srp[i];
        for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) {
            const int j = a.ci[k];
            const double x = a.v[k];
            if (j == i) { diag += x; continue; }
            (x < 0.0 ? neg_all : pos_all) += x;
            while (s < srp[i + 1] && sci[s] < j) ++s;
            if (s < srp[i + 1] && sci[s] == j && state[j] == C)
                (x < 0.0 ? neg_c : pos_c) += x;
        }
        if (pos_c == 0.0) diag += pos_all;
        const double alpha = neg_c != 0.0 ? neg_all / neg_c : 0.0;
        const double beta = pos_c != 0.0 ? pos_all / pos_c : 0.0;
        s = srp[i];
        for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) {
            const int j = a.ci[k];
            if (j == i) continue;
            while (s < srp[i + 1] && sci[s] < j) ++s;
            if (s < srp[i + 1] && sci[s] == j && state[j] == C) {
                const double x = a.v[k];
                P.ci[pos] = cidx[j];
                P.v[pos] = -(x < 0.0 ? alpha : beta) * x / diag;
                ++pos;
            }
        }
    }
}

// ---- aggressive coarsening (the first `agg_levels` levels) ------------------
// A second Ruge-Stueben pass over the first pass's C points, on the
// distance-two strength among them: j is a strong connection of i (both C
// after the first pass, j != i) when there are at least `num_paths` paths of
// length one or two from i to j in S, i.e. [j in S_i] + |{k in S_i : j in
// S_k}| >= num_paths.  The points the second pass makes F join the F points;
// the second pass's C points are the coarse grid.
void aggressive_split(int n, const std::vector<int32_t>& srp, const std::vector<int32_t>& sci,
                      int num_paths, std::vector<int8_t>& state)
{
    // state holds the first pass's split on entry
    std::vector<int32_t> cid(n, -1), cpt;
    for (int i = 0; i < n; ++i)
        if (state[i] == C) {
            cid[i] = int32_t(cpt.size());
            cpt.push_back(i);
        }
    const int nc = int(cpt.size());
    std::vector<int32_t> s2rp(nc + 1, 0), s2ci;
    std::vector<int> cnt(nc, 0);
    std::vector<int32_t> touched;
    for (int a = 0; a < nc; ++a) {
        const int i = cpt[a];
        touched.clear();
        auto add = [&](int j) {
            const int b = cid[j];
            if (b < 0 || j == i) return;
            if (cnt[b]++ == 0) touched.push_back(b);
        };
        for (int k = srp[i]; k < srp[i + 1]; ++k) {
            const int j = sci[k];
            add(j);
            for (int kk = srp[j]; kk < srp[j + 1]; ++kk) add(sci[kk]);
        }
        std::sort(touched.begin(), touched.end());
        for (int b : touched) {
            if (cnt[b] >= num_paths) s2ci.push_back(b);
            cnt[b] = 0;
        }
        s2rp[a + 1] = int32_t(s2ci.size());
    }
    if (s2ci.empty()) s2ci.push_back(0);
    std::vector<int32_t> t2rp, t2ci;
    transpose_pattern(nc, s2rp, s2ci, t2rp, t2ci);
    std::vector<int8_t> st2;
    rs_split(nc, s2rp, s2ci, t2rp, t2ci, st2);
    for (int a = 0; a < nc; ++a) state[cpt[a]] = st2[a];
}

// ---- multipass interpolation (the aggressive levels) -------------------------
// C points are unit rows (pass 0).  Pass p = 1, 2, ... takes the F points
// not yet interpolated that have a strong connection to a point of an
// earlier pass; each interpolates, with the direct-interpolation weights,
// from those strong neighbours P_i of earlier passes, substituting their
// rows: P_i. = sum_{j in P_i} w_ij P_j.  Pass 1 is direct interpolation
// from the strong C neighbours.  F points that no pass reaches keep a zero
// row.  Entries that come out exactly 0.0 are dropped.
void multipass_interpolation(const Csr& a, const std::vector<int32_t>& srp,
                             const std::vector<int32_t>& sci, const std::vector<int8_t>& state,
                             Csr& P)
{
    const int n = a.nr;
    std::vector<int32_t> cidx(n, -1);
    int nc = 0;
    for (int i = 0; i < n; ++i)
        if (state[i] == C) cidx[i] = nc++;
    std::vector<int> pass(n, -1);
    for (int i = 0; i < n; ++i)
        if (state[i] == C) pass[i] = 0;
    // rows of P as sorted (column, value) lists
    std::vector<std::vector<std::pair<int32_t, double>>> row(n);
    for (int i = 0; i < n; ++i)
        if (state[i] == C) row[i].push_back({cidx[i], 1.0});
    std::vector<double> acc(nc, 0.0);
    std::vector<char> mark(nc, 0);
    std::vector<int32_t> cols;
    for (int p = 1;; ++p) {
        std::vector<int> now;
        for (int i = 0; i < n; ++i) {
            if (pass[i] >= 0) continue;
            for (int k = srp[i]; k < srp[i + 1]; ++k)
                if (pass[sci[k]] >= 0 && pass[sci[k]] < p) {
                    now.push_back(i);
                    break;
                }
        }
        if (now.empty()) break;
        for (int i : now) pass[i] = p;
        for (int i : now) {
            double diag = 0.0, neg_all = 0.0, pos_all = 0.0, neg_p = 0.0, pos_p = 0.0;
            auto in_p = [&](int j) {
                // strong neighbour from an earlier pass (S_i sorted)
                if (pass[j] < 0 || pass[j] >= p) return false;
                return std::binary_search(sci.begin() + srp[i], sci.begin() + srp[i + 1], j);
            };
            for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) {
                const int j = a.ci[k];
                const double x = a.v[k];
                if (j == i) { diag += x; continue; }
                (x < 0.0 ? neg_all : pos_all) += x;
                if (in_p(j)) (x < 0.0 ? neg_p : pos_p) += x;
            }
            if (pos_p == 0.0) diag += pos_all;
            const double alpha = neg_p != 0.0 ? neg_all / neg_p : 0.0;
            const double beta = pos_p != 0.0 ? pos_all / pos_p : 0.0;
            cols.clear();
            for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) {
                const int j = a.ci[k];
                if (j == i || !in_p(j)) continue;
                const double x = a.v[k];
                const double w = -(x < 0.0 ? alpha : beta) * x / diag;
                for (const auto& e : row[j]) {
                    if (!mark[e.first]) { mark[e.first] = 1; cols.push_back(e.first); }
                    acc[e.first] += w * e.second;
                }
            }
            std::sort(cols.begin(), cols.end());
            for (int c : cols) {
                if (acc[c] != 0.0) row[i].push_back({c, acc[c]});
                acc[c] = 0.0;
                mark[c] = 0;
            }
        }
    }
    P.nr = n;
    P.nc = nc;
    P.rp.assign(n + 1, 0);
    for (int i = 0; i < n; ++i) P.rp[i + 1] = P.rp[i] + int32_t(row[i].size());
    P.ci.resize(std::max<int64_t>(P.rp[n], 1));
    P.v.resize(std::max<int64_t>(P.rp[n], 1));
    for (int i = 0; i < n; ++i) {
        int pos = P.rp[i];
        for (const auto& e : row[i]) { P.ci[pos] = e.first; P.v[pos] = e.second; ++pos; }
    }
}

void transpose(const Csr& a, Csr& t)
{
    t.nr = a.nc;
    t.nc = a.nr;
    t.rp.assign(t.nr + 1, 0);
    const int64_t nnz = a.nnz();
    for (int64_t k = 0; k < nnz; ++k) t.rp[a.ci[k] + 1]++;
    for (int i = 0; i < t.nr; ++i) t.rp[i + 1] += t.rp[i];
    t.ci.resize(std::max<int64_t>(nnz, 1));
    t.v.resize(std::max<int64_t>(nnz, 1));
    std::vector<int32_t> pos(t.rp.begin(), t.rp.end() - 1);
    for (int i = 0; i < a.nr; ++i)
        for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) {
            const int p = pos[a.ci[k]]++;
            t.ci[p] = i;
            t.v[p] = a.v[k];
        }
}

// C = A * B, row-parallel two-pass Gustavson; exact zeros dropped.
void spgemm(const Csr& A, const Csr& B, Csr& Cm)
{
    const int n = A.nr, nc = B.nc;
    Cm.nr = n;
    Cm.nc = nc;
    Cm.rp.assign(n + 1, 0);
    std::vector<std::vector<int32_t>> rows_c(n);
    std::vector<std::vector<double>> rows_v(n);
#pragma omp parallel
    {
        std::vector<int32_t> mark(nc, -1);
        std::vector<double> acc(nc, 0.0);
        std::vector<int32_t> list;
#pragma omp for schedule(dynamic, 1024)
        for (int i = 0; i < n; ++i) {
            list.clear();
            for (int k = A.rp[i]; k < A.rp[i + 1]; ++k) {
                const int j = A.ci[k];
                const double aij = A.v[k];
                for (int kk = B.rp[j]; kk < B.rp[j + 1]; ++kk) {
                    const int c = B.ci[kk];
                    if (mark[c] != i) { mark[c] = i; acc[c] = 0.0; list.push_back(c); }
                    acc[c] += aij * B.v[kk];
                }
            }
            std::sort(list.begin(), list.end());
            auto& rc = rows_c[i];
            auto& rv = rows_v[i];
            rc.reserve(list.size());
            rv.reserve(list.size());
            for (int c : list)
                if (acc[c] != 0.0) { rc.push_back(c); rv.push_back(acc[c]); }
        }
    }
    for (int i = 0; i < n; ++i) Cm.rp[i + 1] = Cm.rp[i] + int(rows_c[i].size());
    Cm.ci.resize(std::max<int64_t>(Cm.nnz(), 1));
    Cm.v.resize(std::max<int64_t>(Cm.nnz(), 1));
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        std::copy(rows_c[i].begin(), rows_c[i].end(), Cm.ci.begin() + Cm.rp[i]);
        std::copy(rows_v[i].begin(), rows_v[i].end(), Cm.v.begin() + Cm.rp[i]);
        std::vector<int32_t>().swap(rows_c[i]);
        std::vector<double>().swap(rows_v[i]);
    }
}

// SplitMix64 (Steele, Lea, Flood 2014) as a counter-based generator:
// element i of stream `key` is the output for state key*G + (i+1)*G.
double splitmix_uniform(uint64_t key, uint64_t i)
{
    constexpr uint64_t G = 0x9E3779B97F4A7C15ull;
    uint64_t z = key * G + (i + 1) * G;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return double(z >> 11) * 0x1.0p-53 * 2.0 - 1.0;
}

// Largest Ritz value of `steps` Lanczos steps on D^-1/2 A D^-1/2.
double lanczos_lambda_max(const Csr& a, int steps, uint64_t key)
{
    const int n = a.nr;
    steps = std::min(steps, std::min(n, 63));
    std::vector<double> s(n), v(n), vp(n, 0.0), w(n);
    double nrm = 0.0;
    for (int i = 0; i < n; ++i) {
        double d = 0.0;
        for (int k = a.rp[i]; k < a.rp[i + 1]; ++k)
            if (a.ci[k] == i) d += a.v[k];
        s[i] = 1.0 / std::sqrt(d);
        v[i] = splitmix_uniform(key, uint64_t(i));
        nrm += v[i] * v[i];
    }
    nrm = std::sqrt(nrm);
    for (double& x : v) x /= nrm;
    std::vector<double> al, be{0.0};
    for (int j = 0; j < steps; ++j) {
#pragma omp parallel for schedule(static)
        for (int i = 0; i < n; ++i) {
            double acc = 0.0;
            for (int k = a.rp[i]; k < a.rp[i + 1]; ++k) acc += a.v[k] * s[a.ci[k]] * v[a.ci[k]];
            w[i] = s[i] * acc;
        }
        double alpha = 0.0;
        for (int i = 0; i < n; ++i) alpha += w[i] * v[i];
        double beta = 0.0;
        for (int i = 0; i < n; ++i) {
            w[i] -= alpha * v[i] + be[j] * vp[i];
            beta += w[i] * w[i];
        }
        beta = std::sqrt(beta);
        al.push_back(alpha);
        if (j + 1 < steps) {
            be.push_back(beta);
            if (beta == 0.0) break;
            for (int i = 0; i < n; ++i) { vp[i] = v[i]; v[i] = w[i] / beta; }
        }
    }
    // largest eigenvalue of the tridiagonal (al, be) by Sturm bisection
    const int k = int(al.size());
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? std::fabs(be[i]) : 0.0) + (i + 1 < k ? std::fabs(be[i + 1]) : 0.0);
        lo = std::min(lo, al[i] - r);
        hi = std::max(hi, al[i] + r);
    }
    auto below = [&](double x) {
        int c = 0;
        double q = 1.0;
        for (int i = 0; i < k; ++i) {
            q = al[i] - x - (i > 0 ? be[i] * be[i] / q : 0.0);
            if (q == 0.0) q = -1e-300;
            c += q < 0.0;
        }
        return c;
    };
    for (int it = 0; it < 200; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (below(mid) >= k) hi = mid; else lo = mid;
    }
    return hi;
}

}  // namespace

struct HostHierarchy {
    std::vector<Csr> A, P, R;
    std::vector<std::vector<int8_t>> cf;
    std::vector<double> lmax;
    // views handed to xamg_setup
    std::vector<xamg_csr_t> vA, vP, vR;
};

static void make_view(const Csr& c, xamg_csr_t& v)
{
    v.nrows = c.nr;
    v.ncols = c.nc;
    v.nnz = c.nnz();
    v.row_ptr = c.rp.data();
    v.col = c.ci.data();
    v.val = c.v.data();
}

int build_hierarchy(const xamg_csr_t* a0, const xamg_setup_params_t* prm,
                    HostHierarchy** out)
{
    auto h = new (std::nothrow) HostHierarchy;
    if (!h) return XAMG_ENOMEM;
    try {
        Csr A0;
        A0.nr = int(a0->nrows);
        A0.nc = int(a0->ncols);
        A0.rp.assign(a0->row_ptr, a0->row_ptr + a0->nrows + 1);
        A0.ci.assign(a0->col, a0->col + a0->nnz);
        A0.v.assign(a0->val, a0->val + a0->nnz);
        h->A.push_back(std::move(A0));
        while (h->A.back().nr > prm->max_coarse) {
            const Csr& a = h->A.back();
            if (int(h->A.size()) >= prm->max_levels) {
                set_error("hierarchy needs more than %d levels", prm->max_levels);
                delete h;
                return XAMG_EBREAKDOWN;
            }
            std::vector<int32_t> srp, sci, trp, tci;
            strength(a, prm->theta, srp, sci);
            transpose_pattern(a.nr, srp, sci, trp, tci);
            std::vector<int8_t> st;
            rs_split(a.nr, srp, sci, trp, tci, st);
            Csr P, R, AP, Ac;
            if (int(h->A.size()) <= prm->agg_levels) {
                aggressive_split(a.nr, srp, sci, prm->num_paths, st);
                multipass_interpolation(a, srp, sci, st, P);
            } else {
                direct_interpolation(a, srp, sci, st, P);
            }
            transpose(P, R);
            spgemm(a, P, AP);
            spgemm(R, AP, Ac);
            const int nprev = a.nr;
            h->cf.push_back(std::move(st));
            h->P.push_back(std::move(P));
            h->R.push_back(std::move(R));
            h->A.push_back(std::move(Ac));
            const int ncoarse = h->A.back().nr;
            if (ncoarse == 0 || double(ncoarse) > 0.9 * double(nprev)) {
                set_error("coarsening stalled: %d -> %d rows", nprev, ncoarse);
                delete h;
                return XAMG_EBREAKDOWN;
            }
        }
        const int nl = int(h->A.size());
        h->lmax.assign(nl, 0.0);
        for (int l = 0; l + 1 < nl; ++l)
            h->lmax[l] = lanczos_lambda_max(h->A[l], prm->lanczos_steps,
                                            (uint64_t(7) << 32) + uint64_t(l));
        h->vA.resize(nl);
        h->vP.resize(nl - 1);
        h->vR.resize(nl - 1);
        for (int l = 0; l < nl; ++l) make_view(h->A[l], h->vA[l]);
        for (int l = 0; l + 1 < nl; ++l) {
            make_view(h->P[l], h->vP[l]);
            make_view(h->R[l], h->vR[l]);
        }
    } catch (const std::bad_alloc&) {
        delete h;
        set_error("host memory exhausted during setup");
        return XAMG_ENOMEM;
    }
    *out = h;
    return XAMG_OK;
}

void view_hierarchy(const HostHierarchy* h, xamg_hierarchy_t* v)
{
    v->nlevels = int32_t(h->A.size());
    v->A = h->vA.data();
    v->P = h->vP.data();
    v->R = h->vR.data();
    v->lmax = h->lmax.data();
}

int hierarchy_cf(const HostHierarchy* h, int level, int8_t* out)
{
    if (level < 0 || level >= int(h->cf.size())) return XAMG_EINVAL;
    std::memcpy(out, h->cf[level].data(), h->cf[level].size());
    return XAMG_OK;
}

void free_hierarchy(HostHierarchy* h) { delete h; }

// Dense LU with partial pivoting, then the inverse column by column.
int dense_inverse(int n, const double* a, double* inv)
{
    std::vector<double> lu(a, a + size_t(n) * n);
    std::vector<int> piv(n);
    for (int k = 0; k < n; ++k) {
        int p = k;
        for (int i = k + 1; i < n; ++i)
            if (std::fabs(lu[size_t(i) * n + k]) > std::fabs(lu[size_t(p) * n + k])) p = i;
        if (lu[size_t(p) * n + k] == 0.0) return XAMG_EBREAKDOWN;
        piv[k] = p;
        if (p != k)
            for (int j = 0; j < n; ++j) std::swap(lu[size_t(k) * n + j], lu[size_t(p) * n + j]);
        for (int i = k + 1; i < n; ++i) {
            const double l = lu[size_t(i) * n + k] / lu[size_t(k) * n + k];
            lu[size_t(i) * n + k] = l;
            for (int j = k + 1; j < n; ++j) lu[size_t(i) * n + j] -= l * lu[size_t(k) * n + j];
        }
    }
    std::vector<double> col(n);
    for (int c = 0; c < n; ++c) {
        for (int i = 0; i < n; ++i) col[i] = (i == c) ? 1.0 : 0.0;
        for (int i = 0; i < n; ++i)
            if (piv[i] != i) std::swap(col[i], col[piv[i]]);
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < i; ++j) col[i] -= lu[size_t(i) * n + j] * col[j];
        for (int i = n - 1; i >= 0; --i) {
            for (int j = i + 1; j < n; ++j) col[i] -= lu[size_t(i) * n + j] * col[j];
            col[i] /= lu[size_t(i) * n + i];
        }
        for (int i = 0; i < n; ++i) inv[size_t(i) * n + c] = col[i];
    }
    return XAMG_OK;
}

}  // namespace xamg

// ---- C ABI: host setup ------------------------------------------------------
extern "C" {

void xamg_default_setup_params(xamg_setup_params_t* p)
{
    p->theta = 0.25;
    p->max_coarse = 64;
    p->max_levels = 40;
    p->lanczos_steps = 10;
    p->agg_levels = 0;
    p->num_paths = 1;
}

int xamg_hierarchy_build(const xamg_csr_t* A, const xamg_setup_params_t* params,
                         xamg_host_hierarchy_t** out)
{
    xamg::clear_error();
    if (!A || !out) return xamg::fail(XAMG_EINVAL, "null argument");
    xamg_setup_params_t def;
    xamg_default_setup_params(&def);
    const xamg_setup_params_t* p = params ? params : &def;
    int rc = xamg::validate_csr(A, true, "A");
    if (rc) return rc;
    if (!(p->theta > 0.0 && p->theta <= 1.0) || p->max_coarse < 1 || p->max_levels < 1 ||
        p->max_levels > XAMG_MAX_LEVELS || p->lanczos_steps < 1 || p->agg_levels < 0 ||
        p->num_paths < 1)
        return xamg::fail(XAMG_EINVAL, "bad setup parameters");
    xamg::HostHierarchy* h = nullptr;
    rc = xamg::build_hierarchy(A, p, &h);
    if (rc) return rc;
    *out = reinterpret_cast<xamg_host_hierarchy_t*>(h);
    return XAMG_OK;
}

int xamg_hierarchy_view(const xamg_host_hierarchy_t* h, xamg_hierarchy_t* view)
{
    if (!h || !view) return xamg::fail(XAMG_EINVAL, "null argument");
    xamg::view_hierarchy(reinterpret_cast<const xamg::HostHierarchy*>(h), view);
    return XAMG_OK;
}

int xamg_hierarchy_cf(const xamg_host_hierarchy_t* h, int32_t level, int8_t* cf)
{
    if (!h || !cf) return xamg::fail(XAMG_EINVAL, "null argument");
    return xamg::hierarchy_cf(reinterpret_cast<const xamg::HostHierarchy*>(h), level, cf);
}

void xamg_hierarchy_free(xamg_host_hierarchy_t* h)
{
    xamg::free_hierarchy(reinterpret_cast<xamg::HostHierarchy*>(h));
}

}  // extern "C"
