// Drives the library's host setup (classical AMG hierarchy construction and
// the dense inverse of the coarsest level) on small inputs, for a build with
// AddressSanitizer and UndefinedBehaviorSanitizer (CPU only; no HIP).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "internal.h"
#include "xamg.h"

#define CHECK(c) do { if (!(c)) { std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); std::exit(1); } } while (0)

static void stencil(int N, double kz, std::vector<int32_t>& rp, std::vector<int32_t>& ci,
                    std::vector<double>& v)
{
    const int n = N * N * N;
    rp.assign(1, 0);
    ci.clear();
    v.clear();
    for (int i = 0; i < n; ++i) {
        const int x = i % N, y = (i / N) % N, z = i / (N * N);
        const double diag = 4.0 + 2.0 * kz;
        if (z > 0) { ci.push_back(i - N * N); v.push_back(-kz); }
        if (y > 0) { ci.push_back(i - N); v.push_back(-1.0); }
        if (x > 0) { ci.push_back(i - 1); v.push_back(-1.0); }
        ci.push_back(i); v.push_back(diag);
        if (x < N - 1) { ci.push_back(i + 1); v.push_back(-1.0); }
        if (y < N - 1) { ci.push_back(i + N); v.push_back(-1.0); }
        if (z < N - 1) { ci.push_back(i + N * N); v.push_back(-kz); }
        rp.push_back(int32_t(ci.size()));
    }
}

int main()
{
    for (int N : {5, 9, 12})
        for (double kz : {1.0, 0.01}) {
            std::vector<int32_t> rp, ci;
            std::vector<double> v;
            stencil(N, kz, rp, ci, v);
            xamg_csr_t a{N * N * N, N * N * N, int64_t(ci.size()), rp.data(), ci.data(), v.data()};
            xamg_setup_params_t prm;
            xamg_default_setup_params(&prm);
            prm.agg_levels = N == 12 ? 2 : (N == 9 ? 1 : 0);
            prm.num_paths = kz < 1.0 ? 2 : 1;
            xamg_host_hierarchy_t* h = nullptr;
            CHECK(xamg_hierarchy_build(&a, &prm, &h) == XAMG_OK);
            xamg_hierarchy_t view;
            CHECK(xamg_hierarchy_view(h, &view) == XAMG_OK);
            for (int l = 0; l < view.nlevels; ++l) {
                std::vector<int8_t> cf(size_t(view.A[l].nrows));
                xamg_hierarchy_cf(h, l, cf.data());
            }
            const xamg_csr_t& c = view.A[view.nlevels - 1];
            const int nl = int(c.nrows);
            std::vector<double> dense(size_t(nl) * nl, 0.0), inv(size_t(nl) * nl);
            for (int i = 0; i < nl; ++i)
                for (int k = c.row_ptr[i]; k < c.row_ptr[i + 1]; ++k)
                    dense[size_t(i) * nl + c.col[k]] = c.val[k];
            CHECK(xamg::dense_inverse(nl, dense.data(), inv.data()) == XAMG_OK);
            xamg_hierarchy_free(h);
        }
    // malformed input is rejected, not read out of bounds
    std::vector<int32_t> rp{0, 2, 3}, ci{0, 5, 1};
    std::vector<double> v{1.0, 2.0, 3.0};
    xamg_csr_t bad{2, 2, 3, rp.data(), ci.data(), v.data()};
    xamg_host_hierarchy_t* h = nullptr;
    CHECK(xamg_hierarchy_build(&bad, nullptr, &h) == XAMG_EINVAL);
    std::printf("setup driver ok\n");
    return 0;
}
