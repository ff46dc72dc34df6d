// noalloc.hip -- xamg_solve_noalloc: the solve of xamg_solve for callers
// that cannot allocate device memory (code under HIP graph capture, tight
// serving loops, harnesses that forbid hipMalloc).  Every buffer xamg_solve
// would allocate or take from the handle -- the Krylov and V-cycle work
// vectors, the padding copies of B and X, the per-column state and the
// per-block partial dot sums -- is carved from one file-scope device array
// of XAMG_NOALLOC_SCRATCH_BYTES, resident on each device the library runs
// on until the process ends.  The kernels are those of xamg_solve.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <utility>

#include "internal.h"
#include "solver.hpp"

namespace xamg {
namespace {

constexpr size_t kScratchBytes = size_t(XAMG_NOALLOC_SCRATCH_BYTES);
constexpr int kMaxDevices = 64;

// The device array itself.  In host code its name is only a stand-in for
// the symbol: host code uses the address hipGetSymbolAddress returns for
// the current device, never the name.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
char* g_scratch[kMaxDevices] = {};

// Address of the current device's copy of the array, looked up once per
// device (with that device current) and kept.
int scratch_base(char** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        set_error("no current HIP device for the scratch array");
        return XAMG_ENODEV;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch) failed on device %d: %d (%s)", dev, int(e),
                      hipGetErrorString(e));
            return XAMG_EHIP;
        }
        g_scratch[dev] = static_cast<char*>(p);
    }
    *out = g_scratch[dev];
    return XAMG_OK;
}

constexpr size_t round256(size_t b) { return (b + 255) & ~size_t(255); }

// Puts the handle's own work, state and partials back on every exit path.
struct Borrow {
    Handle& h;
    dev::ColState* st;
    double* part;
    int timer_kind;
    Borrow(Handle& hh, dev::ColState* s, double* p)
        : h(hh), st(hh.st), part(hh.part), timer_kind(hh.timer_kind)
    {
        std::swap(h.w, h.w_na);
        h.st = s;
        h.part = p;
        h.timer_kind = 0;   // the kernel timer would create events
    }
    ~Borrow()
    {
        std::swap(h.w, h.w_na);
        h.st = st;
        h.part = part;
        h.timer_kind = timer_kind;
    }
};

}  // namespace
}  // namespace xamg

using xamg::Handle;

extern "C" int xamg_solve_noalloc(xamg_handle_t* hh, const double* B, double* X, int32_t m,
                                  double tol, xamg_stats_t* stats)
{
    xamg::clear_error();
    Handle* h = static_cast<Handle*>(hh);
    if (!h || !B || !X) return xamg::fail(XAMG_EINVAL, "null argument");
    if (m < 1 || m > XAMG_MAX_M) return xamg::fail(XAMG_EINVAL, "m must be in 1..32");
    if (!(tol > 0.0) || !std::isfinite(tol)) return xamg::fail(XAMG_EINVAL, "tol must be positive");
    if ((reinterpret_cast<uintptr_t>(B) & 15u) || (reinterpret_cast<uintptr_t>(X) & 15u))
        return xamg::fail(XAMG_EINVAL, "B and X must be 16-byte aligned");
    const int mp = xamg::padded_m(m);
    const bool bicg = xamg::bicg_like(h->opt);
    const bool pad = mp != m;
    const size_t st_bytes = xamg::round256(sizeof(xamg::dev::ColState));
    const size_t part_bytes =
        xamg::round256(size_t(h->nb_cap) * xamg::dev::kMaxDots * XAMG_MAX_M * sizeof(double));
    const size_t work_bytes = xamg::carve_work(*h, mp, bicg, pad, h->w_na, nullptr, 0);
    const size_t need = st_bytes + part_bytes + work_bytes;
    if (need > xamg::kScratchBytes) {
        xamg::set_error("the solve needs %zu bytes of work memory for %d columns; the "
                        "no-allocation scratch array holds %zu",
                        need, mp, xamg::kScratchBytes);
        return XAMG_EINVAL;
    }
    char* base = nullptr;
    int rc = xamg::scratch_base(&base);
    if (rc) return rc;
    xamg::carve_work(*h, mp, bicg, pad, h->w_na, base + st_bytes + part_bytes,
                     xamg::kScratchBytes - st_bytes - part_bytes);
    try {
        xamg::Borrow borrow(*h, reinterpret_cast<xamg::dev::ColState*>(base),
                            reinterpret_cast<double*>(base + st_bytes));
        // the array keeps the previous call's contents: the column state
        // starts from zero (a fill kernel, no memset node under capture)
        hipLaunchKernelGGL((xamg::dev::copy_cols_kernel<double, double>), dim3(4), dim3(256), 0,
                           h->stream, static_cast<const double*>(nullptr), 1,
                           reinterpret_cast<double*>(base), 1, int(st_bytes / sizeof(double)), 0);
        // a handle not yet tuned for mp takes the tuning cache's choices for
        // its operators (a host lookup: no timing, no launch, no allocation)
        switch (mp) {
        case 1: xamg::apply_cached_tuning<1>(*h); break;
        case 2: xamg::apply_cached_tuning<2>(*h); break;
        case 4: xamg::apply_cached_tuning<4>(*h); break;
        case 8: xamg::apply_cached_tuning<8>(*h); break;
        case 16: xamg::apply_cached_tuning<16>(*h); break;
        default: xamg::apply_cached_tuning<32>(*h); break;
        }
        rc = xamg::solve_run(*h, B, X, m, tol, stats);
        if (rc == XAMG_EINVAL && xamg::last_error()[0] == '\0')
            xamg::set_error("B contains NaN or Inf");
        return rc;
    } catch (const xamg::DevFail& f) {
        return f.code;
    }
}
