// common.cpp -- error reporting and argument validation for libxamg.
#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "internal.h"

namespace xamg {

namespace {
thread_local char g_err[512] = "";
}

void set_error(const char* fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = '\0'; }

const char* last_error() { return g_err; }

int validate_csr(const xamg_csr_t* a, bool square, const char* name)
{
    if (!a) { set_error("%s: null matrix", name); return XAMG_EINVAL; }
    if (a->nrows < 0 || a->ncols < 0 || a->nnz < 0 || a->nrows > INT32_MAX - 1 ||
        a->ncols > INT32_MAX - 1 || a->nnz > INT32_MAX) {
        set_error("%s: sizes out of range", name);
        return XAMG_EINVAL;
    }
    if (square && a->nrows != a->ncols) {
        set_error("%s: not square (%lld x %lld)", name, (long long)a->nrows,
                  (long long)a->ncols);
        return XAMG_EINVAL;
    }
    if (!a->row_ptr || (a->nnz > 0 && (!a->col || !a->val))) {
        set_error("%s: null array", name);
        return XAMG_EINVAL;
    }
    if (a->row_ptr[0] != 0 || a->row_ptr[a->nrows] != a->nnz) {
        set_error("%s: row_ptr[0] must be 0 and row_ptr[n] = nnz", name);
        return XAMG_EINVAL;
    }
    for (int64_t i = 0; i < a->nrows; ++i) {
        const int32_t b = a->row_ptr[i], e = a->row_ptr[i + 1];
        if (e < b) { set_error("%s: row_ptr decreases at row %lld", name, (long long)i); return XAMG_EINVAL; }
        bool diag = false;
        for (int32_t k = b; k < e; ++k) {
            const int32_t c = a->col[k];
            if (c < 0 || c >= a->ncols) {
                set_error("%s: column %d out of range in row %lld", name, c, (long long)i);
                return XAMG_EINVAL;
            }
            if (k > b && c <= a->col[k - 1]) {
                set_error("%s: columns not strictly increasing in row %lld", name, (long long)i);
                return XAMG_EINVAL;
            }
            if (!std::isfinite(a->val[k])) {
                set_error("%s: non-finite value in row %lld", name, (long long)i);
                return XAMG_EINVAL;
            }
            if (c == i) diag = (a->val[k] != 0.0);
        }
        if (square && !diag) {
            set_error("%s: missing or zero diagonal in row %lld", name, (long long)i);
            return XAMG_EINVAL;
        }
    }
    return XAMG_OK;
}

}  // namespace xamg

extern "C" {

const char* xamg_strerror(int code)
{
    switch (code) {
    case XAMG_OK: return "success";
    case XAMG_NOT_CONVERGED: return "not converged within max_iters";
    case XAMG_EINVAL: return "invalid argument";
    case XAMG_ENOMEM: return "out of memory";
    case XAMG_EHIP: return "HIP runtime error";
    case XAMG_ENODEV: return "no usable gfx950 device";
    case XAMG_EBREAKDOWN: return "breakdown";
    default: return "unknown error code";
    }
}

const char* xamg_last_error(void) { return xamg::last_error(); }

}  // extern "C"
