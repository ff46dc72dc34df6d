// internal.h -- shared declarations inside libxamg (not part of the ABI).
#pragma once

#include <cstdarg>
#include <cstdint>
#include <cstdio>

#include "xamg.h"

namespace xamg {

// thread-local detail string of the last error
void set_error(const char* fmt, ...);
void clear_error();
const char* last_error();

inline int fail(int code, const char* msg)
{
    set_error("%s", msg);
    return code;
}

// Structural validation of a host CSR (sizes, monotone row_ptr, sorted
// in-range columns, finite values; `square` also requires the diagonal).
int validate_csr(const xamg_csr_t* a, bool square, const char* name);

struct HostHierarchy;
int build_hierarchy(const xamg_csr_t* a0, const xamg_setup_params_t* prm,
                    HostHierarchy** out);
void view_hierarchy(const HostHierarchy* h, xamg_hierarchy_t* v);
int hierarchy_cf(const HostHierarchy* h, int level, int8_t* out);
void free_hierarchy(HostHierarchy* h);

// inverse of a dense row-major n x n matrix via LU with partial pivoting
int dense_inverse(int n, const double* a, double* inv);

}  // namespace xamg
