// bicgstab.hip -- right-preconditioned BiCGStab driver (placeholder until
// the BiCGStab kernels land; reports EINVAL).
#include "solver.hpp"

namespace xamg {

template <int M>
int bicgstab(Handle&, const double*, double*, double)
{
    set_error("BiCGStab not available in this build");
    return XAMG_EINVAL;
}

template int bicgstab<1>(Handle&, const double*, double*, double);
template int bicgstab<2>(Handle&, const double*, double*, double);
template int bicgstab<4>(Handle&, const double*, double*, double);
template int bicgstab<8>(Handle&, const double*, double*, double);
template int bicgstab<16>(Handle&, const double*, double*, double);
template int bicgstab<32>(Handle&, const double*, double*, double);

}  // namespace xamg
