// inst_m16.hip -- the solver templates instantiated for M = 16 columns.
#include "bicgstab.hpp"
#include "cycle.hpp"

namespace xamg {

template int vcycle<16>(Handle&, const double*, double*, int, const double*, const float*);
template int pcg<16>(Handle&, const double*, double*, double);
template int mg_solve<16>(Handle&, const double*, double*, double);
template int bicgstab<16>(Handle&, const double*, double*, double);
template void spmm64<16>(Handle&, const DCsr&, const double*, double*);
template void autotune<16>(Handle&);

}  // namespace xamg
