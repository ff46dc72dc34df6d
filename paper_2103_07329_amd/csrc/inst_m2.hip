// inst_m2.hip -- the solver templates instantiated for M = 2 columns.
#include "bicgstab.hpp"
#include "cycle.hpp"

namespace xamg {

template int vcycle<2>(Handle&, const double*, double*, int, const double*, const float*);
template int pcg<2>(Handle&, const double*, double*, double);
template int mg_solve<2>(Handle&, const double*, double*, double);
template int bicgstab<2>(Handle&, const double*, double*, double);
template void spmm64<2>(Handle&, const DCsr&, const double*, double*);
template void autotune<2>(Handle&);

}  // namespace xamg
