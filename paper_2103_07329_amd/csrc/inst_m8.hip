// inst_m8.hip -- the solver templates instantiated for M = 8 columns.
#include "bicgstab.hpp"
#include "cycle.hpp"

namespace xamg {

template int vcycle<8>(Handle&, const double*, double*, int, const double*, const float*);
template int pcg<8>(Handle&, const double*, double*, double);
template int mg_solve<8>(Handle&, const double*, double*, double);
template int bicgstab<8>(Handle&, const double*, double*, double);
template void spmm64<8>(Handle&, const DCsr&, const double*, double*);
template void autotune<8>(Handle&);

}  // namespace xamg
