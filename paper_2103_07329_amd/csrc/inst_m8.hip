// inst_m8.hip -- the solver templates instantiated for M = 8 columns.
#include "bicgstab.hpp"
#include "pbicgstab.hpp"
#include "cycle.hpp"

namespace xamg {

template int vcycle<8>(Handle&, const double*, double*, int, const double*, const float*);
template int pcg<8>(Handle&, const double*, double*, double);
template int mg_solve<8>(Handle&, const double*, double*, double);
template int bicgstab<8>(Handle&, const double*, double*, double);
template int pbicgstab<8>(Handle&, const double*, double*, double);
template void spmm64<8>(Handle&, const DCsr&, const double*, double*);
template void autotune<8>(Handle&);
template void apply_cached_tuning<8>(Handle&);
template void pcg_start<8>(Handle&, const double*, double*, double);
template void pcg_iteration<8>(Handle&, double*);
template void pcg_true_enqueue<8>(Handle&, const double*, double*, int);
template int pcg_true_finish<8>(Handle&);

}  // namespace xamg
