// inst_m1.hip -- the solver templates instantiated for M = 1 columns.
#include "bicgstab.hpp"
#include "pbicgstab.hpp"
#include "cycle.hpp"

namespace xamg {

template int vcycle<1>(Handle&, const double*, double*, int, const double*, const float*);
template int pcg<1>(Handle&, const double*, double*, double);
template int mg_solve<1>(Handle&, const double*, double*, double);
template int bicgstab<1>(Handle&, const double*, double*, double);
template int pbicgstab<1>(Handle&, const double*, double*, double);
template void spmm64<1>(Handle&, const DCsr&, const double*, double*);
template void autotune<1>(Handle&);
template void apply_cached_tuning<1>(Handle&);
template void pcg_start<1>(Handle&, const double*, double*, double);
template void pcg_iteration<1>(Handle&, double*);
template void pcg_true_enqueue<1>(Handle&, const double*, double*, int);
template int pcg_true_finish<1>(Handle&);

}  // namespace xamg
