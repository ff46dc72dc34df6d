// inst_m2.hip -- the solver templates instantiated for M = 2 columns.
#include "bicgstab.hpp"
#include "pbicgstab.hpp"
#include "cycle.hpp"

namespace xamg {

template int vcycle<2>(Handle&, const double*, double*, int, const double*, const float*);
template int pcg<2>(Handle&, const double*, double*, double);
template int mg_solve<2>(Handle&, const double*, double*, double);
template int bicgstab<2>(Handle&, const double*, double*, double);
template int pbicgstab<2>(Handle&, const double*, double*, double);
template void spmm64<2>(Handle&, const DCsr&, const double*, double*);
template void autotune<2>(Handle&);
template void apply_cached_tuning<2>(Handle&);
template void pcg_start<2>(Handle&, const double*, double*, double);
template void pcg_iteration<2>(Handle&, double*);
template void pcg_true_enqueue<2>(Handle&, const double*, double*, int);
template int pcg_true_finish<2>(Handle&);

}  // namespace xamg
