// inst_m4.hip -- the solver templates instantiated for M = 4 columns.
#include "bicgstab.hpp"
#include "pbicgstab.hpp"
#include "cycle.hpp"

namespace xamg {

template int vcycle<4>(Handle&, const double*, double*, int, const double*, const float*);
template int pcg<4>(Handle&, const double*, double*, double);
template int mg_solve<4>(Handle&, const double*, double*, double);
template int bicgstab<4>(Handle&, const double*, double*, double);
template int pbicgstab<4>(Handle&, const double*, double*, double);
template void spmm64<4>(Handle&, const DCsr&, const double*, double*);
template void autotune<4>(Handle&);
template void apply_cached_tuning<4>(Handle&);
template void pcg_start<4>(Handle&, const double*, double*, double);
template void pcg_iteration<4>(Handle&, double*);
template void pcg_true_enqueue<4>(Handle&, const double*, double*, int);
template int pcg_true_finish<4>(Handle&);

}  // namespace xamg
