// inst_m16.hip -- the solver templates instantiated for M = 16 columns.
#include "bicgstab.hpp"
#include "pbicgstab.hpp"
#include "cycle.hpp"

namespace xamg {

template int vcycle<16>(Handle&, const double*, double*, int, const double*, const float*);
template int pcg<16>(Handle&, const double*, double*, double);
template int mg_solve<16>(Handle&, const double*, double*, double);
template int bicgstab<16>(Handle&, const double*, double*, double);
template int pbicgstab<16>(Handle&, const double*, double*, double);
template void spmm64<16>(Handle&, const DCsr&, const double*, double*);
template void autotune<16>(Handle&);
template void apply_cached_tuning<16>(Handle&);
template void pcg_start<16>(Handle&, const double*, double*, double);
template void pcg_iteration<16>(Handle&, double*);
template void pcg_true_enqueue<16>(Handle&, const double*, double*, int);
template int pcg_true_finish<16>(Handle&);

}  // namespace xamg
