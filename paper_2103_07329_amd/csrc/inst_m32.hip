// inst_m32.hip -- the solver templates instantiated for M = 32 columns.
#include "bicgstab.hpp"
#include "pbicgstab.hpp"
#include "cycle.hpp"

namespace xamg {

template int vcycle<32>(Handle&, const double*, double*, int, const double*, const float*);
template int pcg<32>(Handle&, const double*, double*, double);
template int mg_solve<32>(Handle&, const double*, double*, double);
template int bicgstab<32>(Handle&, const double*, double*, double);
template int pbicgstab<32>(Handle&, const double*, double*, double);
template void spmm64<32>(Handle&, const DCsr&, const double*, double*);
template void autotune<32>(Handle&);
template void apply_cached_tuning<32>(Handle&);
template void pcg_start<32>(Handle&, const double*, double*, double);
template void pcg_iteration<32>(Handle&, double*);
template void pcg_true_enqueue<32>(Handle&, const double*, double*, int);
template int pcg_true_finish<32>(Handle&);

}  // namespace xamg
