// Instantiates the l1 filtering kernels of one tile class PT (given as
// -DRPCA_PT=<n> by the build) for every rank class; the build compiles this
// file once per PT so the instantiations compile in parallel.
#include "filter_kernel.h"

#ifndef RPCA_PT
#error "compile with -DRPCA_PT=<tile count>"
#endif

namespace filterk {
template int launch_filter_pt<RPCA_PT>(rpca_ctx *, int, const FilterLaunch &, int, bool, hipStream_t);
}
