// Instantiations of the row-mode grouped reductions for (DOM_FP, void) (a translation unit of
// its own, so that the instantiations compile in parallel).
#include "rowred_impl.hpp"

namespace ustat {

template hipError_t launch_rowred_dt<DOM_FP, void>(const ColDesc *, int, dim3, int, int, hipStream_t);

}  // namespace ustat
