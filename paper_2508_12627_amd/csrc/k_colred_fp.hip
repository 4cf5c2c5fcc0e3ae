// Instantiations of the column-mode grouped reductions for (DOM_FP, float), (DOM_FP, double) (a translation unit of
// its own, so that the instantiations compile in parallel).
#include "colred_impl.hpp"

namespace ustat {

template hipError_t launch_colred_dt<DOM_FP, float>(const ColDesc *, int, dim3, int, int, hipStream_t);
template hipError_t launch_colred_dt<DOM_FP, double>(const ColDesc *, int, dim3, int, int, hipStream_t);

}  // namespace ustat
