// Stencil step kernels for element type float.
#include "hstep_impl.hpp"

namespace sparc {
template int hstep_single<float>(sparc_ctx*, StepArgs<float>&, int32_t, int, int);
template int hstep_batched<float>(sparc_ctx*, const void*, const int*, int, int64_t, int, int, int, size_t);
}  // namespace sparc
