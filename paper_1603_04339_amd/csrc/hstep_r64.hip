// Stencil step kernels for element type double.
#include "hstep_impl.hpp"

namespace sparc {
template int hstep_single<double>(sparc_ctx*, StepArgs<double>&, int32_t, int, int);
template int hstep_batched<double>(sparc_ctx*, const void*, const int*, int, int64_t, int, int, int, size_t);
}  // namespace sparc
