// Stencil step kernels for element type cd.
#include "hstep_impl.hpp"

namespace sparc {
template int hstep_single<cd>(sparc_ctx*, StepArgs<cd>&, int32_t, int, int);
template int hstep_batched<cd>(sparc_ctx*, const void*, const int*, int, int64_t, int, int, int, size_t);
}  // namespace sparc
