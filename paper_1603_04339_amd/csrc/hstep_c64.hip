// Stencil step kernels for element type cf.
#include "hstep_impl.hpp"

namespace sparc {
template int hstep_single<cf>(sparc_ctx*, StepArgs<cf>&, int32_t, int, int);
template int hstep_batched<cf>(sparc_ctx*, const void*, const int*, int, int64_t, int, int, int, size_t);
}  // namespace sparc
