// Measurement helper: the streaming rate of the Chebyshev recurrence's memory pattern
// on its own (two reads and one write per element, no stencil), the practical ceiling
// against which the stencil step's HBM rate is judged.
#include "devmath.hpp"

namespace sparc {

typedef double v2d __attribute__((ext_vector_type(2)));

// c = 2 a - b over n2 pairs of doubles: one 16-byte element per thread, all loads and the
// store non-temporal, one pass (a work-group per 256 pairs).  On MI355X this one-shot form
// streams faster than grid-stride loops over a persistent grid (6.4 against 5.3 TB/s
// over a 3.6 GB operand), so it is the ceiling reported.
__global__ __launch_bounds__(256) void stream_triad_kernel(const v2d* __restrict__ a, const v2d* __restrict__ b,
                                                           v2d* __restrict__ c, int64_t n2) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i < n2) {
    const v2d x = __builtin_nontemporal_load(&a[i]), y = __builtin_nontemporal_load(&b[i]);
    __builtin_nontemporal_store(2.0 * x - y, &c[i]);
  }
}

}  // namespace sparc

using namespace sparc;

extern "C" int sparc_stream_triad(sparc_ctx* ctx, const double* a, const double* b, double* c, int64_t n,
                                  int32_t reps, double* ms_per_launch) {
  if (!ctx || !a || !b || !c || !ms_per_launch) return fail(SPARC_EINVAL, "sparc_stream_triad: null argument");
  if (n < 2 || n % 2 != 0 || reps < 1) return fail(SPARC_EINVAL, "sparc_stream_triad: n even >= 2 and reps >= 1");
  if (((uintptr_t)a | (uintptr_t)b | (uintptr_t)c) % 16 != 0)
    return fail(SPARC_EINVAL, "sparc_stream_triad: buffers must be 16-byte aligned");
  const int64_t blocks = (n / 2 + 255) / 256;
  if (blocks > (int64_t)UINT32_MAX) return fail(SPARC_ESHAPE, "sparc_stream_triad: n too large");
  const unsigned grid = (unsigned)blocks;
  hipEvent_t e0, e1;
  SPARC_HIP(hipEventCreate(&e0));
  SPARC_HIP(hipEventCreate(&e1));
  const v2d* va = (const v2d*)a;
  const v2d* vb = (const v2d*)b;
  v2d* vc = (v2d*)c;
  stream_triad_kernel<<<grid, 256, 0, ctx->stream>>>(va, vb, vc, n / 2);  // warm-up
  hipEventRecord(e0, ctx->stream);
  for (int r = 0; r < reps; ++r) stream_triad_kernel<<<grid, 256, 0, ctx->stream>>>(va, vb, vc, n / 2);
  hipEventRecord(e1, ctx->stream);
  int rc = check_launch("stream_triad_kernel");
  hipEventSynchronize(e1);
  float ms = 0;
  hipEventElapsedTime(&ms, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  *ms_per_launch = ms / reps;
  return rc;
}
