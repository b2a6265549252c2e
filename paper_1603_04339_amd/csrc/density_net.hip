// Learned initial density: a small 3-D convolutional network that maps the
// superposition of atomic densities (the SCF start of Sec. 4) to a correction of
// it, trained on converged plain-SCF densities; forward, backward and Adam are
// the kernels below (FP32 storage and arithmetic, FP64 reductions).
//
//   x = rho_SAD / rho_bar,  u = -V_loc,  d = f_theta(x, u),
//   rho_0 = renorm(relu(x + d - mean(d)) * rho_bar)
//   f_theta: four 3x3x3 periodic convolutions with dilations 1, 2, 4, 8, channels
//   2 -> 16 -> 32 -> 32 -> 1, ReLU after the first three.  The local potential is the
//   second input channel: the atomic superposition does not see the well depths.
//
// Layout: a field of C channels for a batch of B cells is [B][N_d][C] (channels
// fastest, voxel index i + n1 (j + n2 k)).  Weights are stored per layer as
// W[tap][C_in][C_out] (tap = 9 kz + 3 ky + kx reads offset q (kz-1, ky-1, kx-1) for
// dilation q),
// then b[C_out]; the host-side parameter vector uses W[C_out][C_in][kz][ky][kx]
// and is transposed on set/get.
//
// Kernels: one thread per output voxel keeps all C_out sums in registers and
// reads the (wave-uniform) weights through the scalar cache; the input gradient
// is the same kernel with the transposed, mirrored weights and the ReLU mask of
// the layer below fused; weight gradients stage a chunk of voxels of both
// operands in LDS and reduce per (tap, group) into partials that a second pass
// sums in a fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace sparc {

static constexpr int kLayers = 4;
static constexpr int kCh[kLayers + 1] = {2, 16, 32, 32, 1};
static constexpr int kDil[kLayers] = {1, 2, 4, 8};
static constexpr int kGroups = 64;   // weight-gradient partial groups
static constexpr int kChunk = 64;    // voxels staged per weight-gradient iteration
static constexpr int kRedBlocks = 256;

static int64_t layer_w(int l) { return 27LL * kCh[l] * kCh[l + 1]; }
static int64_t layer_off(int l) {
  int64_t o = 0;
  for (int q = 0; q < l; ++q) o += layer_w(q) + kCh[q + 1];
  return o;
}
static int64_t total_params() { return layer_off(kLayers); }

__device__ __forceinline__ int wrapi(int a, int n) { return a < 0 ? a + n : (a >= n ? a - n : a); }

// MODE 0: out = conv + bias; 1: out = relu(conv + bias); 2: out = conv * (mask > 0)
template <int CI, int CO, int MODE>
__global__ __launch_bounds__(256) void conv_kernel(int n1, int n2, int n3, int q, const float* __restrict__ in,
                                                   const float* __restrict__ W, const float* __restrict__ bias,
                                                   const float* __restrict__ mask, float* __restrict__ out) {
  const int64_t V = (int64_t)n1 * n2 * n3;
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= V) return;
  const int64_t b = blockIdx.y;
  const int i = (int)(v % n1), j = (int)((v / n1) % n2), k = (int)(v / ((int64_t)n1 * n2));
  const float* __restrict__ inb = in + b * V * CI;
  float acc[CO];
#pragma unroll
  for (int co = 0; co < CO; ++co) acc[co] = (MODE != 2) ? bias[co] : 0.0f;
  for (int kz = 0; kz < 3; ++kz) {
    const int kk = wrapi(k + q * (kz - 1), n3);
    for (int ky = 0; ky < 3; ++ky) {
      const int jj = wrapi(j + q * (ky - 1), n2);
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int ii = wrapi(i + q * (kx - 1), n1);
        const float* __restrict__ src = inb + (((int64_t)kk * n2 + jj) * n1 + ii) * CI;
        const float* __restrict__ w = W + ((kz * 3 + ky) * 3 + kx) * CI * CO;
        if constexpr (CI % 4 == 0) {
#pragma unroll 2
          for (int c = 0; c < CI; c += 4) {
            const float4 xv = *(const float4*)(src + c);
            const float xs[4] = {xv.x, xv.y, xv.z, xv.w};
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
              for (int co = 0; co < CO; ++co) acc[co] = fmaf(xs[u], w[(c + u) * CO + co], acc[co]);
          }
        } else {
#pragma unroll
          for (int c = 0; c < CI; ++c) {
            const float xv = src[c];
#pragma unroll
            for (int co = 0; co < CO; ++co) acc[co] = fmaf(xv, w[c * CO + co], acc[co]);
          }
        }
      }
    }
  }
  float* __restrict__ o = out + (b * V + v) * CO;
  const float* __restrict__ mk = (MODE == 2) ? mask + (b * V + v) * CO : nullptr;
#pragma unroll
  for (int co = 0; co < CO; ++co) {
    float r = acc[co];
    if (MODE == 1) r = r < 0.0f ? 0.0f : r;   // ReLU that keeps a NaN a NaN
    if (MODE == 2) r = mk[co] > 0.0f ? r : 0.0f;
    acc[co] = r;
  }
  if constexpr (CO % 4 == 0) {
#pragma unroll
    for (int co = 0; co < CO; co += 4) *(float4*)(o + co) = make_float4(acc[co], acc[co + 1], acc[co + 2], acc[co + 3]);
  } else {
#pragma unroll
    for (int co = 0; co < CO; ++co) o[co] = acc[co];
  }
}

// BF16 inference form: activations held as bfloat16 (round-to-nearest-even of the FP32
// value), weights rounded to bfloat16 (kept as FP32 numbers), products and sums in FP32.
__device__ __forceinline__ unsigned short f32_to_bf16(float f) {
  const unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);  // NaN stays NaN
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f32(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

__global__ void to_bf16_kernel(int64_t n, const float* __restrict__ x, unsigned short* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = f32_to_bf16(x[i]);
}

__global__ void round_bf16_kernel(int64_t n, const float* __restrict__ x, float* __restrict__ y) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = bf16_to_f32(f32_to_bf16(x[i]));
}

// conv_kernel with bfloat16 input activations; RELU as MODE 1 of conv_kernel; OUT16:
// the output rounded to bfloat16, else FP32
template <int CI, int CO, bool RELU, bool OUT16>
__global__ __launch_bounds__(256) void conv_bf16_kernel(int n1, int n2, int n3, int q,
                                                        const unsigned short* __restrict__ in,
                                                        const float* __restrict__ W, const float* __restrict__ bias,
                                                        void* __restrict__ out) {
  const int64_t V = (int64_t)n1 * n2 * n3;
  const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (v >= V) return;
  const int64_t b = blockIdx.y;
  const int i = (int)(v % n1), j = (int)((v / n1) % n2), k = (int)(v / ((int64_t)n1 * n2));
  const unsigned short* __restrict__ inb = in + b * V * CI;
  float acc[CO];
#pragma unroll
  for (int co = 0; co < CO; ++co) acc[co] = bias[co];
  for (int kz = 0; kz < 3; ++kz) {
    const int kk = wrapi(k + q * (kz - 1), n3);
    for (int ky = 0; ky < 3; ++ky) {
      const int jj = wrapi(j + q * (ky - 1), n2);
#pragma unroll
      for (int kx = 0; kx < 3; ++kx) {
        const int ii = wrapi(i + q * (kx - 1), n1);
        const unsigned short* __restrict__ src = inb + (((int64_t)kk * n2 + jj) * n1 + ii) * CI;
        const float* __restrict__ w = W + ((kz * 3 + ky) * 3 + kx) * CI * CO;
        if constexpr (CI % 4 == 0) {
#pragma unroll 2
          for (int c = 0; c < CI; c += 4) {
            const uint2 p = *(const uint2*)(src + c);  // four bfloat16 values
            const float xs[4] = {__uint_as_float(p.x << 16), __uint_as_float(p.x & 0xffff0000u),
                                 __uint_as_float(p.y << 16), __uint_as_float(p.y & 0xffff0000u)};
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
              for (int co = 0; co < CO; ++co) acc[co] = fmaf(xs[u], w[(c + u) * CO + co], acc[co]);
          }
        } else {
#pragma unroll
          for (int c = 0; c < CI; ++c) {
            const float xv = bf16_to_f32(src[c]);
#pragma unroll
            for (int co = 0; co < CO; ++co) acc[co] = fmaf(xv, w[c * CO + co], acc[co]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int co = 0; co < CO; ++co)
    if (RELU) acc[co] = acc[co] < 0.0f ? 0.0f : acc[co];   // keeps a NaN a NaN
  if constexpr (OUT16) {
    unsigned short* __restrict__ o = (unsigned short*)out + (b * V + v) * CO;
#pragma unroll
    for (int co = 0; co < CO; ++co) o[co] = f32_to_bf16(acc[co]);
  } else {
    float* __restrict__ o = (float*)out + (b * V + v) * CO;
#pragma unroll
    for (int co = 0; co < CO; ++co) o[co] = acc[co];
  }
}

// WT[26 - t][co][ci] = W[t][ci][co]: the adjoint of a correlation is the correlation
// with the mirrored kernel and the channel roles swapped
__global__ void transpose_w_kernel(int ci_n, int co_n, const float* __restrict__ W, float* __restrict__ WT) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 27 * ci_n * co_n) return;
  const int t = idx / (ci_n * co_n), r = idx % (ci_n * co_n), ci = r / co_n, co = r % co_n;
  WT[((26 - t) * co_n + co) * ci_n + ci] = W[idx];
}

// partial weight gradients: part[g][t][ci*CO + co] = sum over the voxels of group g of
// a(v + offset_t)[ci] * gz(v)[co]
template <int CI, int CO>
__global__ __launch_bounds__(256) void wgrad_kernel(int n1, int n2, int n3, int q, int B, const float* __restrict__ a,
                                                    const float* __restrict__ gz, float* __restrict__ part) {
  constexpr int P = CI * CO;
  constexpr int PPT = (P + 255) / 256;
  __shared__ float xs[kChunk][CI + 1];
  __shared__ float gs[kChunk][CO];
  const int t = blockIdx.x, g = blockIdx.y;
  const int oz = q * (t / 9 - 1), oy = q * ((t / 3) % 3 - 1), ox = q * (t % 3 - 1);
  const int64_t V = (int64_t)n1 * n2 * n3, total = V * B;
  const int64_t nchunks = (total + kChunk - 1) / kChunk;
  float acc[PPT];
#pragma unroll
  for (int u = 0; u < PPT; ++u) acc[u] = 0.0f;
  for (int64_t c = g; c < nchunks; c += gridDim.y) {
    const int64_t base = c * kChunk;
    for (int e = threadIdx.x; e < kChunk * CO; e += 256) {
      const int vv = e / CO, co = e % CO;
      const int64_t gv = base + vv;
      gs[vv][co] = gv < total ? gz[gv * CO + co] : 0.0f;
    }
    for (int e = threadIdx.x; e < kChunk * CI; e += 256) {
      const int vv = e / CI, ci = e % CI;
      const int64_t gv = base + vv;
      float val = 0.0f;
      if (gv < total) {
        const int64_t b = gv / V, v = gv % V;
        const int i = (int)(v % n1), j = (int)((v / n1) % n2), k = (int)(v / ((int64_t)n1 * n2));
        const int64_t src = ((int64_t)wrapi(k + oz, n3) * n2 + wrapi(j + oy, n2)) * n1 + wrapi(i + ox, n1);
        val = a[(b * V + src) * CI + ci];
      }
      xs[vv][ci] = val;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PPT; ++u) {
      const int p = threadIdx.x + 256 * u;
      if (p < P) {
        const int ci = p / CO, co = p % CO;
        float s = acc[u];
        for (int vv = 0; vv < kChunk; ++vv) s = fmaf(xs[vv][ci], gs[vv][co], s);
        acc[u] = s;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < PPT; ++u) {
    const int p = threadIdx.x + 256 * u;
    if (p < P) part[((int64_t)g * 27 + t) * P + p] = acc[u];
  }
}

// gW[t][p] = sum_g part[g][t][p] (fixed order)
__global__ void wgrad_reduce_kernel(int np, int groups, const float* __restrict__ part, float* __restrict__ gW) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= np) return;
  double s = 0.0;
  for (int g = 0; g < groups; ++g) s += part[(int64_t)g * np + idx];
  gW[idx] = (float)s;
}

// bias gradient, partial: bpart[blk][co] = sum over the voxels blk, blk + grid, ... of gz[.][co]
template <int CO>
__global__ __launch_bounds__(256) void bgrad_kernel(int64_t total, const float* __restrict__ gz,
                                                    double* __restrict__ bpart) {
  __shared__ double red[256];
  for (int co = 0; co < CO; ++co) {
    double s = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < total; v += (int64_t)gridDim.x * 256)
      s += gz[v * CO + co];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
      __syncthreads();
    }
    if (threadIdx.x == 0) bpart[blockIdx.x * CO + co] = red[0];
    __syncthreads();
  }
}

// gb[co] = sum over blocks of bpart (fixed order)
__global__ void bgrad_final_kernel(int co_n, int nblk, const double* __restrict__ bpart, float* __restrict__ gb) {
  const int co = threadIdx.x;
  if (co >= co_n) return;
  double s = 0.0;
  for (int k = 0; k < nblk; ++k) s += bpart[k * co_n + co];
  gb[co] = (float)s;
}

// per-sample partial sums of up to two fields: part[(b * nblk + blk) * 2 + q]
__global__ __launch_bounds__(256) void sample_sums_kernel(int64_t V, const float* __restrict__ f0,
                                                          const float* __restrict__ f1, double* __restrict__ part) {
  __shared__ double r0[256], r1[256];
  const int64_t b = blockIdx.y;
  double s0 = 0.0, s1 = 0.0;
  for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < V; v += (int64_t)gridDim.x * 256) {
    s0 += f0[b * V + v];
    if (f1) s1 += f1[b * V + v];
  }
  r0[threadIdx.x] = s0;
  r1[threadIdx.x] = s1;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      r0[threadIdx.x] += r0[threadIdx.x + o];
      r1[threadIdx.x] += r1[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[(b * gridDim.x + blockIdx.x) * 2] = r0[0];
    part[(b * gridDim.x + blockIdx.x) * 2 + 1] = r1[0];
  }
}

// sums[b * 2 + q] = sum over blocks of part (fixed order)
__global__ void sample_sums_final_kernel(int B, int nblk, const double* __restrict__ part, double* __restrict__ sums) {
  const int idx = threadIdx.x;
  if (idx >= 2 * B) return;
  const int b = idx / 2, q = idx % 2;
  double s = 0.0;
  for (int k = 0; k < nblk; ++k) s += part[((int64_t)b * nblk + k) * 2 + q];
  sums[idx] = s;
}

// loss head: s = x + d - mean_b(d), r = s - y (before the ReLU of the prediction, so
// that negative s is penalised); g = 2 r / (B V); writes g and r^2 (for the loss sum)
__global__ void head_loss_kernel(int64_t V, int B, const float* __restrict__ in, const float* __restrict__ d,
                                 const double* __restrict__ dsum, const float* __restrict__ y, float* __restrict__ g,
                                 float* __restrict__ r2) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= V * B) return;
  const int64_t b = idx / V;
  const float mean = (float)(dsum[2 * b] / (double)V);
  const float s = in[idx * 2] + (d[idx] - mean);   // channel 0 of the input: x
  const float r = s - y[idx];
  g[idx] = 2.0f * r / (float)((double)B * V);
  r2[idx] = r * r;
}

// g -= mean_b(g) (gradient through d - mean(d))
__global__ void center_kernel(int64_t V, int B, float* __restrict__ g, const double* __restrict__ gsum) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= V * B) return;
  g[idx] -= (float)(gsum[2 * (idx / V)] / (double)V);
}

// prediction head (one cell): s = x + d - mean(d); rho = relu(s) * rho_bar (FP64)
__global__ void head_predict_kernel(int64_t V, const float* __restrict__ in, const float* __restrict__ d,
                                    const double* __restrict__ dsum, double rho_bar, double* __restrict__ rho,
                                    float* __restrict__ yh, float* __restrict__ sv) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= V) return;
  const float s = in[v * 2] + (d[v] - (float)(dsum[0] / (double)V));
  const float y = s < 0.0f ? 0.0f : s;
  yh[v] = y;
  sv[v] = s;   // summed separately so that a NaN anywhere reaches the host check
  rho[v] = (double)y * rho_bar;
}

__global__ void scale_kernel(int64_t n, double* __restrict__ y, double f) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] *= f;
}

__global__ void to_scaled_f32_kernel(int64_t n, const double* __restrict__ rho, double inv, float* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = (float)(rho[i] * inv);
}

// network input [v][2] = (rho / rho_bar, -V_loc)
__global__ void input_kernel(int64_t n, const double* __restrict__ rho, double inv, const double* __restrict__ vloc,
                             float* __restrict__ in) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    in[2 * i] = (float)(rho[i] * inv);
    in[2 * i + 1] = (float)(-vloc[i]);
  }
}

// Adam (Kingma & Ba) with bias corrections c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t)
__global__ void adam_kernel(int64_t n, float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float c1, float c2, float eps) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

template <int CI, int CO, int MODE>
static int launch_conv(hipStream_t s, int n1, int n2, int n3, int q, int B, const float* in, const float* W,
                       const float* bias, const float* mask, float* out) {
  const int64_t V = (int64_t)n1 * n2 * n3;
  dim3 grid((unsigned)((V + 255) / 256), (unsigned)B);
  conv_kernel<CI, CO, MODE><<<grid, 256, 0, s>>>(n1, n2, n3, q, in, W, bias, mask, out);
  return check_launch("conv_kernel");
}

template <int CI, int CO, bool RELU, bool OUT16>
static int launch_conv_bf16(hipStream_t s, int n1, int n2, int n3, int q, int B, const void* in, const float* W,
                            const float* bias, void* out) {
  const int64_t V = (int64_t)n1 * n2 * n3;
  dim3 grid((unsigned)((V + 255) / 256), (unsigned)B);
  conv_bf16_kernel<CI, CO, RELU, OUT16><<<grid, 256, 0, s>>>(n1, n2, n3, q, (const unsigned short*)in, W, bias, out);
  return check_launch("conv_bf16_kernel");
}

template <int CI, int CO>
static int launch_wgrad(hipStream_t s, int n1, int n2, int n3, int q, int B, const float* a, const float* gz,
                        float* part, double* bpart, float* gW, float* gb) {
  wgrad_kernel<CI, CO><<<dim3(27, kGroups), 256, 0, s>>>(n1, n2, n3, q, B, a, gz, part);
  SPARC_TRY(check_launch("wgrad_kernel"));
  const int np = 27 * CI * CO;
  wgrad_reduce_kernel<<<(np + 255) / 256, 256, 0, s>>>(np, kGroups, part, gW);
  SPARC_TRY(check_launch("wgrad_reduce_kernel"));
  bgrad_kernel<CO><<<kGroups, 256, 0, s>>>((int64_t)n1 * n2 * n3 * B, gz, bpart);
  SPARC_TRY(check_launch("bgrad_kernel"));
  bgrad_final_kernel<<<1, 64, 0, s>>>(CO, kGroups, bpart, gb);
  return check_launch("bgrad_final_kernel");
}

}  // namespace sparc

using namespace sparc;

struct sparc_dnet {
  sparc_ctx* ctx;
  int n[3];
  int64_t V;
  int max_batch;
  float *theta, *grad, *m, *v;
  int adam_t;
  float* a[kLayers + 1];   // a[0]: input copy, a[1..3]: ReLU outputs, a[4]: d
  float* gz[kLayers];      // gz[l]: gradient at the pre-activation of layer l
  float* wt;               // transposed weights of one layer
  float* part;             // weight-gradient partials
  double *rpart, *rsum;    // per-sample reduction partials and sums
  double* bpart;           // bias-gradient partials
  float* r2;               // squared residuals
  int bf16;                // inference precision: 0 FP32, 1 bfloat16 activations and weights
  bool bf_stale;           // theta_bf no longer holds the rounded theta
  float* theta_bf;         // theta rounded to bfloat16 (FP32 numbers)
  std::vector<void*> allocs;
};

namespace sparc {

static int dnet_alloc(sparc_dnet* N, void** p, size_t bytes) {
  *p = nullptr;
  if (hipMalloc(p, std::max<size_t>(bytes, 16)) != hipSuccess)
    return fail(SPARC_ENOMEM, "density net: device allocation of %zu bytes failed", bytes);
  N->allocs.push_back(*p);
  return SPARC_OK;
}

static float* Wl(sparc_dnet* N, float* base, int l) { return base + layer_off(l); }
static float* bl(sparc_dnet* N, float* base, int l) { return base + layer_off(l) + layer_w(l); }

static int dnet_forward(sparc_dnet* N, const float* x, int B, bool bf16 = false) {
  hipStream_t s = N->ctx->stream;
  const int n1 = N->n[0], n2 = N->n[1], n3 = N->n[2];
  if (bf16) {
    const int64_t np = total_params();
    if (N->bf_stale) {
      round_bf16_kernel<<<(unsigned)((np + 255) / 256), 256, 0, s>>>(np, N->theta, N->theta_bf);
      SPARC_TRY(check_launch("round_bf16_kernel"));
      N->bf_stale = false;
    }
    const int64_t ni = (int64_t)B * N->V * kCh[0];
    to_bf16_kernel<<<(unsigned)((ni + 255) / 256), 256, 0, s>>>(ni, x, (unsigned short*)N->a[0]);
    SPARC_TRY(check_launch("to_bf16_kernel"));
    float* T = N->theta_bf;
    SPARC_TRY((launch_conv_bf16<2, 16, true, true>(s, n1, n2, n3, kDil[0], B, N->a[0], Wl(N, T, 0), bl(N, T, 0),
                                                   N->a[1])));
    SPARC_TRY((launch_conv_bf16<16, 32, true, true>(s, n1, n2, n3, kDil[1], B, N->a[1], Wl(N, T, 1), bl(N, T, 1),
                                                    N->a[2])));
    SPARC_TRY((launch_conv_bf16<32, 32, true, true>(s, n1, n2, n3, kDil[2], B, N->a[2], Wl(N, T, 2), bl(N, T, 2),
                                                    N->a[3])));
    return launch_conv_bf16<32, 1, false, false>(s, n1, n2, n3, kDil[3], B, N->a[3], Wl(N, T, 3), bl(N, T, 3),
                                                 N->a[4]);
  }
  SPARC_HIP(hipMemcpyAsync(N->a[0], x, (size_t)B * N->V * kCh[0] * sizeof(float), hipMemcpyDeviceToDevice, s));
  SPARC_TRY((launch_conv<2, 16, 1>(s, n1, n2, n3, kDil[0], B, N->a[0], Wl(N, N->theta, 0), bl(N, N->theta, 0), nullptr,
                                   N->a[1])));
  SPARC_TRY((launch_conv<16, 32, 1>(s, n1, n2, n3, kDil[1], B, N->a[1], Wl(N, N->theta, 1), bl(N, N->theta, 1), nullptr,
                                    N->a[2])));
  SPARC_TRY((launch_conv<32, 32, 1>(s, n1, n2, n3, kDil[2], B, N->a[2], Wl(N, N->theta, 2), bl(N, N->theta, 2), nullptr,
                                    N->a[3])));
  SPARC_TRY((launch_conv<32, 1, 0>(s, n1, n2, n3, kDil[3], B, N->a[3], Wl(N, N->theta, 3), bl(N, N->theta, 3), nullptr,
                                   N->a[4])));
  return SPARC_OK;
}

// per-sample sums of f0 (and f1) into N->rsum[b*2 + q]
static int dnet_sample_sums(sparc_dnet* N, int B, const float* f0, const float* f1) {
  hipStream_t s = N->ctx->stream;
  sample_sums_kernel<<<dim3(kRedBlocks, B), 256, 0, s>>>(N->V, f0, f1, N->rpart);
  SPARC_TRY(check_launch("sample_sums_kernel"));
  sample_sums_final_kernel<<<1, 256, 0, s>>>(B, kRedBlocks, N->rpart, N->rsum);
  return check_launch("sample_sums_final_kernel");
}

static int dnet_backward(sparc_dnet* N, int B) {
  hipStream_t s = N->ctx->stream;
  const int n1 = N->n[0], n2 = N->n[1], n3 = N->n[2];
  auto transpose = [&](int l) -> int {
    const int np = 27 * kCh[l] * kCh[l + 1];
    transpose_w_kernel<<<(np + 255) / 256, 256, 0, s>>>(kCh[l], kCh[l + 1], Wl(N, N->theta, l), N->wt);
    return check_launch("transpose_w_kernel");
  };
  // layer 3 (linear): gz[3] is the head gradient
  SPARC_TRY((launch_wgrad<32, 1>(s, n1, n2, n3, kDil[3], B, N->a[3], N->gz[3], N->part, N->bpart, Wl(N, N->grad, 3),
                                  bl(N, N->grad, 3))));
  SPARC_TRY(transpose(3));
  SPARC_TRY((launch_conv<1, 32, 2>(s, n1, n2, n3, kDil[3], B, N->gz[3], N->wt, nullptr, N->a[3], N->gz[2])));
  SPARC_TRY((launch_wgrad<32, 32>(s, n1, n2, n3, kDil[2], B, N->a[2], N->gz[2], N->part, N->bpart, Wl(N, N->grad, 2),
                                   bl(N, N->grad, 2))));
  SPARC_TRY(transpose(2));
  SPARC_TRY((launch_conv<32, 32, 2>(s, n1, n2, n3, kDil[2], B, N->gz[2], N->wt, nullptr, N->a[2], N->gz[1])));
  SPARC_TRY((launch_wgrad<16, 32>(s, n1, n2, n3, kDil[1], B, N->a[1], N->gz[1], N->part, N->bpart, Wl(N, N->grad, 1),
                                   bl(N, N->grad, 1))));
  SPARC_TRY(transpose(1));
  SPARC_TRY((launch_conv<32, 16, 2>(s, n1, n2, n3, kDil[1], B, N->gz[1], N->wt, nullptr, N->a[1], N->gz[0])));
  SPARC_TRY((launch_wgrad<2, 16>(s, n1, n2, n3, kDil[0], B, N->a[0], N->gz[0], N->part, N->bpart, Wl(N, N->grad, 0),
                                  bl(N, N->grad, 0))));
  return SPARC_OK;
}

// host <-> internal parameter layouts
static void to_internal(const float* pub, std::vector<float>& in) {
  in.assign(total_params(), 0.0f);
  for (int l = 0; l < kLayers; ++l) {
    const int ci_n = kCh[l], co_n = kCh[l + 1];
    const int64_t o = layer_off(l);
    for (int co = 0; co < co_n; ++co)
      for (int ci = 0; ci < ci_n; ++ci)
        for (int t = 0; t < 27; ++t) in[o + ((int64_t)t * ci_n + ci) * co_n + co] = pub[o + ((int64_t)co * ci_n + ci) * 27 + t];
    for (int co = 0; co < co_n; ++co) in[o + layer_w(l) + co] = pub[o + layer_w(l) + co];
  }
}
static void to_public(const float* in, float* pub) {
  for (int l = 0; l < kLayers; ++l) {
    const int ci_n = kCh[l], co_n = kCh[l + 1];
    const int64_t o = layer_off(l);
    for (int co = 0; co < co_n; ++co)
      for (int ci = 0; ci < ci_n; ++ci)
        for (int t = 0; t < 27; ++t) pub[o + ((int64_t)co * ci_n + ci) * 27 + t] = in[o + ((int64_t)t * ci_n + ci) * co_n + co];
    for (int co = 0; co < co_n; ++co) pub[o + layer_w(l) + co] = in[o + layer_w(l) + co];
  }
}

static int check_batch(sparc_dnet* N, int B) {
  if (!N) return fail(SPARC_EINVAL, "density net: NULL handle");
  if (B < 1 || B > N->max_batch) return fail(SPARC_ESHAPE, "density net: batch %d outside 1..%d", B, N->max_batch);
  return SPARC_OK;
}

}  // namespace sparc

extern "C" {

int64_t sparc_dnet_num_params(void) { return total_params(); }

int sparc_dnet_create(sparc_ctx* ctx, const int32_t* n, int32_t max_batch, sparc_dnet** out) {
  if (!ctx || !n || !out) return fail(SPARC_EINVAL, "sparc_dnet_create: null argument");
  *out = nullptr;
  for (int s3 = 0; s3 < 3; ++s3)
    if (n[s3] <= kDil[kLayers - 1] || n[s3] > 1024)
      return fail(SPARC_ESHAPE, "sparc_dnet_create: grid size outside %d..1024", kDil[kLayers - 1] + 1);
  if (max_batch < 1 || max_batch > 128) return fail(SPARC_ESHAPE, "sparc_dnet_create: max_batch outside 1..128");
  sparc_dnet* N = new sparc_dnet();
  N->ctx = ctx;
  for (int s3 = 0; s3 < 3; ++s3) N->n[s3] = n[s3];
  N->V = (int64_t)n[0] * n[1] * n[2];
  N->max_batch = max_batch;
  N->adam_t = 0;
  const size_t np = (size_t)total_params();
  const size_t BV = (size_t)max_batch * N->V;
  int rc = SPARC_OK;
  auto A = [&](void** p, size_t bytes) {
    if (rc == SPARC_OK) rc = dnet_alloc(N, p, bytes);
  };
  A((void**)&N->theta, np * 4);
  A((void**)&N->theta_bf, np * 4);
  N->bf16 = 0;
  N->bf_stale = true;
  A((void**)&N->grad, np * 4);
  A((void**)&N->m, np * 4);
  A((void**)&N->v, np * 4);
  for (int l = 0; l <= kLayers; ++l) A((void**)&N->a[l], BV * kCh[l] * 4);
  for (int l = 0; l < kLayers; ++l) A((void**)&N->gz[l], BV * kCh[l + 1] * 4);
  A((void**)&N->wt, 27 * 32 * 32 * 4);
  A((void**)&N->part, (size_t)kGroups * 27 * 32 * 32 * 4);
  A((void**)&N->rpart, (size_t)max_batch * kRedBlocks * 2 * 8);
  A((void**)&N->rsum, (size_t)std::max(2 * max_batch, 2) * 8);
  A((void**)&N->bpart, (size_t)kGroups * 32 * 8);
  A((void**)&N->r2, BV * 4);
  if (rc == SPARC_OK) {
    hipStream_t s = ctx->stream;
    if (hipMemsetAsync(N->theta, 0, np * 4, s) != hipSuccess || hipMemsetAsync(N->m, 0, np * 4, s) != hipSuccess ||
        hipMemsetAsync(N->v, 0, np * 4, s) != hipSuccess || hipMemsetAsync(N->grad, 0, np * 4, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      rc = fail(SPARC_EDEVICE, "sparc_dnet_create: initialisation failed");
  }
  if (rc != SPARC_OK) {
    sparc_dnet_destroy(N);
    return rc;
  }
  *out = N;
  return SPARC_OK;
}

void sparc_dnet_destroy(sparc_dnet* N) {
  if (!N) return;
  for (void* p : N->allocs) hipFree(p);
  delete N;
}

int sparc_dnet_set_params(sparc_dnet* N, const float* theta) {
  if (!N || !theta) return fail(SPARC_EINVAL, "sparc_dnet_set_params: null argument");
  std::vector<float> in;
  to_internal(theta, in);
  SPARC_HIP(hipStreamSynchronize(N->ctx->stream));
  SPARC_HIP(hipMemcpy(N->theta, in.data(), in.size() * 4, hipMemcpyHostToDevice));
  // a new parameter set restarts the optimiser
  const size_t np = in.size();
  SPARC_HIP(hipMemset(N->m, 0, np * 4));
  SPARC_HIP(hipMemset(N->v, 0, np * 4));
  N->adam_t = 0;
  N->bf_stale = true;
  return SPARC_OK;
}

int sparc_dnet_set_precision(sparc_dnet* N, int32_t bf16) {
  if (!N) return fail(SPARC_EINVAL, "sparc_dnet_set_precision: NULL handle");
  if (bf16 != 0 && bf16 != 1) return fail(SPARC_EINVAL, "sparc_dnet_set_precision: precision must be 0 or 1");
  N->bf16 = bf16;
  return SPARC_OK;
}

int sparc_dnet_get_params(const sparc_dnet* N, float* theta) {
  if (!N || !theta) return fail(SPARC_EINVAL, "sparc_dnet_get_params: null argument");
  std::vector<float> in(total_params());
  SPARC_HIP(hipStreamSynchronize(N->ctx->stream));
  SPARC_HIP(hipMemcpy(in.data(), N->theta, in.size() * 4, hipMemcpyDeviceToHost));
  to_public(in.data(), theta);
  return SPARC_OK;
}

int sparc_dnet_scale_density(sparc_dnet* N, const double* rho_dev, double n_elec, double dV, float* x_dev) {
  if (!N || !rho_dev || !x_dev) return fail(SPARC_EINVAL, "sparc_dnet_scale_density: null argument");
  if (!(n_elec > 0) || !(dV > 0)) return fail(SPARC_EINVAL, "sparc_dnet_scale_density: n_elec, dV must be positive");
  const double rho_bar = n_elec / ((double)N->V * dV);
  to_scaled_f32_kernel<<<(unsigned)((N->V + 255) / 256), 256, 0, N->ctx->stream>>>(N->V, rho_dev, 1.0 / rho_bar, x_dev);
  return check_launch("to_scaled_f32_kernel");
}

int sparc_dnet_prepare_input(sparc_dnet* N, const double* rho_dev, const double* vloc_dev, double n_elec, double dV,
                             float* in_dev) {
  if (!N || !rho_dev || !vloc_dev || !in_dev) return fail(SPARC_EINVAL, "sparc_dnet_prepare_input: null argument");
  if (!(n_elec > 0) || !(dV > 0)) return fail(SPARC_EINVAL, "sparc_dnet_prepare_input: n_elec, dV must be positive");
  const double rho_bar = n_elec / ((double)N->V * dV);
  input_kernel<<<(unsigned)((N->V + 255) / 256), 256, 0, N->ctx->stream>>>(N->V, rho_dev, 1.0 / rho_bar, vloc_dev, in_dev);
  return check_launch("input_kernel");
}

int sparc_dnet_forward(sparc_dnet* N, const float* x_dev, int32_t B, float* d_dev) {
  SPARC_TRY(check_batch(N, B));
  if (!x_dev || !d_dev) return fail(SPARC_EINVAL, "sparc_dnet_forward: null argument");
  SPARC_TRY(dnet_forward(N, x_dev, B, N->bf16 != 0));
  SPARC_HIP(hipMemcpyAsync(d_dev, N->a[4], (size_t)B * N->V * 4, hipMemcpyDeviceToDevice, N->ctx->stream));
  return SPARC_OK;
}

int sparc_dnet_loss_grad(sparc_dnet* N, const float* x_dev, const float* y_dev, int32_t B, double* loss,
                         float* grad_host) {
  SPARC_TRY(check_batch(N, B));
  if (!x_dev || !y_dev || !loss) return fail(SPARC_EINVAL, "sparc_dnet_loss_grad: null argument");
  hipStream_t s = N->ctx->stream;
  const int64_t BV = (int64_t)B * N->V;
  SPARC_TRY(dnet_forward(N, x_dev, B));
  SPARC_TRY(dnet_sample_sums(N, B, N->a[4], nullptr));
  head_loss_kernel<<<(unsigned)((BV + 255) / 256), 256, 0, s>>>(N->V, B, N->a[0], N->a[4], N->rsum, y_dev, N->gz[3],
                                                                 N->r2);
  SPARC_TRY(check_launch("head_loss_kernel"));
  SPARC_TRY(dnet_sample_sums(N, B, N->gz[3], N->r2));
  center_kernel<<<(unsigned)((BV + 255) / 256), 256, 0, s>>>(N->V, B, N->gz[3], N->rsum);
  SPARC_TRY(check_launch("center_kernel"));
  std::vector<double> sums(2 * B);
  SPARC_HIP(hipMemcpyAsync(sums.data(), N->rsum, 2 * B * 8, hipMemcpyDeviceToHost, s));
  SPARC_TRY(dnet_backward(N, B));
  SPARC_HIP(hipStreamSynchronize(s));
  double tot = 0.0;
  for (int b = 0; b < B; ++b) tot += sums[2 * b + 1];
  *loss = tot / (double)BV;
  if (grad_host) {
    std::vector<float> in(total_params());
    SPARC_HIP(hipMemcpy(in.data(), N->grad, in.size() * 4, hipMemcpyDeviceToHost));
    to_public(in.data(), grad_host);
  }
  if (!std::isfinite(*loss)) return fail(SPARC_ENAN, "sparc_dnet_loss_grad: non-finite loss");
  return SPARC_OK;
}

int sparc_dnet_adam_step(sparc_dnet* N, double lr) {
  if (!N) return fail(SPARC_EINVAL, "sparc_dnet_adam_step: NULL handle");
  if (!(lr > 0)) return fail(SPARC_EINVAL, "sparc_dnet_adam_step: lr must be positive");
  const double b1 = 0.9, b2 = 0.999;
  N->adam_t += 1;
  const double c1 = 1.0 / (1.0 - std::pow(b1, N->adam_t)), c2 = 1.0 / (1.0 - std::pow(b2, N->adam_t));
  const int64_t np = total_params();
  N->bf_stale = true;
  adam_kernel<<<(unsigned)((np + 255) / 256), 256, 0, N->ctx->stream>>>(np, N->theta, N->grad, N->m, N->v, (float)lr,
                                                                         (float)b1, (float)b2, (float)c1, (float)c2, 1e-8f);
  return check_launch("adam_kernel");
}

int sparc_dnet_train_step(sparc_dnet* N, const float* x_dev, const float* y_dev, int32_t B, double lr, double* loss) {
  SPARC_TRY(sparc_dnet_loss_grad(N, x_dev, y_dev, B, loss, nullptr));
  return sparc_dnet_adam_step(N, lr);
}

int sparc_dnet_predict_density(sparc_dnet* N, const double* rho_sad_dev, const double* vloc_dev, double n_elec,
                               double dV, double charge_tol, double* rho_dev, int32_t* used_net) {
  if (!N || !rho_sad_dev || !vloc_dev || !rho_dev || !used_net)
    return fail(SPARC_EINVAL, "sparc_dnet_predict_density: null argument");
  if (!(n_elec > 0) || !(dV > 0) || !(charge_tol > 0))
    return fail(SPARC_EINVAL, "sparc_dnet_predict_density: n_elec, dV and charge_tol must be positive");
  hipStream_t s = N->ctx->stream;
  const int64_t V = N->V;
  const double rho_bar = n_elec / ((double)V * dV);
  float* in = N->gz[1];   // scratch: one cell, two channels
  SPARC_TRY(sparc_dnet_prepare_input(N, rho_sad_dev, vloc_dev, n_elec, dV, in));
  SPARC_TRY(dnet_forward(N, in, 1, N->bf16 != 0));
  SPARC_TRY(dnet_sample_sums(N, 1, N->a[4], nullptr));
  float* yh = N->r2;
  float* sv = N->gz[2];
  // the head adds the correction to the FP32 input (in either precision of the network)
  head_predict_kernel<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(V, in, N->a[4], N->rsum, rho_bar, rho_dev, yh, sv);
  SPARC_TRY(check_launch("head_predict_kernel"));
  SPARC_TRY(dnet_sample_sums(N, 1, yh, sv));
  double sums[2];
  SPARC_HIP(hipMemcpyAsync(sums, N->rsum, 16, hipMemcpyDeviceToHost, s));
  SPARC_HIP(hipStreamSynchronize(s));
  const double charge = sums[0] * rho_bar * dV;
  if (!std::isfinite(sums[0]) || !std::isfinite(sums[1]) || !(std::fabs(charge - n_elec) <= charge_tol * n_elec)) {
    // fallback: the atomic superposition itself
    SPARC_HIP(hipMemcpyAsync(rho_dev, rho_sad_dev, V * 8, hipMemcpyDeviceToDevice, s));
    SPARC_HIP(hipStreamSynchronize(s));
    *used_net = 0;
    return SPARC_OK;
  }
  scale_kernel<<<(unsigned)((V + 255) / 256), 256, 0, s>>>(V, rho_dev, n_elec / charge);
  SPARC_TRY(check_launch("scale_kernel"));
  SPARC_HIP(hipStreamSynchronize(s));
  *used_net = 1;
  return SPARC_OK;
}

}  // extern "C"
