// Device arithmetic on the four orbital element types (double, float and their
// complex forms stored as interleaved (re, im)).
#pragma once
#include "internal.hpp"

namespace sparc {

template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
template <typename T>
__host__ __device__ __forceinline__ cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

template <typename E> __device__ __forceinline__ E zero();
template <> __device__ __forceinline__ double zero<double>() { return 0.0; }
template <> __device__ __forceinline__ float zero<float>() { return 0.0f; }
template <> __device__ __forceinline__ cd zero<cd>() { return {0.0, 0.0}; }
template <> __device__ __forceinline__ cf zero<cf>() { return {0.0f, 0.0f}; }

// acc + w * v with a real weight w
__device__ __forceinline__ double fmar(double acc, double w, double v) { return fma(w, v, acc); }
__device__ __forceinline__ float fmar(float acc, float w, float v) { return fmaf(w, v, acc); }
__device__ __forceinline__ cd fmar(cd acc, double w, cd v) { return {fma(w, v.re, acc.re), fma(w, v.im, acc.im)}; }
__device__ __forceinline__ cf fmar(cf acc, float w, cf v) { return {fmaf(w, v.re, acc.re), fmaf(w, v.im, acc.im)}; }

// acc + a * b (element product)
__device__ __forceinline__ double fmae(double acc, double a, double b) { return fma(a, b, acc); }
__device__ __forceinline__ float fmae(float acc, float a, float b) { return fmaf(a, b, acc); }
__device__ __forceinline__ cd fmae(cd acc, cd a, cd b) {
  return {fma(a.re, b.re, fma(-a.im, b.im, acc.re)), fma(a.re, b.im, fma(a.im, b.re, acc.im))};
}
__device__ __forceinline__ cf fmae(cf acc, cf a, cf b) {
  return {fmaf(a.re, b.re, fmaf(-a.im, b.im, acc.re)), fmaf(a.re, b.im, fmaf(a.im, b.re, acc.im))};
}

// acc + conj(a) * b
__device__ __forceinline__ double fmac(double acc, double a, double b) { return fma(a, b, acc); }
__device__ __forceinline__ float fmac(float acc, float a, float b) { return fmaf(a, b, acc); }
__device__ __forceinline__ cd fmac(cd acc, cd a, cd b) {
  return {fma(a.re, b.re, fma(a.im, b.im, acc.re)), fma(a.re, b.im, fma(-a.im, b.re, acc.im))};
}
__device__ __forceinline__ cf fmac(cf acc, cf a, cf b) {
  return {fmaf(a.re, b.re, fmaf(a.im, b.im, acc.re)), fmaf(a.re, b.im, fmaf(-a.im, b.re, acc.im))};
}

__device__ __forceinline__ double scale(double s, double v) { return s * v; }
__device__ __forceinline__ float scale(float s, float v) { return s * v; }
__device__ __forceinline__ cd scale(double s, cd v) { return {s * v.re, s * v.im}; }
__device__ __forceinline__ cf scale(float s, cf v) { return {s * v.re, s * v.im}; }

// multiply by the unit phase (c, s) = e^{i theta}; identity for real types
__device__ __forceinline__ double rot(double v, double, double) { return v; }
__device__ __forceinline__ float rot(float v, float, float) { return v; }
__device__ __forceinline__ cd rot(cd v, double c, double s) { return {c * v.re - s * v.im, c * v.im + s * v.re}; }
__device__ __forceinline__ cf rot(cf v, float c, float s) { return {c * v.re - s * v.im, c * v.im + s * v.re}; }

__device__ __forceinline__ double abs2(double v) { return v * v; }
__device__ __forceinline__ double abs2(float v) { return (double)v * (double)v; }
__device__ __forceinline__ double abs2(cd v) { return v.re * v.re + v.im * v.im; }
__device__ __forceinline__ double abs2(cf v) { return (double)v.re * v.re + (double)v.im * v.im; }

// streaming (non-temporal) loads and stores
__device__ __forceinline__ double nt_load(const double* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float nt_load(const float* p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ cd nt_load(const cd* p) {
  const double* q = (const double*)p;
  return {__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1)};
}
__device__ __forceinline__ cf nt_load(const cf* p) {
  const float* q = (const float*)p;
  return {__builtin_nontemporal_load(q), __builtin_nontemporal_load(q + 1)};
}
__device__ __forceinline__ void nt_store(double v, double* p) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void nt_store(float v, float* p) { __builtin_nontemporal_store(v, p); }
__device__ __forceinline__ void nt_store(cd v, cd* p) {
  double* q = (double*)p;
  __builtin_nontemporal_store(v.re, q);
  __builtin_nontemporal_store(v.im, q + 1);
}
__device__ __forceinline__ void nt_store(cf v, cf* p) {
  float* q = (float*)p;
  __builtin_nontemporal_store(v.re, q);
  __builtin_nontemporal_store(v.im, q + 1);
}

// atomic add into work-group (LDS) memory: each real component separately
__device__ __forceinline__ void lds_add(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(float* p, float v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(cd* p, cd v) {
  lds_add(&p->re, v.re);
  lds_add(&p->im, v.im);
}
__device__ __forceinline__ void lds_add(cf* p, cf v) {
  lds_add(&p->re, v.re);
  lds_add(&p->im, v.im);
}

// wave64 butterfly sum
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// DPP move of a double across lanes (CTRL: a DPP_* control word; all lanes active)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}
// Sum over the 64 lanes of a wave (all lanes active), the same value on every lane:
// quad sums (quad_perm [1,0,3,2], [2,3,0,1]), row sums (row_ror 4, 8), then the four
// row sums read from lanes 0, 16, 32, 48.  Register-only, unlike the LDS permutes of
// wave_sum.
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_f64<0xB1>(v);
  v += dpp_f64<0x4E>(v);
  v += dpp_f64<0x124>(v);
  v += dpp_f64<0x128>(v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// K sums over a grid of 256-thread blocks in one launch: every block stores its K partial
// sums (part[k * cap + block], gridDim.x <= cap); the last block to take a ticket (the
// word after the K * cap partials, device-scope release/acquire, zero between launches)
// adds the partials in block order, writes out[0 .. K-1] and resets the ticket.  The
// partials are read with device-scope loads, past any stale L1 line.
template <int K>
__device__ void finish_sums(double (&s)[K], double* part, int cap, double* __restrict__ out) {
  __shared__ double red[K][4];
  __shared__ int last;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double v = wave_sum_dpp(s[k]);
    if (lane == 0) red[k][wv] = v;
  }
  __syncthreads();
  unsigned* ticket = (unsigned*)(part + (size_t)K * cap);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      __hip_atomic_store(&part[(size_t)k * cap + blockIdx.x], red[k][0] + red[k][1] + red[k][2] + red[k][3],
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = (t == gridDim.x - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!last) return;
  double t2[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    t2[k] = 0;
    for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x)
      t2[k] += __hip_atomic_load(&part[(size_t)k * cap + i], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    t2[k] = wave_sum_dpp(t2[k]);
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (lane == 0) red[k][wv] = t2[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) out[k] = red[k][0] + red[k][1] + red[k][2] + red[k][3];
    __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__device__ __forceinline__ int floordiv_i(int a, int b) {
  int q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

}  // namespace sparc
