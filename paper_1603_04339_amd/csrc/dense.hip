// Dense FP64 linear algebra on the N_s x N_s subspace matrices of the
// Rayleigh-Ritz step, all on the GPU:
//   * column-scaled Cholesky factorisation and triangular inverse (the
//     orthonormalising transform of a Cholesky-QR pass);
//   * Hermitian eigensolver: Householder reduction to a real symmetric
//     tridiagonal (blocked: one work-group per 32-column panel, the trailing
//     update on many work-groups; matrix resident in L2), eigenvalues by Sturm
//     multisection (one wave per eigenvalue, 64 Sturm counts per round),
//     eigenvectors by inverse iteration with pivoted tridiagonal LU (one 64-lane
//     work-group per cluster of close eigenvalues, the factorisation on lane 0 with
//     its factors in LDS, Gram-Schmidt inside a cluster), and the
//     back-transformation by the Householder reflectors (one wave per column).
// Matrices are column-major with leading dimension n; complex matrices are
// interleaved (re, im).
#include <algorithm>
#include <cmath>

#include "devmath.hpp"

namespace sparc {

template <bool C> struct scal;
template <> struct scal<false> { typedef double t; };
template <> struct scal<true> { typedef cd t; };

__device__ __forceinline__ double conj_(double v) { return v; }
__device__ __forceinline__ cd conj_(cd v) { return {v.re, -v.im}; }
__device__ __forceinline__ double re_(double v) { return v; }
__device__ __forceinline__ double re_(cd v) { return v.re; }
__device__ __forceinline__ double mk(double r, double) { return r; }
template <typename T> __device__ __forceinline__ T mkT(double r, double i);
template <> __device__ __forceinline__ double mkT<double>(double r, double) { return r; }
template <> __device__ __forceinline__ cd mkT<cd>(double r, double i) { return {r, i}; }
__device__ __forceinline__ double mul_(double a, double b) { return a * b; }
__device__ __forceinline__ cd mul_(cd a, cd b) { return a * b; }
__device__ __forceinline__ double sub_(double a, double b) { return a - b; }
__device__ __forceinline__ cd sub_(cd a, cd b) { return a - b; }
__device__ __forceinline__ double add_(double a, double b) { return a + b; }
__device__ __forceinline__ cd add_(cd a, cd b) { return a + b; }
__device__ __forceinline__ double rscale(double s, double v) { return s * v; }
__device__ __forceinline__ cd rscale(double s, cd v) { return {s * v.re, s * v.im}; }

// block-wide sum of a double (blockDim multiple of 64, <= 1024), the same on every thread
__device__ double block_sum(double v, double* sh) {
  v = wave_sum_dpp(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0;
  for (int i = 0; i < nw; ++i) s += sh[i];
  __syncthreads();
  return s;
}

// ------------------------------------------------------------ scaled Cholesky (blocked)
// S = D^{-1} M D^{-1} + shift I (D = sqrt(diag M)); then S = R^H R (upper) by a
// right-looking blocked factorisation with 64-column panels: the diagonal block is
// factorised in LDS by one work-group, the row panel R12 = R11^{-H} S12 is formed by
// one work-group per 64 columns, and the trailing update S22 -= R12^H R12 runs on
// one work-group per 64 x 64 upper tile.  The inverse of R is then formed by columns
// with the kept diagonal-block inverses.  info = failing column + 1 (0: success);
// every kernel returns early once info is set.
constexpr int CB = 64;

template <typename T>
__global__ __launch_bounds__(256) void chol_scale_kernel(int n, const T* __restrict__ M, T* __restrict__ S,
                                                         double* __restrict__ dinv, double shift, double min_rel_diag,
                                                         int* info) {
  // one work-group per column j; every work-group checks the diagonal itself
  __shared__ int s_fail;
  __shared__ double s_red[4];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int j = blockIdx.x;
  double dm = 0;
  for (int i = tid; i < n; i += blockDim.x) dm = fmax(dm, re_(M[i + (int64_t)i * n]));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o, 64));
  if (lane == 0) s_red[wv] = dm;
  if (tid == 0) s_fail = 0x7fffffff;
  __syncthreads();
  const double dmax = fmax(fmax(s_red[0], s_red[1]), fmax(s_red[2], s_red[3]));
  for (int i = tid; i < n; i += blockDim.x) {
    double d = re_(M[i + (int64_t)i * n]);
    if (!(d > 0.0) || !isfinite(d) || d < min_rel_diag * dmax) atomicMin(&s_fail, i + 1);
    if (j == 0) dinv[i] = (d > 0.0) ? 1.0 / sqrt(d) : 0.0;
  }
  __syncthreads();
  if (j == 0 && tid == 0) *info = (s_fail != 0x7fffffff) ? s_fail : 0;
  if (s_fail != 0x7fffffff) return;
  const double dj = 1.0 / sqrt(re_(M[j + (int64_t)j * n]));
  for (int i = tid; i < n; i += blockDim.x) {
    const double di = 1.0 / sqrt(re_(M[i + (int64_t)i * n]));
    T v = rscale(di * dj, M[i + (int64_t)j * n]);
    if (i == j) v = mkT<T>(re_(v) + shift, 0.0);
    S[i + (int64_t)j * n] = v;
  }
}

// factor the diagonal block S[k0:k0+kb, k0:k0+kb] in LDS; also R11^{-1} -> Rinv (kb x kb).
// Right-looking elimination on unscaled rows: step k subtracts conj(a_ki) a_kj / a_kk from
// the trailing block, so row k (final after step k - 1) is only read during the step and
// one barrier per step suffices; the rows are scaled by 1 / sqrt(a_kk) at the end.  The
// inverse of the triangular factor is formed by 16 x 16 blocks.
template <typename T>
__global__ __launch_bounds__(256) void chol_diag_kernel(int n, T* __restrict__ S, int k0, int kb,
                                                        T* __restrict__ Rinv, int* info) {
  constexpr int LD = CB + 1;   // padded: column-strided accesses spread over the banks
  __shared__ T a[CB * LD];
  __shared__ T r[CB * LD];
  __shared__ T tmp[3 * 16 * 16];  // sums of the off-diagonal 16-blocks of the inverse
  __shared__ double dg[CB];
  if (*info != 0) return;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kb * kb; idx += blockDim.x) {
    int i = idx % kb, j = idx / kb;
    a[i + j * LD] = (i <= j) ? S[(k0 + i) + (int64_t)(k0 + j) * n] : mkT<T>(0.0, 0.0);
  }
  __syncthreads();
  const int jc = tid % CB, g = tid / CB;  // column jc, rows i = k + 1 + g (mod 4); 256 threads
  int fail = 0;
  for (int k = 0; k < kb; ++k) {
    const double akk = re_(a[k + k * LD]);   // the same value in every thread
    if (!(akk > 1e-15) || !isfinite(akk)) {  // unit-diagonal S: relative floor
      fail = k0 + k + 1;
      break;
    }
    if (jc > k && jc < kb) {
      const T akj = rscale(1.0 / akk, a[k + jc * LD]);
      int i = k + 1 + g;
      // four rows at a time with every load issued before the stores (row k is not
      // written in step k), then the remainder
      for (; i + 12 <= jc; i += 16) {
        const T r0 = a[k + i * LD], r1 = a[k + (i + 4) * LD], r2 = a[k + (i + 8) * LD], r3 = a[k + (i + 12) * LD];
        const T c0 = a[i + jc * LD], c1 = a[i + 4 + jc * LD], c2 = a[i + 8 + jc * LD], c3 = a[i + 12 + jc * LD];
        a[i + jc * LD] = sub_(c0, mul_(conj_(r0), akj));
        a[i + 4 + jc * LD] = sub_(c1, mul_(conj_(r1), akj));
        a[i + 8 + jc * LD] = sub_(c2, mul_(conj_(r2), akj));
        a[i + 12 + jc * LD] = sub_(c3, mul_(conj_(r3), akj));
      }
      for (; i <= jc; i += 4) a[i + jc * LD] = sub_(a[i + jc * LD], mul_(conj_(a[k + i * LD]), akj));
    }
    __syncthreads();
  }
  if (fail) {
    if (tid == 0) *info = fail;
    return;
  }
  for (int i = tid; i < kb; i += blockDim.x) dg[i] = sqrt(re_(a[i + i * LD]));
  __syncthreads();
  for (int idx = tid; idx < kb * kb; idx += blockDim.x) {
    int i = idx % kb, j = idx / kb;
    if (i < j) a[i + j * LD] = rscale(1.0 / dg[i], a[i + j * LD]);
    else if (i == j) a[i + j * LD] = mkT<T>(dg[i], 0.0);
  }
  __syncthreads();
  // R11^{-1} by 16 x 16 blocks: the diagonal blocks by back substitution (one thread per
  // column, at most 16 rows), then the blocks at distance d = 1, 2, 3 from the diagonal,
  // X_IJ = -X_II (sum_{K=I+1..J} R_IK X_KJ), each level in two barrier-separated halves
  for (int idx = tid; idx < CB * CB; idx += blockDim.x) r[(idx % CB) + (idx / CB) * LD] = mkT<T>(0.0, 0.0);
  __syncthreads();
  constexpr int B16 = 16;
  const int nbl = (kb + B16 - 1) / B16;
  if (tid < kb) {
    const int j = tid, b0 = (j / B16) * B16;
    r[j + j * LD] = mkT<T>(1.0 / dg[j], 0.0);
    for (int i = j - 1; i >= b0; --i) {
      T sacc = mkT<T>(0.0, 0.0);
      for (int k = i + 1; k <= j; ++k) sacc = add_(sacc, mul_(a[i + k * LD], r[k + j * LD]));
      r[i + j * LD] = rscale(-1.0 / dg[i], sacc);
    }
  }
  __syncthreads();
  for (int d = 1; d < nbl; ++d) {
    const int nblk = nbl - d;
    for (int idx = tid; idx < nblk * B16 * B16; idx += blockDim.x) {
      const int bI = idx / (B16 * B16), e = idx % (B16 * B16), rr = e % B16, cc = e / B16;
      const int i = bI * B16 + rr, j = (bI + d) * B16 + cc;
      T sacc = mkT<T>(0.0, 0.0);
      if (i < kb && j < kb)
        for (int k = (bI + 1) * B16; k <= j; ++k) sacc = add_(sacc, mul_(a[i + k * LD], r[k + j * LD]));
      tmp[idx] = sacc;
    }
    __syncthreads();
    for (int idx = tid; idx < nblk * B16 * B16; idx += blockDim.x) {
      const int bI = idx / (B16 * B16), e = idx % (B16 * B16), rr = e % B16, cc = e / B16;
      const int i = bI * B16 + rr, j = (bI + d) * B16 + cc;
      if (i < kb && j < kb) {
        T x = mkT<T>(0.0, 0.0);
        const int kend = min((bI + 1) * B16, kb);
        for (int k = i; k < kend; ++k) x = add_(x, mul_(r[i + k * LD], tmp[bI * B16 * B16 + (k - bI * B16) + cc * B16]));
        r[i + j * LD] = sub_(mkT<T>(0.0, 0.0), x);
      }
    }
    __syncthreads();
  }
  for (int idx = tid; idx < kb * kb; idx += blockDim.x) {
    int i = idx % kb, j = idx / kb;
    if (i <= j) S[(k0 + i) + (int64_t)(k0 + j) * n] = a[i + j * LD];
    Rinv[idx] = r[i + j * LD];
  }
}

// row panel: S[k0:k0+kb, c] <- R11^{-H} S[k0:k0+kb, c] for the columns c of this work-group
template <typename T>
__global__ __launch_bounds__(256) void chol_panel_kernel(int n, T* __restrict__ S, int k0, int kb,
                                                         const T* __restrict__ Rinv, const int* info) {
  __shared__ T riT[CB * CB];   // riT[i + l kb] = Rinv[l + i kb]: threads of consecutive i read consecutive words
  __shared__ T col[CB * CB];
  if (*info != 0) return;
  const int c0 = k0 + kb + blockIdx.x * CB;
  const int nc = min(CB, n - c0);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kb * kb; idx += blockDim.x) riT[(idx / kb) + (idx % kb) * kb] = Rinv[idx];
  for (int idx = tid; idx < kb * nc; idx += blockDim.x) {
    int l = idx % kb, c = idx / kb;
    col[idx] = S[(k0 + l) + (int64_t)(c0 + c) * n];
  }
  __syncthreads();
  for (int idx = tid; idx < kb * nc; idx += blockDim.x) {
    int i = idx % kb, c = idx / kb;
    T acc = mkT<T>(0.0, 0.0);
    for (int l = 0; l <= i; ++l) acc = add_(acc, mul_(conj_(riT[i + l * kb]), col[l + c * kb]));
    S[(k0 + i) + (int64_t)(c0 + c) * n] = acc;
  }
}

// trailing update: upper tiles of S22 -= R12^H R12 (R12 = S[k0:k0+kb, k0+kb:n])
template <typename T>
__global__ __launch_bounds__(256) void chol_syrk_kernel(int n, T* __restrict__ S, int k0, int kb, int tiles,
                                                        const int* info) {
  __shared__ T paT[CB * CB];   // paT[i + l CB]: threads of consecutive i read consecutive words
  __shared__ T pb[CB * CB];
  if (*info != 0) return;
  // upper-triangular tile enumeration
  const int t = blockIdx.x;
  int tj = 0;
  while ((tj + 1) * (tj + 2) / 2 <= t) ++tj;
  const int ti = t - tj * (tj + 1) / 2;
  const int base = k0 + kb;
  const int i0 = base + ti * CB, j0 = base + tj * CB;
  const int ni = min(CB, n - i0), nj = min(CB, n - j0);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kb * CB; idx += blockDim.x) {
    int l = idx % kb, c = idx / kb;
    paT[c + l * CB] = (c < ni) ? S[(k0 + l) + (int64_t)(i0 + c) * n] : mkT<T>(0.0, 0.0);
    pb[idx] = (c < nj) ? S[(k0 + l) + (int64_t)(j0 + c) * n] : mkT<T>(0.0, 0.0);
  }
  __syncthreads();
  for (int idx = tid; idx < CB * CB; idx += blockDim.x) {
    int i = idx % CB, j = idx / CB;
    if (i >= ni || j >= nj || i0 + i > j0 + j) continue;
    T acc = mkT<T>(0.0, 0.0);
    for (int l = 0; l < kb; ++l) acc = add_(acc, mul_(conj_(paT[i + l * CB]), pb[l + j * kb]));
    T* sp = &S[(i0 + i) + (int64_t)(j0 + j) * n];
    *sp = sub_(*sp, acc);
  }
}

// T = D^{-1} R^{-1} (R upper triangular in S), one 64-lane work-group per column j:
// x = R^{-1} e_j by 64-row blocks from the bottom, with the diagonal-block inverses of
// the factorisation (Rinv_blk, block b at b CB^2, column-major kb x kb): the block of
// row j is a column of its diagonal-block inverse, and each block I above it is
// x_I = -R_II^{-1} (R_I,(I+1..) x_(I+1..)), a matrix-vector product read from L2 (lane r
// takes row r, so the lanes read a column segment together) followed by the small
// triangular product.  x lives in LDS.
template <typename T>
__global__ __launch_bounds__(64) void trinv_col_kernel(int n, const T* __restrict__ R, const T* __restrict__ Rinv_blk,
                                                       const double* __restrict__ dinv, T* __restrict__ Tout,
                                                       const int* info) {
  extern __shared__ char smem[];
  T* x = (T*)smem;   // [n]
  T* y = x + n;      // [CB]
  if (*info != 0) return;
  const int j = blockIdx.x, lane = threadIdx.x;
  const int J = j / CB, jj0 = J * CB, nJ = min(CB, n - jj0);
  {
    const T* Rj = Rinv_blk + (int64_t)J * CB * CB;
    const int c = j - jj0;
    if (lane < nJ) x[jj0 + lane] = (lane <= c) ? Rj[lane + c * nJ] : mkT<T>(0.0, 0.0);
  }
  __syncthreads();
  for (int I = J - 1; I >= 0; --I) {
    const int i0 = I * CB;   // full blocks above the last one
    T s0 = mkT<T>(0.0, 0.0), s1 = s0;
    int k = i0 + CB;
    for (; k + 1 <= j; k += 2) {
      s0 = add_(s0, mul_(R[(i0 + lane) + (int64_t)k * n], x[k]));
      s1 = add_(s1, mul_(R[(i0 + lane) + (int64_t)(k + 1) * n], x[k + 1]));
    }
    if (k <= j) s0 = add_(s0, mul_(R[(i0 + lane) + (int64_t)k * n], x[k]));
    y[lane] = add_(s0, s1);
    __syncthreads();
    const T* Ri = Rinv_blk + (int64_t)I * CB * CB;
    T t = mkT<T>(0.0, 0.0);
    for (int c = lane; c < CB; ++c) t = add_(t, mul_(Ri[lane + c * CB], y[c]));
    x[i0 + lane] = sub_(mkT<T>(0.0, 0.0), t);
    __syncthreads();
  }
  for (int i = lane; i < n; i += 64) Tout[i + (int64_t)j * n] = (i <= j) ? rscale(dinv[i], x[i]) : mkT<T>(0.0, 0.0);
}

size_t chol_orth_work_bytes(int32_t n, bool cplx) {
  const size_t e = cplx ? 16 : 8;
  const size_t blocks = ((size_t)n + CB - 1) / CB;  // the diagonal-block inverses, kept for the full inverse
  return (size_t)n * n * e + 256 + (size_t)n * 8 + 256 + blocks * CB * CB * e + 256;
}

template <typename T>
static int chol_orth_t(hipStream_t s, int n, const T* M, T* Tout, int* info, void* work, double shift,
                       double min_rel_diag) {
  char* p = (char*)work;
  T* S = (T*)p;
  p += (((size_t)n * n * sizeof(T) + 255) / 256) * 256;
  double* dinv = (double*)p;
  p += (((size_t)n * 8 + 255) / 256) * 256;
  T* Rinv = (T*)p;
  chol_scale_kernel<T><<<n, 256, 0, s>>>(n, M, S, dinv, shift, min_rel_diag, info);
  SPARC_TRY(check_launch("chol_scale_kernel"));
  for (int k0 = 0; k0 < n; k0 += CB) {
    const int kb = std::min(CB, n - k0);
    T* Rb = Rinv + (size_t)(k0 / CB) * CB * CB;
    chol_diag_kernel<T><<<1, 256, 0, s>>>(n, S, k0, kb, Rb, info);
    SPARC_TRY(check_launch("chol_diag_kernel"));
    const int m = n - k0 - kb;
    if (m <= 0) break;
    const int tiles = (m + CB - 1) / CB;
    chol_panel_kernel<T><<<tiles, 256, 0, s>>>(n, S, k0, kb, Rb, info);
    SPARC_TRY(check_launch("chol_panel_kernel"));
    chol_syrk_kernel<T><<<tiles * (tiles + 1) / 2, 256, 0, s>>>(n, S, k0, kb, tiles, info);
    SPARC_TRY(check_launch("chol_syrk_kernel"));
  }
  trinv_col_kernel<T><<<n, 64, (n + CB) * sizeof(T), s>>>(n, S, Rinv, dinv, Tout, info);
  return check_launch("trinv_col_kernel");
}

// Condition estimate of the column-scaled Gram matrix M_s = D^{-1} M D^{-1} (D = sqrt of
// diag M) after chol_orth: a Gershgorin bound on lambda_max(M_s) times a power-iteration
// estimate of lambda_max(M_s^{-1}) = ||R^{-1}||_2^2 (R^{-1} = D T with T = D^{-1} R^{-1}
// from chol_orth), from a fixed start vector.  One work-group; *out = the estimate, or
// 1e300 after a failed factorisation.
// With STAGE (small n) the triangle of T, 1 / D^{-1} and the scaled |M| are first put in
// LDS with coalesced loads, so the column sums and the power iterations read no global
// memory; the arithmetic is the same in both forms.
template <typename T, bool STAGE>
__global__ __launch_bounds__(1024) void cond_est_kernel(int n, const T* __restrict__ M, const T* __restrict__ Tg,
                                                        const double* __restrict__ dinv_g, int iters,
                                                        const int* __restrict__ info, double* __restrict__ out) {
  extern __shared__ char smem[];
  T* v = (T*)smem;  // [n]
  T* y = v + n;     // [n]
  __shared__ double red[16];
  const int tid = threadIdx.x, nt = blockDim.x;
  if (*info != 0) {
    if (tid == 0) *out = 1e300;
    return;
  }
  const T* Tm = Tg;
  double* rinv = nullptr;   // 1 / dinv (STAGE)
  double* am = nullptr;     // |M_ij| dinv_i (STAGE)
  if constexpr (STAGE) {
    T* ts = y + n;          // [n][n], upper triangle filled
    rinv = (double*)(ts + (size_t)n * n);
    am = rinv + n;
    for (int q = tid; q < n * n; q += nt) {
      const int i = q % n, j = q / n;
      if (i <= j) ts[q] = Tg[q];
      const T m = M[q];
      am[q] = sqrt(re_(mul_(conj_(m), m))) * dinv_g[i];
    }
    for (int i = tid; i < n; i += nt) rinv[i] = 1.0 / dinv_g[i];
    __syncthreads();
    Tm = ts;
  }
  // Gershgorin: largest column sum of |M_s| (M_s Hermitian)
  double g = 0.0;
  for (int j = tid; j < n; j += nt) {
    double c = 0.0;
#pragma unroll 8
    for (int i = 0; i < n; ++i) {
      if constexpr (STAGE) {
        c += am[i + (int64_t)j * n];
      } else {
        const T m = M[i + (int64_t)j * n];
        c += sqrt(re_(mul_(conj_(m), m))) * dinv_g[i];
      }
    }
    g = fmax(g, c * dinv_g[j]);
  }
  for (int o = 32; o > 0; o >>= 1) g = fmax(g, __shfl_xor(g, o, 64));
  if ((tid & 63) == 0) red[tid >> 6] = g;
  __syncthreads();
  g = 0.0;
  for (int w = 0; w < nt / 64; ++w) g = fmax(g, red[w]);
  __syncthreads();
  for (int i = tid; i < n; i += nt) v[i] = mkT<T>(1.0 + 0.5 * (double)((i * 7919) % 13) / 13.0, 0.0);
  __syncthreads();
  auto ri = [&](int i) -> double {
    if constexpr (STAGE) return rinv[i];
    else return 1.0 / dinv_g[i];
  };
  double mu = 0.0;
  for (int it = 0; it < iters; ++it) {
    // y = B^H v, B = R^{-1} (upper triangular): y_j = sum_{i <= j} conj(T_ij / dinv_i) v_i
    for (int j = tid; j < n; j += nt) {
      T acc = mkT<T>(0.0, 0.0);
#pragma unroll 8
      for (int i = 0; i <= j; ++i) acc = add_(acc, mul_(conj_(rscale(ri(i), Tm[i + (int64_t)j * n])), v[i]));
      y[j] = acc;
    }
    __syncthreads();
    // v = B y: v_i = sum_{j >= i} (T_ij / dinv_i) y_j
    double nrm = 0.0;
    for (int i = tid; i < n; i += nt) {
      T acc = mkT<T>(0.0, 0.0);
#pragma unroll 8
      for (int j = i; j < n; ++j) acc = add_(acc, mul_(Tm[i + (int64_t)j * n], y[j]));
      acc = rscale(ri(i), acc);
      v[i] = acc;
      nrm += re_(mul_(conj_(acc), acc));
    }
    nrm = block_sum(nrm, red);
    // v was normalised at the previous step (the first start vector is not)
    const double sq = sqrt(nrm);
    if (it > 0) mu = sq;
    for (int i = tid; i < n; i += nt) v[i] = rscale(1.0 / fmax(sq, 1e-300), v[i]);
    __syncthreads();
  }
  if (tid == 0) *out = g * mu;
}

template <typename T>
static int chol_cond_est_t(hipStream_t s, int n, const T* M, const T* Tm, const int* info, void* work, double* out) {
  char* p = (char*)work;
  p += (((size_t)n * n * sizeof(T) + 255) / 256) * 256;
  const double* dinv = (const double*)p;
  // one thread per column up to 1024 (a small matrix keeps the barriers of a small group)
  const int threads = std::min(1024, ((n + 63) / 64) * 64);
  const size_t staged = ((size_t)n * n + 2 * n) * sizeof(T) + ((size_t)n * n + n) * 8;
  if (staged <= 150 * 1024) {
    SPARC_HIP(hipFuncSetAttribute((const void*)cond_est_kernel<T, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)staged));
    cond_est_kernel<T, true><<<1, threads, staged, s>>>(n, M, Tm, dinv, 8, info, out);
  } else {
    cond_est_kernel<T, false><<<1, threads, 2 * (size_t)n * sizeof(T), s>>>(n, M, Tm, dinv, 8, info, out);
  }
  return check_launch("cond_est_kernel");
}

int chol_cond_est(hipStream_t s, bool cplx, int32_t n, const void* M, const void* T, const int32_t* info_dev,
                  void* work, double* out_dev) {
  if (cplx) return chol_cond_est_t<cd>(s, n, (const cd*)M, (const cd*)T, info_dev, work, out_dev);
  return chol_cond_est_t<double>(s, n, (const double*)M, (const double*)T, info_dev, work, out_dev);
}

int chol_orth(hipStream_t s, bool cplx, int32_t n, const void* M, void* T, int32_t* info_dev, void* work,
              double shift, double min_rel_diag) {
  if (cplx) return chol_orth_t<cd>(s, n, (const cd*)M, (cd*)T, info_dev, work, shift, min_rel_diag);
  return chol_orth_t<double>(s, n, (const double*)M, (double*)T, info_dev, work, shift, min_rel_diag);
}

// ------------------------------------------------------------ Householder tridiagonalisation
// Lower Hermitian reduction A = Q T Q^H, Q = H_0 H_1 ... H_{n-2}, H_i = I - tau_i v_i v_i^H,
// v_i = (0..0, 1, A[i+2:, i]) after the call.  d, e: real tridiagonal.
template <typename T>
__global__ __launch_bounds__(1024) void hetrd_kernel(int n, T* __restrict__ A, double* __restrict__ d,
                                                     double* __restrict__ e, T* __restrict__ tau) {
  extern __shared__ char smem[];
  T* v = (T*)smem;        // [n]
  T* w = v + n;           // [n]
  __shared__ double red[16];
  __shared__ T s_tau, s_scale;
  __shared__ double s_beta;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int i = 0; i < n - 1; ++i) {
    const int m = n - i - 1;  // rows i+1 .. n-1
    double xn = 0;
    for (int r = i + 2 + tid; r < n; r += nt) {
      T x = A[r + (int64_t)i * n];
      xn += re_(mul_(conj_(x), x));
    }
    xn = block_sum(xn, red);
    if (tid == 0) {
      T alpha = A[i + 1 + (int64_t)i * n];
      double ar = re_(alpha);
      double ai = 0;
      if constexpr (sizeof(T) == 16) ai = ((cd&)alpha).im;
      if (xn == 0.0 && ai == 0.0) {
        s_tau = mkT<T>(0.0, 0.0);
        s_beta = ar;
        s_scale = mkT<T>(0.0, 0.0);
      } else {
        double beta = -copysign(sqrt(ar * ar + ai * ai + xn), ar);
        s_beta = beta;
        s_tau = mkT<T>((beta - ar) / beta, -ai / beta);
        // 1 / (alpha - beta)
        double dr = ar - beta, di = ai, den = dr * dr + di * di;
        s_scale = mkT<T>(dr / den, -di / den);
      }
    }
    __syncthreads();
    const T tau_i = s_tau;
    const double beta = s_beta;
    if (tid == 0) tau[i] = tau_i;
    const bool trivial = (re_(tau_i) == 0.0) && (re_(mul_(conj_(tau_i), tau_i)) == 0.0);
    // v = (1, x * scale)
    for (int r = i + 1 + tid; r < n; r += nt) {
      T val;
      if (r == i + 1) val = mkT<T>(1.0, 0.0);
      else {
        val = mul_(A[r + (int64_t)i * n], s_scale);
        A[r + (int64_t)i * n] = val;
      }
      v[r] = val;
    }
    __syncthreads();
    if (!trivial) {
      // p = tau * A_sub v  (rows and columns i+1..n-1)
      for (int r = i + 1 + tid; r < n; r += nt) {
        T acc = mkT<T>(0.0, 0.0);
        for (int c = i + 1; c < n; ++c) acc = add_(acc, mul_(A[r + (int64_t)c * n], v[c]));
        w[r] = mul_(tau_i, acc);
      }
      __syncthreads();
      // alpha2 = -1/2 tau (p^H v)
      double pr = 0, pi = 0;
      for (int r = i + 1 + tid; r < n; r += nt) {
        T t = mul_(conj_(w[r]), v[r]);
        pr += re_(t);
        if constexpr (sizeof(T) == 16) pi += ((cd&)t).im;
      }
      pr = block_sum(pr, red);
      if constexpr (sizeof(T) == 16) pi = block_sum(pi, red);
      T a2 = mul_(mkT<T>(-0.5, 0.0), mul_(tau_i, mkT<T>(pr, pi)));
      for (int r = i + 1 + tid; r < n; r += nt) w[r] = add_(w[r], mul_(a2, v[r]));
      __syncthreads();
      // A_sub -= v w^H + w v^H
      for (int64_t idx = tid; idx < (int64_t)m * m; idx += nt) {
        int r = i + 1 + (int)(idx % m), c = i + 1 + (int)(idx / m);
        T upd = add_(mul_(v[r], conj_(w[c])), mul_(w[r], conj_(v[c])));
        A[r + (int64_t)c * n] = sub_(A[r + (int64_t)c * n], upd);
      }
    }
    if (tid == 0) {
      e[i] = beta;
      d[i] = re_(A[i + (int64_t)i * n]);
    }
    __syncthreads();
  }
  if (tid == 0) d[n - 1] = re_(A[(n - 1) + (int64_t)(n - 1) * n]);
}

// Same reduction with a two-dimensional thread map for memory-level parallelism:
// lanes run over 64 consecutive rows (coalesced column segments), the 16 waves over
// interleaved columns; the matrix-vector product is reduced across waves in LDS.
// LDS: 16 partial vectors + v + w (n <= 1066 real, n <= 533 complex).
template <typename T>
__global__ __launch_bounds__(1024) void hetrd2_kernel(int n, T* __restrict__ A, double* __restrict__ d,
                                                      double* __restrict__ e, T* __restrict__ tau) {
  extern __shared__ char smem[];
  T* v = (T*)smem;           // [n]
  T* w = v + n;              // [n]
  T* part = w + n;           // [16][n]
  __shared__ double red[16];
  __shared__ T s_tau, s_scale;
  __shared__ double s_beta;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;
  for (int i = 0; i < n - 1; ++i) {
    const int r0 = i + 1;       // first row/column of the trailing block
    const int m = n - r0;
    double xn = 0;
    for (int r = i + 2 + tid; r < n; r += nt) {
      T x = A[r + (int64_t)i * n];
      xn += re_(mul_(conj_(x), x));
    }
    xn = block_sum(xn, red);
    if (tid == 0) {
      T alpha = A[i + 1 + (int64_t)i * n];
      double ar = re_(alpha);
      double ai = 0;
      if constexpr (sizeof(T) == 16) ai = ((cd&)alpha).im;
      if (xn == 0.0 && ai == 0.0) {
        s_tau = mkT<T>(0.0, 0.0);
        s_beta = ar;
        s_scale = mkT<T>(0.0, 0.0);
      } else {
        double beta = -copysign(sqrt(ar * ar + ai * ai + xn), ar);
        s_beta = beta;
        s_tau = mkT<T>((beta - ar) / beta, -ai / beta);
        double dr = ar - beta, di = ai, den = dr * dr + di * di;
        s_scale = mkT<T>(dr / den, -di / den);
      }
    }
    __syncthreads();
    const T tau_i = s_tau;
    const double beta = s_beta;
    if (tid == 0) tau[i] = tau_i;
    const bool trivial = re_(mul_(conj_(tau_i), tau_i)) == 0.0;
    for (int r = r0 + tid; r < n; r += nt) {
      T val;
      if (r == r0) val = mkT<T>(1.0, 0.0);
      else {
        val = mul_(A[r + (int64_t)i * n], s_scale);
        A[r + (int64_t)i * n] = val;
      }
      v[r] = val;
    }
    __syncthreads();
    if (!trivial) {
      // partial products over this wave's columns
      for (int rb = r0; rb < n; rb += 64) {
        const int r = rb + lane;
        T acc = mkT<T>(0.0, 0.0);
        if (r < n) {
          int c = r0 + wave;
#pragma unroll 4
          for (; c < n; c += nwave) acc = add_(acc, mul_(A[r + (int64_t)c * n], v[c]));
        }
        if (r < n) part[wave * n + r] = acc;
      }
      __syncthreads();
      for (int r = r0 + tid; r < n; r += nt) {
        T acc = mkT<T>(0.0, 0.0);
        for (int q = 0; q < nwave; ++q) acc = add_(acc, part[q * n + r]);
        w[r] = mul_(tau_i, acc);
      }
      __syncthreads();
      double pr = 0, pi = 0;
      for (int r = r0 + tid; r < n; r += nt) {
        T t = mul_(conj_(w[r]), v[r]);
        pr += re_(t);
        if constexpr (sizeof(T) == 16) pi += ((cd&)t).im;
      }
      pr = block_sum(pr, red);
      if constexpr (sizeof(T) == 16) pi = block_sum(pi, red);
      T a2 = mul_(mkT<T>(-0.5, 0.0), mul_(tau_i, mkT<T>(pr, pi)));
      for (int r = r0 + tid; r < n; r += nt) w[r] = add_(w[r], mul_(a2, v[r]));
      __syncthreads();
      // A_sub -= v w^H + w v^H
      for (int rb = r0; rb < n; rb += 64) {
        const int r = rb + lane;
        if (r < n) {
          const T vr = v[r], wr = w[r];
          int c = r0 + wave;
#pragma unroll 4
          for (; c < n; c += nwave) {
            T upd = add_(mul_(vr, conj_(w[c])), mul_(wr, conj_(v[c])));
            A[r + (int64_t)c * n] = sub_(A[r + (int64_t)c * n], upd);
          }
        }
      }
    }
    if (tid == 0) {
      e[i] = beta;
      d[i] = re_(A[i + (int64_t)i * n]);
    }
    __syncthreads();
  }
  if (tid == 0) d[n - 1] = re_(A[(n - 1) + (int64_t)(n - 1) * n]);
}

// The same reduction for n <= 64 with the whole matrix in LDS (column-major, leading
// dimension n + 1), eight waves: lane r of every wave owns row r, wave q the columns
// c = q mod 8 of the matrix-vector product and of the rank-2 update.  Sums over rows are
// wave butterflies, whose result is the same on every lane of every wave, so each wave
// forms the same reflector without exchanging it (register-only DPP sums).  The matrix
// is read once and written back once.
template <typename T>
__global__ __launch_bounds__(512) void hetrd_small_kernel(int n, T* __restrict__ A, double* __restrict__ d,
                                                          double* __restrict__ e, T* __restrict__ tau) {
  extern __shared__ char smem[];
  const int ld = n + 1;
  T* a = (T*)smem;       // [n][ld]
  T* v = a + n * ld;     // [64]
  T* w = v + 64;         // [64]
  T* part = w + 64;      // [8][64]
  const int r = threadIdx.x & 63, q = threadIdx.x >> 6;
  for (int c = q; c < n; c += 8)
    if (r < n) a[r + c * ld] = A[r + (int64_t)c * n];
  __syncthreads();
  for (int i = 0; i < n - 1; ++i) {
    const int r0 = i + 1;
    double xn = 0.0;
    if (r >= i + 2 && r < n) {
      const T x = a[r + i * ld];
      xn = re_(mul_(conj_(x), x));
    }
    xn = wave_sum_dpp(xn);
    const T alpha = a[r0 + i * ld];
    const double ar = re_(alpha);
    double ai = 0;
    if constexpr (sizeof(T) == 16) ai = ((const cd&)alpha).im;
    T tau_i, scl;
    double beta;
    if (xn == 0.0 && ai == 0.0) {
      tau_i = mkT<T>(0.0, 0.0);
      beta = ar;
      scl = mkT<T>(0.0, 0.0);
    } else {
      beta = -copysign(sqrt(ar * ar + ai * ai + xn), ar);
      tau_i = mkT<T>((beta - ar) / beta, -ai / beta);
      const double dr = ar - beta, di = ai, den = dr * dr + di * di;
      scl = mkT<T>(dr / den, -di / den);
    }
    const bool trivial = re_(mul_(conj_(tau_i), tau_i)) == 0.0;
    T vr = mkT<T>(0.0, 0.0);
    if (r == r0) vr = mkT<T>(1.0, 0.0);
    else if (r > r0 && r < n) vr = mul_(a[r + i * ld], scl);
    __syncthreads();   // every wave has read column i
    if (q == 0) {
      if (r > r0 && r < n) a[r + i * ld] = vr;
      v[r] = vr;
    }
    __syncthreads();
    if (!trivial) {
      // p = tau A_sub v (partial products over this wave's columns), alpha2 = -1/2 tau
      // (p^H v), w = p + alpha2 v
      T acc = mkT<T>(0.0, 0.0);
      if (r >= r0 && r < n) {
        int c = r0 + ((q - r0) & 7);
#pragma unroll 2
        for (; c < n; c += 8) acc = add_(acc, mul_(a[r + c * ld], v[c]));
      }
      part[q * 64 + r] = acc;
      __syncthreads();
      const T sum = add_(add_(add_(part[r], part[64 + r]), add_(part[128 + r], part[192 + r])),
                         add_(add_(part[256 + r], part[320 + r]), add_(part[384 + r], part[448 + r])));
      const T pr = (r >= r0 && r < n) ? mul_(tau_i, sum) : mkT<T>(0.0, 0.0);
      const T t = mul_(conj_(pr), vr);
      double sr = wave_sum_dpp(re_(t)), si = 0.0;
      if constexpr (sizeof(T) == 16) si = wave_sum_dpp(((const cd&)t).im);
      const T a2 = mul_(mkT<T>(-0.5, 0.0), mul_(tau_i, mkT<T>(sr, si)));
      const T wr = add_(pr, mul_(a2, vr));
      if (q == 0) w[r] = wr;
      __syncthreads();
      // A_sub -= v w^H + w v^H over this wave's columns
      if (r >= r0 && r < n) {
        int c = r0 + ((q - r0) & 7);
#pragma unroll 2
        for (; c < n; c += 8)
          a[r + c * ld] = sub_(a[r + c * ld], add_(mul_(vr, conj_(w[c])), mul_(wr, conj_(v[c]))));
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      e[i] = beta;
      d[i] = re_(a[i + i * ld]);
      tau[i] = tau_i;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) d[n - 1] = re_(a[(n - 1) + (n - 1) * ld]);
  for (int c = q; c < n; c += 8)
    if (r < n) A[r + (int64_t)c * n] = a[r + c * ld];
}

// Blocked Householder tridiagonalisation (lower; panel / trailing-update split).
// latrd_kernel reduces columns i0 .. i0+jb-1 with one work-group: column i is first
// brought up to date with the panel's earlier reflectors (A(i:n, i) -= V W(i)^H +
// W V(i)^H), its reflector is formed as in hetrd2_kernel, and the product with the
// trailing block reads that block as it stood before the panel, corrected by
// -V (W^H v) - W (V^H v).  The trailing block is read once per column instead of read
// twice and written once.  trail_kernel then applies A -= V W^H + W V^H to the block
// past the panel on many work-groups.  V, W: [jb][n] (vector k contiguous, zero above
// its first row); storage of the reflectors in A, tau, d and e as hetrd2_kernel.
template <typename T>
__global__ __launch_bounds__(1024) void latrd_kernel(int n, int i0, int jb, T* __restrict__ A, double* __restrict__ d,
                                                     double* __restrict__ e, T* __restrict__ tau, T* __restrict__ V,
                                                     T* __restrict__ W) {
  extern __shared__ char smem[];
  T* v = (T*)smem;           // [n]
  T* y = v + n;              // [n]
  T* part = y + n;           // [16][n]
  __shared__ T pq[2][64];    // pq[0][k] = W_k^H v, pq[1][k] = V_k^H v
  __shared__ double red[16];
  __shared__ T s_tau, s_scale;
  __shared__ double s_beta;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;
  __shared__ T s_alpha;
  // one row per thread (n <= blockDim.x): thread r keeps its element of column i in a
  // register through the update, the reflector and the scaling, and its element of y
  // through the correction and the dot product
  const bool one = n <= nt;
  for (int j = 0; j < jb; ++j) {
    const int i = i0 + j, r0 = i + 1;
    T* Vj = V + (int64_t)j * n;
    T* Wj = W + (int64_t)j * n;
    T areg = mkT<T>(0.0, 0.0);
    double xn = 0;
    if (one) {
      // (1) column i up to date with the panel's earlier reflectors, (2) its norm below
      // the sub-diagonal; alpha from the thread of row i + 1, d[i] from that of row i
      const int r = tid;
      if (r >= i && r < n) {
        areg = A[r + (int64_t)i * n];
        if (j > 0) {
#pragma unroll 8
          for (int k = 0; k < j; ++k) {
            const int64_t o = (int64_t)k * n;
            areg = sub_(areg, add_(mul_(V[o + r], conj_(W[o + i])), mul_(W[o + r], conj_(V[o + i]))));
          }
          if (r <= r0) A[r + (int64_t)i * n] = areg;
        }
        if (r == r0) s_alpha = areg;
        if (r == i) d[i] = re_(areg);
        if (r >= i + 2) xn = re_(mul_(conj_(areg), areg));
      }
      xn = block_sum(xn, red);
    } else {
      // (1) column i up to date with the panel's earlier reflectors
      if (j > 0) {
        for (int r = i + tid; r < n; r += nt) {
          T a = A[r + (int64_t)i * n];
#pragma unroll 8
          for (int k = 0; k < j; ++k) {
            const int64_t o = (int64_t)k * n;
            a = sub_(a, add_(mul_(V[o + r], conj_(W[o + i])), mul_(W[o + r], conj_(V[o + i]))));
          }
          A[r + (int64_t)i * n] = a;
        }
        __syncthreads();
      }
      // (2) reflector of A(i+2:n, i) (as hetrd2_kernel)
      for (int r = i + 2 + tid; r < n; r += nt) {
        T x = A[r + (int64_t)i * n];
        xn += re_(mul_(conj_(x), x));
      }
      xn = block_sum(xn, red);
      if (tid == 0) {
        s_alpha = A[i + 1 + (int64_t)i * n];
        d[i] = re_(A[i + (int64_t)i * n]);
      }
    }
    if (tid == 0) {
      const T alpha = s_alpha;
      double ar = re_(alpha);
      double ai = 0;
      if constexpr (sizeof(T) == 16) ai = ((const cd&)alpha).im;
      if (xn == 0.0 && ai == 0.0) {
        s_tau = mkT<T>(0.0, 0.0);
        s_beta = ar;
        s_scale = mkT<T>(0.0, 0.0);
      } else {
        double beta = -copysign(sqrt(ar * ar + ai * ai + xn), ar);
        s_beta = beta;
        s_tau = mkT<T>((beta - ar) / beta, -ai / beta);
        double dr = ar - beta, di = ai, den = dr * dr + di * di;
        s_scale = mkT<T>(dr / den, -di / den);
      }
    }
    __syncthreads();
    const T tau_i = s_tau;
    const double beta = s_beta;
    const bool trivial = re_(mul_(conj_(tau_i), tau_i)) == 0.0;
    if (one) {
      const int r = tid;
      if (r < n) {
        T val = mkT<T>(0.0, 0.0);
        if (r == r0) {
          val = mkT<T>(1.0, 0.0);
        } else if (r > r0) {
          val = mul_(areg, s_scale);
          A[r + (int64_t)i * n] = val;
        }
        if (r >= r0) v[r] = val;
        Vj[r] = val;
      }
    } else {
      for (int r = tid; r < n; r += nt) {
        T val = mkT<T>(0.0, 0.0);
        if (r == r0) {
          val = mkT<T>(1.0, 0.0);
        } else if (r > r0) {
          val = mul_(A[r + (int64_t)i * n], s_scale);
          A[r + (int64_t)i * n] = val;
        }
        if (r >= r0) v[r] = val;
        Vj[r] = val;
      }
    }
    __syncthreads();
    if (!trivial) {
      // y = A_old(r0:n, r0:n) v: partial products over this wave's columns
      if constexpr (sizeof(T) == 8) {
        if ((n & 1) == 0) {
          // two rows per lane, 16-byte loads (rows paired from an even start)
          for (int rb = r0 & ~1; rb < n; rb += 128) {
            const int r = rb + 2 * lane;
            if (r < n) {
              double a0 = 0.0, a1 = 0.0;
              int c = r0 + wave;
#pragma unroll 8
              for (; c < n; c += nwave) {
                const double2 t = *(const double2*)&A[r + (int64_t)c * n];
                a0 += t.x * v[c];
                a1 += t.y * v[c];
              }
              if (r >= r0) part[wave * n + r] = a0;
              if (r + 1 >= r0) part[wave * n + r + 1] = a1;
            }
          }
        } else {
          for (int rb = r0; rb < n; rb += 64) {
            const int r = rb + lane;
            if (r < n) {
              double acc = 0.0;
              int c = r0 + wave;
#pragma unroll 8
              for (; c < n; c += nwave) acc += A[r + (int64_t)c * n] * v[c];
              part[wave * n + r] = acc;
            }
          }
        }
      } else {
        for (int rb = r0; rb < n; rb += 64) {
          const int r = rb + lane;
          if (r < n) {
            T acc = mkT<T>(0.0, 0.0);
            int c = r0 + wave;
#pragma unroll 8
            for (; c < n; c += nwave) acc = add_(acc, mul_(A[r + (int64_t)c * n], v[c]));
            part[wave * n + r] = acc;
          }
        }
      }
      // W_k^H v and V_k^H v for the panel's earlier reflectors: one wave per product
      for (int task = wave; task < 2 * j; task += nwave) {
        const int k = task >> 1;
        const T* u = ((task & 1) ? V : W) + (int64_t)k * n;
        double pr = 0, pi = 0;
#pragma unroll 4
        for (int r = r0 + lane; r < n; r += 64) {
          T t = mul_(conj_(u[r]), v[r]);
          pr += re_(t);
          if constexpr (sizeof(T) == 16) pi += ((cd&)t).im;
        }
        pr = wave_sum_dpp(pr);
        if constexpr (sizeof(T) == 16) pi = wave_sum_dpp(pi);
        if (lane == 0) pq[task & 1][k] = mkT<T>(pr, pi);
      }
      __syncthreads();
      if (one) {
        // y = tau (A_old v - V (W^H v) - W (V^H v)) for this thread's row, kept in a register
        const int r = tid;
        T yr = mkT<T>(0.0, 0.0), vr = mkT<T>(0.0, 0.0);
        if (r >= r0 && r < n) {
          T acc = mkT<T>(0.0, 0.0);
          for (int q = 0; q < nwave; ++q) acc = add_(acc, part[q * n + r]);
#pragma unroll 8
          for (int k = 0; k < j; ++k) {
            const int64_t o = (int64_t)k * n;
            acc = sub_(acc, add_(mul_(V[o + r], pq[0][k]), mul_(W[o + r], pq[1][k])));
          }
          yr = mul_(tau_i, acc);
          vr = v[r];
        }
        const T t = mul_(conj_(yr), vr);
        double pr = block_sum(re_(t), red), pi = 0.0;
        if constexpr (sizeof(T) == 16) pi = block_sum(((const cd&)t).im, red);
        const T a2 = mul_(mkT<T>(-0.5, 0.0), mul_(tau_i, mkT<T>(pr, pi)));
        if (r < n) Wj[r] = (r >= r0) ? add_(yr, mul_(a2, vr)) : mkT<T>(0.0, 0.0);
      } else {
        for (int r = r0 + tid; r < n; r += nt) {
          T acc = mkT<T>(0.0, 0.0);
          for (int q = 0; q < nwave; ++q) acc = add_(acc, part[q * n + r]);
#pragma unroll 8
          for (int k = 0; k < j; ++k) {
            const int64_t o = (int64_t)k * n;
            acc = sub_(acc, add_(mul_(V[o + r], pq[0][k]), mul_(W[o + r], pq[1][k])));
          }
          y[r] = mul_(tau_i, acc);
        }
        __syncthreads();
        double pr = 0, pi = 0;
        for (int r = r0 + tid; r < n; r += nt) {
          T t = mul_(conj_(y[r]), v[r]);
          pr += re_(t);
          if constexpr (sizeof(T) == 16) pi += ((cd&)t).im;
        }
        pr = block_sum(pr, red);
        if constexpr (sizeof(T) == 16) pi = block_sum(pi, red);
        const T a2 = mul_(mkT<T>(-0.5, 0.0), mul_(tau_i, mkT<T>(pr, pi)));
        for (int r = tid; r < n; r += nt) Wj[r] = (r >= r0) ? add_(y[r], mul_(a2, v[r])) : mkT<T>(0.0, 0.0);
      }
    } else {
      for (int r = tid; r < n; r += nt) Wj[r] = mkT<T>(0.0, 0.0);
    }
    if (tid == 0) {
      e[i] = beta;
      tau[i] = tau_i;
    }
    __syncthreads();
  }
}

// A(c0:n, c0:n) -= V W^H + W V^H over the jb panel reflectors; 16 x 16 tiles
template <typename T>
__global__ __launch_bounds__(256) void trail_kernel(int n, int c0, int jb, T* __restrict__ A, const T* __restrict__ V,
                                                    const T* __restrict__ W) {
  __shared__ T sVr[32][16], sWr[32][16], sVc[32][16], sWc[32][16];
  const int tid = threadIdx.x;
  const int r_base = c0 + blockIdx.x * 16, c_base = c0 + blockIdx.y * 16;
  for (int idx = tid; idx < jb * 16; idx += 256) {
    const int k = idx / 16, t = idx % 16;
    const int r = r_base + t, c = c_base + t;
    const int64_t o = (int64_t)k * n;
    sVr[k][t] = r < n ? V[o + r] : mkT<T>(0.0, 0.0);
    sWr[k][t] = r < n ? W[o + r] : mkT<T>(0.0, 0.0);
    sVc[k][t] = c < n ? V[o + c] : mkT<T>(0.0, 0.0);
    sWc[k][t] = c < n ? W[o + c] : mkT<T>(0.0, 0.0);
  }
  __syncthreads();
  const int tx = tid % 16, ty = tid / 16;
  const int r = r_base + tx, c = c_base + ty;
  if (r < n && c < n) {
    T acc = A[r + (int64_t)c * n];
    for (int k = 0; k < jb; ++k)
      acc = sub_(acc, add_(mul_(sVr[k][tx], conj_(sWc[k][ty])), mul_(sWr[k][tx], conj_(sVc[k][ty]))));
    A[r + (int64_t)c * n] = acc;
  }
}

template <typename T>
__global__ void last_diag_kernel(int n, const T* __restrict__ A, double* __restrict__ d) {
  if (threadIdx.x == 0) d[n - 1] = re_(A[(n - 1) + (int64_t)(n - 1) * n]);
}

// ------------------------------------------------------------ tridiagonal eigenvalues (bisection)
__device__ int sturm_count(int n, const double* d, const double* e2, double x, double pivmin) {
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int cnt = q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// one wave per eigenvalue (4 per work-group): each round evaluates the Sturm count at 64
// interior points of the current interval (one per lane) and keeps the sub-interval
// where the count crosses j, so the interval shrinks 65-fold per round instead of 2-fold
__global__ __launch_bounds__(256) void bisect_kernel(int n, const double* __restrict__ d, const double* __restrict__ e,
                                                     double* __restrict__ w, double* __restrict__ e2g) {
  extern __shared__ double sm[];
  double* ds = sm;
  double* e2 = sm + n;
  __shared__ double red[3][4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < n; i += blockDim.x) {
    ds[i] = d[i];
    e2[i] = (i < n - 1) ? e[i] * e[i] : 0.0;
  }
  __syncthreads();
  // Gershgorin interval and pivot floor (block-wide min / max)
  double lo = 1e300, hi = -1e300, emax = 0;
  for (int i = tid; i < n; i += blockDim.x) {
    double r = (i > 0 ? sqrt(e2[i - 1]) : 0.0) + (i < n - 1 ? sqrt(e2[i]) : 0.0);
    lo = fmin(lo, ds[i] - r);
    hi = fmax(hi, ds[i] + r);
    emax = fmax(emax, e2[i]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
    emax = fmax(emax, __shfl_xor(emax, o, 64));
  }
  if (lane == 0) {
    red[0][wave] = lo;
    red[1][wave] = hi;
    red[2][wave] = emax;
  }
  __syncthreads();
  lo = fmin(fmin(red[0][0], red[0][1]), fmin(red[0][2], red[0][3]));
  hi = fmax(fmax(red[1][0], red[1][1]), fmax(red[1][2], red[1][3]));
  emax = fmax(fmax(red[2][0], red[2][1]), fmax(red[2][2], red[2][3]));
  const double pivmin = 1e-290 * fmax(1.0, emax);
  const double tnorm = fmax(fabs(lo), fabs(hi));
  lo -= 2.2e-16 * tnorm * n + 2 * pivmin;
  hi += 2.2e-16 * tnorm * n + 2 * pivmin;
  const int j = blockIdx.x * 4 + wave;
  if (j >= n) return;
  for (int it = 0; it < 64; ++it) {
    if (hi - lo <= 4.4e-16 * fmax(fabs(lo), fabs(hi)) + 2.2e-16 * tnorm + pivmin) break;
    const double step = (hi - lo) / 65.0;
    const double x = lo + step * (lane + 1);
    const unsigned long long above = __ballot(x < hi && sturm_count(n, ds, e2, x, pivmin) > j);
    const int f = above ? __ffsll((long long)above) - 1 : 64;   // first point above lambda_j
    const double nlo = (f == 0) ? lo : lo + step * f;
    const double nhi = (f == 64) ? hi : lo + step * (f + 1);
    if (!(nlo > lo) && !(nhi < hi)) break;   // no progress in floating point
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) w[j] = 0.5 * (lo + hi);
  if (j == 0 && lane == 0) e2g[0] = tnorm;
}

// ------------------------------------------------------------ inverse iteration
// One work-group (one wave) per cluster of eigenvalues (gap <= 1e-6 ||T||); Y (n x n, real)
// column j = eigenvector j of T.  The pivoted LU of T - lambda I and the substitutions
// are sequential and run on lane 0 with the factors in LDS (an LDS round trip per step
// instead of an L2 one); start vector, Gram-Schmidt against the earlier vectors of the
// cluster and normalisation use the whole wave.
__global__ __launch_bounds__(64) void inviter_kernel(int n, const double* __restrict__ d,
                                                     const double* __restrict__ e, const double* __restrict__ w,
                                                     const double* __restrict__ tnorm_p, double* __restrict__ Y) {
  extern __shared__ double sm[];
  double* dl = sm;
  double* dd = dl + n;
  double* du = dd + n;
  double* du2 = du + n;
  double* b = du2 + n;
  double* rd = b + n;    // 1 / diagonal of U
  unsigned char* ip = (unsigned char*)(rd + n);
  const int j0 = blockIdx.x;
  const int lane = threadIdx.x;
  const double tnorm = fmax(*tnorm_p, 1e-300);
  const double gtol = 1e-6 * tnorm;
  if (j0 > 0 && w[j0] - w[j0 - 1] <= gtol) return;  // not the start of a cluster (uniform)
  int j1 = j0;
  while (j1 + 1 < n && w[j1 + 1] - w[j1] <= gtol) ++j1;
  const double eps = 2.2e-16;
  double prev = -1e300;
  auto wave_dot = [&](const double* x, const double* y) {
    double s = 0;
    for (int i = lane; i < n; i += 64) s += x[i] * y[i];
    return wave_sum(s);
  };
  for (int j = j0; j <= j1; ++j) {
    double lam = w[j];
    if (lam - prev < 10.0 * eps * tnorm) lam = prev + 10.0 * eps * tnorm;
    prev = lam;
    for (int i = lane; i < n; i += 64) {
      dd[i] = d[i] - lam;
      if (i < n - 1) { dl[i] = e[i]; du[i] = e[i]; }
      du2[i] = 0.0;
      // deterministic start vector
      uint32_t h = (uint32_t)(i * 2654435761u) ^ (uint32_t)(j * 40503u + 0x9e3779b9u);
      h ^= h >> 16; h *= 0x7feb352du; h ^= h >> 15; h *= 0x846ca68bu; h ^= h >> 16;
      b[i] = ((h & 0xffffff) / 16777216.0) - 0.5 + 1e-3;
    }
    __syncthreads();
    if (lane == 0) {
      // LU with partial pivoting of T - lam I (general tridiagonal form); the entries
      // that step i updates for step i + 1 (the diagonal and super-diagonal element) are
      // carried in registers, the rest read from LDS ahead of the chain
      double dcur = dd[0], ucur = (n > 1) ? du[0] : 0.0;
#pragma unroll 4
      for (int i = 0; i < n - 1; ++i) {
        const double li = dl[i], dnext = dd[i + 1], unext = (i < n - 2) ? du[i + 1] : 0.0;
        if (fabs(dcur) >= fabs(li)) {
          ip[i] = 0;
          if (dcur == 0.0) dcur = eps * tnorm;
          dd[i] = dcur;
          const double f = li / dcur;
          dl[i] = f;
          du[i] = ucur;
          if (i < n - 2) du2[i] = 0.0;
          dcur = dnext - f * ucur;
          ucur = unext;
        } else {
          ip[i] = 1;
          const double f = dcur / li;
          dd[i] = li;
          dl[i] = f;
          du[i] = dnext;
          dcur = ucur - f * dnext;
          if (i < n - 2) du2[i] = unext;
          ucur = -f * unext;
        }
      }
      if (dcur == 0.0) dcur = eps * tnorm;
      dd[n - 1] = dcur;
    }
    __syncthreads();
    for (int i = lane; i < n; i += 64) rd[i] = 1.0 / dd[i];
    __syncthreads();
    for (int it = 0; it < 4; ++it) {
      if (lane == 0) {
        // forward: row interchanges and multipliers (the running element in a register;
        // both cases formed and one selected, so the loop has no branch)
        double bc = b[0];
#pragma unroll 4
        for (int i = 0; i < n - 1; ++i) {
          const double bn = b[i + 1], l = dl[i];
          const bool sw = ip[i] != 0;
          const double keep = bn - l * bc, swap = bc - l * bn;
          b[i] = sw ? bn : bc;
          bc = sw ? swap : keep;
        }
        b[n - 1] = bc;
        // back substitution with U (reciprocal diagonal rd, super du, super-2 du2), the
        // last two solved elements in registers
        double x1 = b[n - 1] * rd[n - 1], x2 = 0.0;
        b[n - 1] = x1;
        if (n > 1) {
          x2 = x1;
          x1 = (b[n - 2] - du[n - 2] * x2) * rd[n - 2];
          b[n - 2] = x1;
        }
#pragma unroll 4
        for (int i = n - 3; i >= 0; --i) {
          const double xi = (b[i] - du[i] * x1 - du2[i] * x2) * rd[i];
          b[i] = xi;
          x2 = x1;
          x1 = xi;
        }
      }
      __syncthreads();
      // orthogonalise against the earlier vectors of the cluster (twice)
      for (int pass = 0; pass < 2; ++pass)
        for (int q = j0; q < j; ++q) {
          const double* yq = Y + (int64_t)q * n;
          const double dot = wave_dot(yq, b);
          for (int i = lane; i < n; i += 64) b[i] = b[i] - dot * yq[i];
          __syncthreads();
        }
      const double inv = 1.0 / sqrt(wave_dot(b, b));
      for (int i = lane; i < n; i += 64) b[i] = b[i] * inv;
      __syncthreads();
    }
    for (int i = lane; i < n; i += 64) Y[i + (int64_t)j * n] = b[i];
    __syncthreads();   // the next vector of the cluster reads this column
  }
}

// ------------------------------------------------------------ back-transformation Z = Q Y
// The same product with the column held in registers (row r = lane + 64 k in z[k], RPL
// rows per lane) and the next reflector and tau loaded while the current one is applied;
// the wave sums are register-only (DPP).
template <typename T, int RPL>
__global__ __launch_bounds__(256) void ormtr_reg_kernel(int n, const T* __restrict__ A, const T* __restrict__ tau,
                                                        const double* __restrict__ Y, T* __restrict__ Z) {
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;   // whole waves
  T z[RPL], vn[RPL];
#pragma unroll
  for (int k = 0; k < RPL; ++k) {
    const int r = lane + 64 * k;
    z[k] = mkT<T>(r < n ? Y[r + (int64_t)c * n] : 0.0, 0.0);
  }
  auto load_v = [&](int i, T (&vv)[RPL]) {
    const T* __restrict__ v = A + (int64_t)i * n;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      const int r = lane + 64 * k;
      vv[k] = (r == i + 1) ? mkT<T>(1.0, 0.0) : ((r > i + 1 && r < n) ? v[r] : mkT<T>(0.0, 0.0));
    }
  };
  if (n < 2) {
    if (lane < n) Z[lane + (int64_t)c * n] = z[0];
    return;
  }
  load_v(n - 2, vn);
  T tn = tau[n - 2];
  for (int i = n - 2; i >= 0; --i) {
    T vc[RPL];
#pragma unroll
    for (int k = 0; k < RPL; ++k) vc[k] = vn[k];
    const T ti = tn;
    if (i > 0) {
      load_v(i - 1, vn);
      tn = tau[i - 1];
    }
    double sr = 0, si = 0;
#pragma unroll
    for (int k = 0; k < RPL; ++k) {
      const T p = mul_(conj_(vc[k]), z[k]);
      sr += re_(p);
      if constexpr (sizeof(T) == 16) si += ((const cd&)p).im;
    }
    sr = wave_sum_dpp(sr);
    if constexpr (sizeof(T) == 16) si = wave_sum_dpp(si);
    const T sc = mul_(ti, mkT<T>(sr, si));
#pragma unroll
    for (int k = 0; k < RPL; ++k)
      if (lane + 64 * k > i) z[k] = sub_(z[k], mul_(vc[k], sc));
  }
#pragma unroll
  for (int k = 0; k < RPL; ++k) {
    const int r = lane + 64 * k;
    if (r < n) Z[r + (int64_t)c * n] = z[k];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void ormtr_kernel(int n, const T* __restrict__ A, const T* __restrict__ tau,
                                                    const double* __restrict__ Y, T* __restrict__ Z) {
  // one wave per column z of Z: z = H_0 H_1 ... H_{n-2} y, the reflectors applied from
  // the last one; row r is always handled by lane r % 64, so each lane only re-reads
  // what it wrote itself and the wave needs no barrier
  const int lane = threadIdx.x & 63;
  const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (c >= n) return;
  T* __restrict__ z = Z + (int64_t)c * n;
  for (int r = lane; r < n; r += 64) z[r] = mkT<T>(Y[r + (int64_t)c * n], 0.0);
  for (int i = n - 2; i >= 0; --i) {
    const T* __restrict__ v = A + (int64_t)i * n;
    const int rb = (i + 1) & ~63;
    double sr = 0, si = 0;
    for (int r = rb + lane; r < n; r += 64) {
      if (r <= i) continue;
      const T vr = (r == i + 1) ? mkT<T>(1.0, 0.0) : v[r];
      const T p = mul_(conj_(vr), z[r]);
      sr += re_(p);
      if constexpr (sizeof(T) == 16) si += ((const cd&)p).im;
    }
    sr = wave_sum(sr);
    if constexpr (sizeof(T) == 16) si = wave_sum(si);
    const T sc = mul_(tau[i], mkT<T>(sr, si));
    for (int r = rb + lane; r < n; r += 64) {
      if (r <= i) continue;
      const T vr = (r == i + 1) ? mkT<T>(1.0, 0.0) : v[r];
      z[r] = sub_(z[r], mul_(vr, sc));
    }
  }
}

size_t heev_work_bytes(int32_t n, bool cplx) {
  size_t b = (size_t)n * 8 * 3 + 64;                  // d, e, tnorm
  b += (size_t)n * (cplx ? 16 : 8);                   // tau
  b += (size_t)n * n * 8;                             // Y
  b += (size_t)5 * n * n * 8 + (size_t)n * n * 4;     // inverse-iteration scratch and pivots
  return b + 1024;
}

template <typename T>
static int heev_t(hipStream_t s, int n, T* A, double* w, T* Z, void* work) {
  char* p = (char*)work;
  auto take = [&](size_t bytes) { char* q = p; p += ((bytes + 255) / 256) * 256; return q; };
  double* d = (double*)take(n * 8);
  double* e = (double*)take(n * 8);
  double* tn = (double*)take(64);
  T* tau = (T*)take(n * sizeof(T));
  double* Y = (double*)take((size_t)n * n * 8);
  double* scr = (double*)take((size_t)5 * n * n * 8);
  (void)take((size_t)n * n * 4);  // reserved (pivots are kept in LDS)
  const size_t lds2 = (size_t)18 * n * sizeof(T);
  constexpr int NB = 32;   // panel width of the blocked reduction
  if (n >= 64 && lds2 <= 150 * 1024) {
    T* Vb = (T*)scr;       // [NB][n] each; the inverse-iteration scratch is free until then
    T* Wb = Vb + (size_t)NB * n;
    SPARC_HIP(hipFuncSetAttribute((const void*)latrd_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2));
    // about two threads per row (the barriers of a larger group cost more than it adds)
    const int lt = std::min(1024, std::max(256, ((2 * n + 63) / 64) * 64));
    for (int i0 = 0; i0 < n - 1; i0 += NB) {
      const int jb = std::min(NB, n - 1 - i0);
      latrd_kernel<T><<<1, lt, lds2, s>>>(n, i0, jb, A, d, e, tau, Vb, Wb);
      SPARC_TRY(check_launch("latrd_kernel"));
      const int c0 = i0 + jb, m = n - c0;
      if (m > 0) {
        trail_kernel<T><<<dim3((m + 15) / 16, (m + 15) / 16), 256, 0, s>>>(n, c0, jb, A, Vb, Wb);
        SPARC_TRY(check_launch("trail_kernel"));
      }
    }
    last_diag_kernel<T><<<1, 64, 0, s>>>(n, A, d);
  } else if (n == 1) {
    hetrd_kernel<T><<<1, 64, 2 * n * sizeof(T), s>>>(n, A, d, e, tau);
  } else if (n <= 64) {
    const size_t lds_s = ((size_t)n * (n + 1) + 640) * sizeof(T);
    SPARC_HIP(hipFuncSetAttribute((const void*)hetrd_small_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  (int)lds_s));
    hetrd_small_kernel<T><<<1, 512, lds_s, s>>>(n, A, d, e, tau);
  } else if (lds2 <= 150 * 1024) {
    SPARC_HIP(hipFuncSetAttribute((const void*)hetrd2_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2));
    hetrd2_kernel<T><<<1, n < 64 ? 128 : 1024, lds2, s>>>(n, A, d, e, tau);
  } else {
    int nt = n >= 1024 ? 1024 : ((n + 63) / 64) * 64;
    hetrd_kernel<T><<<1, nt, 2 * n * sizeof(T), s>>>(n, A, d, e, tau);
  }
  SPARC_TRY(check_launch("hetrd_kernel"));
  SPARC_HIP(hipFuncSetAttribute((const void*)bisect_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 2 * n * 8));
  bisect_kernel<<<(n + 3) / 4, 256, 2 * n * 8, s>>>(n, d, e, w, tn);
  SPARC_TRY(check_launch("bisect_kernel"));
  const size_t lds_inv = (size_t)n * (6 * 8 + 1);
  SPARC_HIP(hipFuncSetAttribute((const void*)inviter_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_inv));
  inviter_kernel<<<n, 64, lds_inv, s>>>(n, d, e, w, tn, Y);
  SPARC_TRY(check_launch("inviter_kernel"));
  const unsigned gb = (unsigned)((n + 3) / 4);
  const int rpl = (n + 63) / 64;
  if (rpl <= 1) ormtr_reg_kernel<T, 1><<<gb, 256, 0, s>>>(n, A, tau, Y, Z);
  else if (rpl <= 2) ormtr_reg_kernel<T, 2><<<gb, 256, 0, s>>>(n, A, tau, Y, Z);
  else if (rpl <= 4) ormtr_reg_kernel<T, 4><<<gb, 256, 0, s>>>(n, A, tau, Y, Z);
  else if (rpl <= 8) ormtr_reg_kernel<T, 8><<<gb, 256, 0, s>>>(n, A, tau, Y, Z);
  else ormtr_kernel<T><<<gb, 256, 0, s>>>(n, A, tau, Y, Z);
  return check_launch("ormtr_kernel");
}

int heev(hipStream_t s, bool cplx, int32_t n, void* A, double* w, void* Z, void* work) {
  if (n > 2048) return fail(SPARC_ESHAPE, "heev: n=%d above 2048", n);
  if (cplx) return heev_t<cd>(s, n, (cd*)A, w, (cd*)Z, work);
  return heev_t<double>(s, n, (double*)A, w, (double*)Z, work);
}

int small_gemm(hipStream_t s, bool cplx, int32_t n, int opA, const void* A, const void* B, void* C, void* work,
               size_t work_bytes, int n_cu) {
  sparc_dtype dt = cplx ? SPARC_C128 : SPARC_R64;
  if (opA == 1) return gram(s, dt, n, n, n, A, n, B, n, C, n, work, work_bytes, SPARC_GEMM_NATIVE, n_cu);
  return rotate(s, dt, n, n, n, A, n, B, n, C, n, 0);
}

}  // namespace sparc
