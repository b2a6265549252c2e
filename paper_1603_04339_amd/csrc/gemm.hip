// Matrix-core (MFMA) contractions of the Rayleigh-Ritz step.
//
//  gram:   C = A^H B with A, B tall N x n (N = number of grid nodes, up to ~10^6;
//          n = number of states, up to ~10^3).  The N dimension is split into
//          slabs; each work-group owns one 64 x 64 output tile of one slab and
//          writes its partial tile, a second kernel sums the slabs in a fixed
//          order (deterministic).  Work-groups sharing a slab are placed on the
//          same XCD so that the slab is read from HBM once and reused from L2.
//  rotate: Out = A Q with A tall N x n_in and Q small n_in x n_out (FP64), used
//          for the orthonormalisation and the subspace rotation U = U_f Y.
//          Computed as Out^T = Q^T A^T so that each output column is written
//          with contiguous 128-byte segments.
//
// FP64 blocks use v_mfma_f64_16x16x4f64, FP32 blocks v_mfma_f32_16x16x4f32
// (FP32 accumulation inside a slab, FP64 across slabs); complex products are
// four real MFMAs on the (re, im) parts.  Operand lane layout (both types):
// A[i][k] in lane i + 16k, B[k][j] in lane j + 16k.  Result element v of lane
// l is C[l/16 + 4v][l%16] for f64 and C[4(l/16) + v][l%16] for f32.
#include "devmath.hpp"

namespace sparc {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename R> struct mfma_t;
template <> struct mfma_t<double> {
  typedef v4d acc;
  static __device__ __forceinline__ acc step(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return (l >> 4) + 4 * v; }
};
template <> struct mfma_t<float> {
  typedef v4f acc;
  static __device__ __forceinline__ acc step(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int v) { return 4 * (l >> 4) + v; }
};

// split an element into (re, im) reals
template <typename E> __device__ __forceinline__ void split(E v, typename elem<E>::real& r, typename elem<E>::real& i);
template <> __device__ __forceinline__ void split<double>(double v, double& r, double& i) { r = v; i = 0; }
template <> __device__ __forceinline__ void split<float>(float v, float& r, float& i) { r = v; i = 0; }
template <> __device__ __forceinline__ void split<cd>(cd v, double& r, double& i) { r = v.re; i = v.im; }
template <> __device__ __forceinline__ void split<cf>(cf v, float& r, float& i) { r = v.re; i = v.im; }

constexpr int GT = 64;   // tile-edge unit of the Hermitian fill and of the work-space layout

template <typename E> struct gram_tile { static constexpr int T = elem<E>::is_cplx ? 64 : 128; };

// ---------------------------------------------------------------- gram
// One work-group: a T x T output tile of one slab.  4 waves in 2 x 2, each wave
// (T/2) x (T/2) = WB x WB MFMA blocks.  The next k-chunk is loaded into registers
// while the current one is consumed from LDS.
template <typename E, int T>
__global__ __launch_bounds__(256) void gram_kernel(int64_t N, int na, int nb, const E* __restrict__ A, int64_t lda,
                                                   const E* __restrict__ B, int64_t ldb, int n_slab, int64_t slab_len,
                                                   int tiles_a, int n_tiles, int herm,
                                                   double* __restrict__ part, int xcd_remap) {
  typedef typename elem<E>::real R;
  constexpr bool CPX = elem<E>::is_cplx;
  constexpr int NCP = CPX ? 2 : 1;
  constexpr int KC = 16;
  constexpr int WB = T / 32;
  constexpr int PER = T * KC / 256;     // values per thread per operand per chunk
  constexpr int TPC = KC / PER;         // threads per column
  typedef mfma_t<R> M;
  __shared__ R As[NCP][T][KC + 1];
  __shared__ R Bs[NCP][T][KC + 1];

  int bid = blockIdx.x;
  const int total = n_slab * n_tiles;
  if (xcd_remap) bid = (bid % 8) * (total / 8) + bid / 8;
  const int slab = bid / n_tiles;
  const int tile = bid % n_tiles;
  int ti, tj;
  if (herm) {  // upper-triangular tile enumeration: tile = tj (tj + 1) / 2 + ti, ti <= tj
    tj = 0;
    while ((tj + 1) * (tj + 2) / 2 <= tile) ++tj;
    ti = tile - tj * (tj + 1) / 2;
  } else {
    ti = tile % tiles_a;
    tj = tile / tiles_a;
  }
  const int i0 = ti * T, j0 = tj * T;
  const int64_t k_beg = (int64_t)slab * slab_len;
  const int64_t k_end = min(N, k_beg + slab_len);

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wi = (wv & 1) * (T / 2), wj = (wv >> 1) * (T / 2);
  typename M::acc acc_r[WB][WB], acc_i[WB][WB];
#pragma unroll
  for (int a = 0; a < WB; ++a)
#pragma unroll
    for (int b = 0; b < WB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) { acc_r[a][b][v] = 0; if constexpr (CPX) acc_i[a][b][v] = 0; }

  const int lc = tid / TPC, lk = (tid % TPC) * PER;
  const int ia = i0 + lc, jb = j0 + lc;
  E ra[PER], rb[PER];
  auto fetch = [&](int64_t k0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int64_t k = k0 + lk + u;
      ra[u] = zero<E>();
      rb[u] = zero<E>();
      if (k < k_end) {
        if (ia < na) ra[u] = A[k + (int64_t)ia * lda];
        if (jb < nb) rb[u] = B[k + (int64_t)jb * ldb];
      }
    }
  };
  fetch(k_beg);
  for (int64_t k0 = k_beg; k0 < k_end; k0 += KC) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      R ar, ai, br, bi;
      split<E>(ra[u], ar, ai);
      split<E>(rb[u], br, bi);
      As[0][lc][lk + u] = ar;
      Bs[0][lc][lk + u] = br;
      if constexpr (CPX) {
        As[1][lc][lk + u] = ai;
        Bs[1][lc][lk + u] = bi;
      }
    }
    __syncthreads();
    if (k0 + KC < k_end) fetch(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int kq = kk + (lane >> 4), r16 = lane & 15;
      R a_r[WB], a_i[WB], b_r[WB], b_i[WB];
#pragma unroll
      for (int a = 0; a < WB; ++a) {
        a_r[a] = As[0][wi + 16 * a + r16][kq];
        b_r[a] = Bs[0][wj + 16 * a + r16][kq];
        if constexpr (CPX) {
          a_i[a] = As[1][wi + 16 * a + r16][kq];
          b_i[a] = Bs[1][wj + 16 * a + r16][kq];
        }
      }
#pragma unroll
      for (int a = 0; a < WB; ++a)
#pragma unroll
        for (int b = 0; b < WB; ++b) {
          acc_r[a][b] = M::step(a_r[a], b_r[b], acc_r[a][b]);
          if constexpr (CPX) {
            // conj(A)^T B: re += ar br + ai bi ; im += ar bi - ai br
            acc_r[a][b] = M::step(a_i[a], b_i[b], acc_r[a][b]);
            acc_i[a][b] = M::step(a_r[a], b_i[b], acc_i[a][b]);
            acc_i[a][b] = M::step(-a_i[a], b_r[b], acc_i[a][b]);
          }
        }
    }
    __syncthreads();
  }
  // partial tile -> part[slab] (column-major na x nb, FP64; complex interleaved)
  const int64_t mat = (int64_t)na * nb * NCP;
  double* P = part + (int64_t)slab * mat;
#pragma unroll
  for (int a = 0; a < WB; ++a)
#pragma unroll
    for (int b = 0; b < WB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int i = i0 + wi + 16 * a + M::row(lane, v);
        int j = j0 + wj + 16 * b + (lane & 15);
        if (i < na && j < nb) {
          if constexpr (CPX) {
            P[2 * (i + (int64_t)j * na)] = (double)acc_r[a][b][v];
            P[2 * (i + (int64_t)j * na) + 1] = (double)acc_i[a][b][v];
          } else {
            P[i + (int64_t)j * na] = (double)acc_r[a][b][v];
          }
        }
      }
}

// C = sum over slabs; herm: only tiles with ti <= tj were computed, fill the
// lower triangle by conjugate symmetry and make the diagonal real.
__global__ void gram_reduce_kernel(int na, int nb, int n_slab, const double* __restrict__ part, double* __restrict__ C,
                                   int ldc, int cplx, int herm) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)na * nb) return;
  int i = (int)(idx % na), j = (int)(idx / na);
  int si = i, sj = j;
  bool conj_ = false;
  if (herm && i > j) { si = j; sj = i; conj_ = true; }
  const int64_t mat = (int64_t)na * nb * (cplx ? 2 : 1);
  const int64_t off = (si + (int64_t)sj * na) * (cplx ? 2 : 1);
  double re = 0, im = 0;
  for (int s = 0; s < n_slab; ++s) {
    re += part[s * mat + off];
    if (cplx) im += part[s * mat + off + 1];
  }
  if (herm && i == j) im = 0;
  if (cplx) {
    C[2 * (i + (int64_t)j * ldc)] = re;
    C[2 * (i + (int64_t)j * ldc) + 1] = conj_ ? -im : im;
  } else {
    C[i + (int64_t)j * ldc] = re;
  }
}

struct GramPlan {
  int tiles_a, tiles_b, n_tiles, n_slab;
  int64_t slab_len;
};

static GramPlan gram_plan(int64_t N, int na, int nb, bool herm, int n_cu, int T) {
  GramPlan p;
  p.tiles_a = (na + T - 1) / T;
  p.tiles_b = (nb + T - 1) / T;
  p.n_tiles = 0;
  for (int tj = 0; tj < p.tiles_b; ++tj)
    for (int ti = 0; ti < p.tiles_a; ++ti)
      if (!herm || ti <= tj) p.n_tiles++;
  // enough work-groups for ~4 per CU, each slab at least 2048 nodes long
  int64_t want = 4 * (int64_t)n_cu;
  int64_t s = (want + p.n_tiles - 1) / p.n_tiles;
  int64_t smax = std::max<int64_t>(1, N / 2048);
  s = std::max<int64_t>(1, std::min<int64_t>(s, smax));
  s = std::min<int64_t>(s, 256);
  // make the work-group count a multiple of 8 where possible (XCD placement)
  while (s < smax && s < 256 && ((s * p.n_tiles) % 8) != 0) ++s;
  p.slab_len = (N + s - 1) / s;
  p.slab_len = ((p.slab_len + 15) / 16) * 16;
  p.n_slab = (int)((N + p.slab_len - 1) / p.slab_len);
  return p;
}

size_t gram_work_bytes(int64_t N, int32_t n_a, int32_t n_b, sparc_dtype dt) {
  GramPlan p = gram_plan(N, n_a, n_b, false, 256, 64);
  // plans for other CU counts use at most 256 slabs
  int64_t slabs = std::max<int64_t>(p.n_slab, 256);
  return (size_t)slabs * n_a * n_b * 8 * (dtype_complex(dt) ? 2 : 1);
}

template <typename E>
static int gram_t(hipStream_t s, int64_t N, int na, int nb, const E* A, int64_t lda, const E* B, int64_t ldb, void* C,
                  int ldc, void* work, size_t work_bytes, int n_cu) {
  const bool herm = (A == B) && (na == nb) && (lda == ldb);
  constexpr int T = gram_tile<E>::T;
  GramPlan p = gram_plan(N, na, nb, herm, n_cu, T);
  const bool cplx = elem<E>::is_cplx;
  size_t part_bytes = (size_t)p.n_slab * na * nb * 8 * (cplx ? 2 : 1);
  if (part_bytes > work_bytes) return fail(SPARC_ENOMEM, "gram: workspace %zu < %zu bytes", work_bytes, part_bytes);
  double* part = (double*)work;
  int total = p.n_slab * p.n_tiles;
  int remap = (total % 8 == 0) ? 1 : 0;
  gram_kernel<E, T><<<total, 256, 0, s>>>(N, na, nb, A, lda, B, ldb, p.n_slab, p.slab_len, p.tiles_a, p.n_tiles,
                                          herm ? 1 : 0, part, remap);
  SPARC_TRY(check_launch("gram_kernel"));
  int64_t ne = (int64_t)na * nb;
  gram_reduce_kernel<<<(unsigned)((ne + 255) / 256), 256, 0, s>>>(na, nb, p.n_slab, part, (double*)C, ldc,
                                                                  cplx ? 1 : 0, herm ? 1 : 0);
  return check_launch("gram_reduce_kernel");
}

int gram(hipStream_t s, sparc_dtype dt, int64_t N, int32_t na, int32_t nb, const void* A, int64_t lda, const void* B,
         int64_t ldb, void* C, int32_t ldc, void* work, size_t work_bytes, sparc_gemm_mode mode, int n_cu) {
  (void)mode;
  switch (dt) {
    case SPARC_R64: return gram_t<double>(s, N, na, nb, (const double*)A, lda, (const double*)B, ldb, C, ldc, work, work_bytes, n_cu);
    case SPARC_R32: return gram_t<float>(s, N, na, nb, (const float*)A, lda, (const float*)B, ldb, C, ldc, work, work_bytes, n_cu);
    case SPARC_C128: return gram_t<cd>(s, N, na, nb, (const cd*)A, lda, (const cd*)B, ldb, C, ldc, work, work_bytes, n_cu);
    case SPARC_C64: return gram_t<cf>(s, N, na, nb, (const cf*)A, lda, (const cf*)B, ldb, C, ldc, work, work_bytes, n_cu);
  }
  return fail(SPARC_EINVAL, "gram: bad dtype");
}

// ---------------------------------------------------------------- rotate
// One work-group: T rows of A (grid nodes) x T output columns; 4 waves in 2 x 2,
// each (T/2) x (T/2); next k-chunk prefetched into registers.
template <typename E, int T>
__global__ __launch_bounds__(256) void rotate_kernel(int64_t N, int n_in, int n_out, const E* __restrict__ A,
                                                     int64_t lda, const double* __restrict__ Q, int ldq,
                                                     E* __restrict__ Out, int64_t ldo, int tiles_n, int xcd_remap,
                                                     int64_t total, int q_upper) {
  typedef typename elem<E>::real R;
  constexpr bool CPX = elem<E>::is_cplx;
  constexpr int NCP = CPX ? 2 : 1;
  constexpr int KC = 16;
  constexpr int WB = T / 32;
  constexpr int PER = T * KC / 256;
  typedef mfma_t<R> M;
  __shared__ R As[NCP][KC][T + 1];
  __shared__ R Qs[NCP][KC][T + 1];
  int64_t bid = blockIdx.x;
  if (xcd_remap) bid = (bid % 8) * (total / 8) + bid / 8;
  const int tn = (int)(bid % tiles_n);
  const int64_t m0 = (bid / tiles_n) * T;
  const int j0 = tn * T;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wj = (wv & 1) * (T / 2), wm = (wv >> 1) * (T / 2);
  typename M::acc acc_r[WB][WB], acc_i[WB][WB];
#pragma unroll
  for (int a = 0; a < WB; ++a)
#pragma unroll
    for (int b = 0; b < WB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) { acc_r[a][b][v] = 0; if constexpr (CPX) acc_i[a][b][v] = 0; }
  // A loader: column k = tid / (T/PER), PER consecutive rows; Q loader: column j = tid / (KC/PER), PER consecutive k
  constexpr int ATPC = T / PER;
  const int ak = tid / ATPC, am = (tid % ATPC) * PER;
  constexpr int QTPC = KC / PER;
  const int qj = tid / QTPC, qk = (tid % QTPC) * PER;
  // an upper-triangular Q has no entries below row j0 + T - 1 in this column tile
  const int k_stop = q_upper ? min(n_in, j0 + T) : n_in;
  E ra[PER];
  double qr_[PER], qi_[PER];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int64_t m = m0 + am + u;
      const int k = k0 + ak;
      ra[u] = (m < N && k < n_in) ? A[m + (int64_t)k * lda] : zero<E>();
      const int kq = k0 + qk + u, j = j0 + qj;
      qr_[u] = 0;
      qi_[u] = 0;
      if (kq < n_in && j < n_out) {
        if constexpr (CPX) {
          qr_[u] = Q[2 * (kq + (int64_t)j * ldq)];
          qi_[u] = Q[2 * (kq + (int64_t)j * ldq) + 1];
        } else {
          qr_[u] = Q[kq + (int64_t)j * ldq];
        }
      }
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < k_stop; k0 += KC) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      R vr, vi;
      split<E>(ra[u], vr, vi);
      As[0][ak][am + u] = vr;
      if constexpr (CPX) As[1][ak][am + u] = vi;
      Qs[0][qk + u][qj] = (R)qr_[u];
      if constexpr (CPX) Qs[1][qk + u][qj] = (R)qi_[u];
    }
    __syncthreads();
    if (k0 + KC < k_stop) fetch(k0 + KC);
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      const int kq = kk + (lane >> 4), r16 = lane & 15;
      R q_r[WB], q_i[WB], a_r[WB], a_i[WB];
#pragma unroll
      for (int a = 0; a < WB; ++a) {
        q_r[a] = Qs[0][kq][wj + 16 * a + r16];  // Q^T[j][k]
        a_r[a] = As[0][kq][wm + 16 * a + r16];  // A^T[k][m]
        if constexpr (CPX) {
          q_i[a] = Qs[1][kq][wj + 16 * a + r16];
          a_i[a] = As[1][kq][wm + 16 * a + r16];
        }
      }
#pragma unroll
      for (int a = 0; a < WB; ++a)
#pragma unroll
        for (int b = 0; b < WB; ++b) {
          acc_r[a][b] = M::step(q_r[a], a_r[b], acc_r[a][b]);
          if constexpr (CPX) {
            // (A Q): re = Ar Qr - Ai Qi ; im = Ar Qi + Ai Qr
            acc_r[a][b] = M::step(-q_i[a], a_i[b], acc_r[a][b]);
            acc_i[a][b] = M::step(q_i[a], a_r[b], acc_i[a][b]);
            acc_i[a][b] = M::step(q_r[a], a_i[b], acc_i[a][b]);
          }
        }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < WB; ++a)
#pragma unroll
    for (int b = 0; b < WB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        int j = j0 + wj + 16 * a + M::row(lane, v);
        int64_t m = m0 + wm + 16 * b + (lane & 15);
        if (j < n_out && m < N) {
          if constexpr (CPX) {
            E o;
            o.re = acc_r[a][b][v];
            o.im = acc_i[a][b][v];
            Out[m + (int64_t)j * ldo] = o;
          } else {
            Out[m + (int64_t)j * ldo] = acc_r[a][b][v];
          }
        }
      }
}

template <typename E>
static int rotate_t(hipStream_t s, int64_t N, int n_in, int n_out, const E* A, int64_t lda, const double* Q, int ldq,
                    E* Out, int64_t ldo, int q_upper) {
  constexpr int T = gram_tile<E>::T;
  int tiles_n = (n_out + T - 1) / T;
  int64_t tiles_m = (N + T - 1) / T;
  int64_t total = tiles_m * tiles_n;
  if (total > (int64_t)INT32_MAX) return fail(SPARC_ESHAPE, "rotate: too many tiles");
  int remap = (total % 8 == 0) ? 1 : 0;
  rotate_kernel<E, T><<<(unsigned)total, 256, 0, s>>>(N, n_in, n_out, A, lda, Q, ldq, Out, ldo, tiles_n, remap,
                                                       total, q_upper);
  return check_launch("rotate_kernel");
}

int rotate(hipStream_t s, sparc_dtype dt, int64_t N, int32_t n_in, int32_t n_out, const void* A, int64_t lda,
           const void* Q, int32_t ldq, void* Out, int64_t ldo, int q_upper) {
  switch (dt) {
    case SPARC_R64: return rotate_t<double>(s, N, n_in, n_out, (const double*)A, lda, (const double*)Q, ldq, (double*)Out, ldo, q_upper);
    case SPARC_R32: return rotate_t<float>(s, N, n_in, n_out, (const float*)A, lda, (const double*)Q, ldq, (float*)Out, ldo, q_upper);
    case SPARC_C128: return rotate_t<cd>(s, N, n_in, n_out, (const cd*)A, lda, (const double*)Q, ldq, (cd*)Out, ldo, q_upper);
    case SPARC_C64: return rotate_t<cf>(s, N, n_in, n_out, (const cf*)A, lda, (const double*)Q, ldq, (cf*)Out, ldo, q_upper);
  }
  return fail(SPARC_EINVAL, "rotate: bad dtype");
}

}  // namespace sparc
