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
#include <cstdint>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "devmath.hpp"

namespace sparc {

sparc_ctx* g_timer_ctx = nullptr;

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
// Loader for one T x KC operand chunk (columns c of a tall block, KC consecutive rows k):
// element pairs (k, k+1) of one column per lane, 8 lanes per 128-byte column segment,
// so that every wave-wide load covers whole cache lines.  `vec` selects 16-byte loads
// (leading dimension even and base 16-byte aligned), else two 8-byte loads.
template <typename E, int T, int KC>
struct PairLoader {
  static constexpr int PAIRS = T * KC / 2 / 256;  // pairs per thread
  E v0[PAIRS], v1[PAIRS];
  __device__ __forceinline__ void fetch(const E* __restrict__ A, int64_t lda, int c0, int ncol, int64_t k0,
                                        int64_t k_end, bool vec) {
#pragma unroll
    for (int u = 0; u < PAIRS; ++u) {
      const int q = threadIdx.x + 256 * u;
      const int c = q / (KC / 2), kk = (q % (KC / 2)) * 2;
      const int64_t k = k0 + kk;
      v0[u] = zero<E>();
      v1[u] = zero<E>();
      if (c0 + c < ncol) {
        const E* p = A + k + (int64_t)(c0 + c) * lda;
        if constexpr (!elem<E>::is_cplx && sizeof(E) == 8) {
          if (vec && k + 1 < k_end) {
            double2 t = *(const double2*)p;
            v0[u] = t.x;
            v1[u] = t.y;
            continue;
          }
        }
        if (k < k_end) v0[u] = p[0];
        if (k + 1 < k_end) v1[u] = p[1];
      }
    }
  }
};

// One work-group: a T x T output tile of one slab.  4 waves in 2 x 2, each wave
// (T/2) x (T/2) = WB x WB MFMA blocks.  The next k-chunk is loaded into registers
// while the current one is consumed from LDS (k-major: operand reads are
// conflict-free rows).
template <typename E, int T, int KC>
__global__ __launch_bounds__(256) void gram_kernel(int64_t N, int na, int nb, const E* __restrict__ A, int64_t lda,
                                                   const E* __restrict__ B, int64_t ldb, int n_slab, int64_t slab_len,
                                                   int tiles_a, int n_tiles, int herm,
                                                   double* __restrict__ part, int xcd_remap, int vec) {
  typedef typename elem<E>::real R;
  constexpr bool CPX = elem<E>::is_cplx;
  constexpr int NCP = CPX ? 2 : 1;
  constexpr int WB = T / 32;
  typedef mfma_t<R> M;
  typedef PairLoader<E, T, KC> LD;
  __shared__ R As[NCP][KC][T + 1];
  __shared__ R Bs[NCP][KC][T + 1];

  // persistent: the grid (a multiple of 8 work-groups) walks the (slab, tile) items in rounds;
  // within a round the work-groups of one XCD take consecutive items (tiles of the same slab)
  const int total = n_slab * n_tiles;
  const int G = gridDim.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wi = (wv & 1) * (T / 2), wj = (wv >> 1) * (T / 2);
  for (int round = 0;; ++round) {
    const int bid = xcd_remap ? round * G + (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8)
                              : round * G + (int)blockIdx.x;
    if (bid >= total) break;
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

    typename M::acc acc_r[WB][WB], acc_i[WB][WB];
#pragma unroll
    for (int a = 0; a < WB; ++a)
#pragma unroll
      for (int b = 0; b < WB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) { acc_r[a][b][v] = 0; if constexpr (CPX) acc_i[a][b][v] = 0; }

    LD la, lb;
    la.fetch(A, lda, i0, na, k_beg, k_end, vec);
    lb.fetch(B, ldb, j0, nb, k_beg, k_end, vec);
    for (int64_t k0 = k_beg; k0 < k_end; k0 += KC) {
#pragma unroll
      for (int u = 0; u < LD::PAIRS; ++u) {
        const int q = tid + 256 * u;
        const int c = q / (KC / 2), kk = (q % (KC / 2)) * 2;
        R r0, i0_, r1, i1_;
        split<E>(la.v0[u], r0, i0_);
        split<E>(la.v1[u], r1, i1_);
        As[0][kk][c] = r0;
        As[0][kk + 1][c] = r1;
        if constexpr (CPX) { As[1][kk][c] = i0_; As[1][kk + 1][c] = i1_; }
        split<E>(lb.v0[u], r0, i0_);
        split<E>(lb.v1[u], r1, i1_);
        Bs[0][kk][c] = r0;
        Bs[0][kk + 1][c] = r1;
        if constexpr (CPX) { Bs[1][kk][c] = i0_; Bs[1][kk + 1][c] = i1_; }
      }
      __syncthreads();
      if (k0 + KC < k_end) {
        la.fetch(A, lda, i0, na, k0 + KC, k_end, vec);
        lb.fetch(B, ldb, j0, nb, k0 + KC, k_end, vec);
      }
#pragma unroll
      for (int kk = 0; kk < KC; kk += 4) {
        const int kq = kk + (lane >> 4), r16 = lane & 15;
        R a_r[WB], a_i[WB], b_r[WB], b_i[WB];
#pragma unroll
        for (int a = 0; a < WB; ++a) {
          a_r[a] = As[0][kq][wi + 16 * a + r16];
          b_r[a] = Bs[0][kq][wj + 16 * a + r16];
          if constexpr (CPX) {
            a_i[a] = As[1][kq][wi + 16 * a + r16];
            b_i[a] = Bs[1][kq][wj + 16 * a + r16];
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
}

// ---------------------------------------------------------------- gram, split-BF16 operands
// FP32 operands split into P bfloat16 pieces, x = x_0 + x_1 (+ x_2), each piece the
// round-to-nearest bf16 of what the previous pieces leave (exact differences).  A
// product of two elements is the sum of the piece products x_p y_q with p + q < P
// (P = 2: three products; P = 3: six), each exact in v_mfma_f32_16x16x16_bf16 with FP32
// accumulation.  The pieces are formed when a chunk is written to LDS (hardware
// round-to-nearest conversion), stored k-contiguous per column, so one 8-byte LDS read
// gives a lane the four k values of its MFMA operand.  Lane layout of the bf16 MFMA:
// A[i][k] in lane i + 16 (k / 4), element k % 4; B[k][j] likewise with j; result as for
// v_mfma_f32_16x16x4f32.
typedef short v4s __attribute__((ext_vector_type(4)));

template <int P>
__device__ __forceinline__ void bf16_pieces(float x, unsigned short out[P]) {
  float r = x;
#pragma unroll
  for (int q = 0; q < P; ++q) {
    const __bf16 h = (__bf16)r;
    out[q] = __builtin_bit_cast(unsigned short, h);
    if (q + 1 < P) r = r - (float)h;
  }
}

__device__ __forceinline__ v4s neg_bf16(v4s v) {
  return v ^ (v4s){(short)0x8000, (short)0x8000, (short)0x8000, (short)0x8000};
}

template <typename E, int T, int KC, int P>
__global__ __launch_bounds__(256) void gram_split_kernel(int64_t N, int na, int nb, const E* __restrict__ A,
                                                         int64_t lda, const E* __restrict__ B, int64_t ldb,
                                                         int n_slab, int64_t slab_len, int tiles_a, int n_tiles,
                                                         int herm, double* __restrict__ part, int xcd_remap,
                                                         int vec) {
  static_assert(sizeof(typename elem<E>::real) == 4, "split-BF16 products take FP32 operands");
  constexpr bool CPX = elem<E>::is_cplx;
  constexpr int NCP = CPX ? 2 : 1;
  constexpr int WB = T / 32;
  constexpr int KP = KC + 4;  // padded row: 8-byte aligned, rows spread over the banks
  typedef mfma_t<float> M;
  typedef PairLoader<E, T, KC> LD;
  __shared__ __attribute__((aligned(16))) unsigned short As[NCP][P][T][KP];
  __shared__ __attribute__((aligned(16))) unsigned short Bs[NCP][P][T][KP];

  const int total = n_slab * n_tiles;
  const int G = gridDim.x;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wi = (wv & 1) * (T / 2), wj = (wv >> 1) * (T / 2);
  for (int round = 0;; ++round) {
    const int bid = xcd_remap ? round * G + (int)(blockIdx.x % 8) * (G / 8) + (int)(blockIdx.x / 8)
                              : round * G + (int)blockIdx.x;
    if (bid >= total) break;
    const int slab = bid / n_tiles;
    const int tile = bid % n_tiles;
    int ti, tj;
    if (herm) {
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

    typename M::acc acc_r[WB][WB], acc_i[WB][WB];
#pragma unroll
    for (int a = 0; a < WB; ++a)
#pragma unroll
      for (int b = 0; b < WB; ++b)
#pragma unroll
        for (int v = 0; v < 4; ++v) { acc_r[a][b][v] = 0; if constexpr (CPX) acc_i[a][b][v] = 0; }

    LD la, lb;
    la.fetch(A, lda, i0, na, k_beg, k_end, vec);
    lb.fetch(B, ldb, j0, nb, k_beg, k_end, vec);
    for (int64_t k0 = k_beg; k0 < k_end; k0 += KC) {
#pragma unroll
      for (int u = 0; u < LD::PAIRS; ++u) {
        const int q = tid + 256 * u;
        const int c = q / (KC / 2), kk = (q % (KC / 2)) * 2;
        float r0, im0, r1, im1;
        unsigned short p0[P], p1[P];
        split<E>(la.v0[u], r0, im0);
        split<E>(la.v1[u], r1, im1);
        bf16_pieces<P>(r0, p0);
        bf16_pieces<P>(r1, p1);
#pragma unroll
        for (int t = 0; t < P; ++t) *(unsigned*)&As[0][t][c][kk] = (unsigned)p0[t] | ((unsigned)p1[t] << 16);
        if constexpr (CPX) {
          bf16_pieces<P>(im0, p0);
          bf16_pieces<P>(im1, p1);
#pragma unroll
          for (int t = 0; t < P; ++t) *(unsigned*)&As[1][t][c][kk] = (unsigned)p0[t] | ((unsigned)p1[t] << 16);
        }
        split<E>(lb.v0[u], r0, im0);
        split<E>(lb.v1[u], r1, im1);
        bf16_pieces<P>(r0, p0);
        bf16_pieces<P>(r1, p1);
#pragma unroll
        for (int t = 0; t < P; ++t) *(unsigned*)&Bs[0][t][c][kk] = (unsigned)p0[t] | ((unsigned)p1[t] << 16);
        if constexpr (CPX) {
          bf16_pieces<P>(im0, p0);
          bf16_pieces<P>(im1, p1);
#pragma unroll
          for (int t = 0; t < P; ++t) *(unsigned*)&Bs[1][t][c][kk] = (unsigned)p0[t] | ((unsigned)p1[t] << 16);
        }
      }
      __syncthreads();
      if (k0 + KC < k_end) {
        la.fetch(A, lda, i0, na, k0 + KC, k_end, vec);
        lb.fetch(B, ldb, j0, nb, k0 + KC, k_end, vec);
      }
      // one 16-wide k step at a time keeps the three-piece operands within two waves per SIMD
#pragma unroll(P == 2 ? KC / 16 : 1)
      for (int kk = 0; kk < KC; kk += 16) {
        const int kq = kk + 4 * (lane >> 4), r16 = lane & 15;
        v4s a_[NCP][P][WB], b_[NCP][P][WB];
#pragma unroll
        for (int cp = 0; cp < NCP; ++cp)
#pragma unroll
          for (int t = 0; t < P; ++t)
#pragma unroll
            for (int a = 0; a < WB; ++a) {
              a_[cp][t][a] = *(const v4s*)&As[cp][t][wi + 16 * a + r16][kq];
              b_[cp][t][a] = *(const v4s*)&Bs[cp][t][wj + 16 * a + r16][kq];
            }
#pragma unroll
        for (int a = 0; a < WB; ++a)
#pragma unroll
          for (int b = 0; b < WB; ++b)
#pragma unroll
            for (int ta = P - 1; ta >= 0; --ta)
#pragma unroll
              for (int tb = P - 1 - ta; tb >= 0; --tb) {
                acc_r[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_[0][ta][a], b_[0][tb][b], acc_r[a][b], 0, 0, 0);
                if constexpr (CPX) {
                  // conj(A)^T B: re += ar br + ai bi ; im += ar bi - ai br
                  acc_r[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_[1][ta][a], b_[1][tb][b], acc_r[a][b], 0, 0, 0);
                  acc_i[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a_[0][ta][a], b_[1][tb][b], acc_i[a][b], 0, 0, 0);
                  acc_i[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(neg_bf16(a_[1][ta][a]), b_[0][tb][b], acc_i[a][b], 0, 0, 0);
                }
              }
      }
      __syncthreads();
    }
    const int64_t mat = (int64_t)na * nb * NCP;
    double* Pp = part + (int64_t)slab * mat;
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
              Pp[2 * (i + (int64_t)j * na)] = (double)acc_r[a][b][v];
              Pp[2 * (i + (int64_t)j * na) + 1] = (double)acc_i[a][b][v];
            } else {
              Pp[i + (int64_t)j * na] = (double)acc_r[a][b][v];
            }
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
#pragma unroll 8
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

// The Hermitian form: one thread per element of the upper triangle (column j = block y,
// consecutive threads consecutive rows, so the partials are read in full lines), which
// writes the element and its mirror; the same sum in the same order as above.
__global__ __launch_bounds__(256) void gram_reduce_herm_kernel(int n, int n_slab, const double* __restrict__ part,
                                                               double* __restrict__ C, int ldc, int cplx) {
  const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y;
  if (i > j || i >= n) return;
  const int64_t mat = (int64_t)n * n * (cplx ? 2 : 1);
  const int64_t off = (i + (int64_t)j * n) * (cplx ? 2 : 1);
  double re = 0, im = 0;
#pragma unroll 8
  for (int s = 0; s < n_slab; ++s) {
    re += part[s * mat + off];
    if (cplx) im += part[s * mat + off + 1];
  }
  if (i == j) im = 0;
  if (cplx) {
    C[2 * (i + (int64_t)j * ldc)] = re;
    C[2 * (i + (int64_t)j * ldc) + 1] = im;
    if (i != j) {
      C[2 * (j + (int64_t)i * ldc)] = re;
      C[2 * (j + (int64_t)i * ldc) + 1] = -im;
    }
  } else {
    C[i + (int64_t)j * ldc] = re;
    if (i != j) C[j + (int64_t)i * ldc] = re;
  }
}

// The same sum for small outputs over many slabs: one wave per output element, lanes
// over the slabs (lane l takes slabs l, l + 64, ...), then a fixed butterfly.
__global__ __launch_bounds__(256) void gram_reduce_wave_kernel(int na, int nb, int n_slab,
                                                               const double* __restrict__ part, double* __restrict__ C,
                                                               int ldc, int cplx, int herm) {
  const int64_t idx = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (idx >= (int64_t)na * nb) return;
  int i = (int)(idx % na), j = (int)(idx / na);
  int si = i, sj = j;
  bool conj_ = false;
  if (herm && i > j) { si = j; sj = i; conj_ = true; }
  const int64_t mat = (int64_t)na * nb * (cplx ? 2 : 1);
  const int64_t off = (si + (int64_t)sj * na) * (cplx ? 2 : 1);
  double re = 0, im = 0;
  for (int s = lane; s < n_slab; s += 64) {
    re += part[s * mat + off];
    if (cplx) im += part[s * mat + off + 1];
  }
  re = wave_sum(re);
  if (cplx) im = wave_sum(im);
  if (lane != 0) return;
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

// Most slabs a product may use (sizes the partial-sum workspace): 256 in general, up to
// 2048 for skinny products (na * nb <= 32, e.g. the Lanczos projections), so that these
// too spread over the chip.  cap * na * nb never decreases with na * nb, so a workspace
// sized for a product also fits every smaller one.
static int64_t gram_cap(int na, int nb) {
  const int64_t e = std::max<int64_t>(1, (int64_t)na * nb);
  return std::max<int64_t>(256, std::min<int64_t>(2048, 65536 / e));
}

static GramPlan gram_plan(int64_t N, int na, int nb, bool herm, int n_cu, int T, int64_t slabs = 0) {
  GramPlan p;
  p.tiles_a = (na + T - 1) / T;
  p.tiles_b = (nb + T - 1) / T;
  p.n_tiles = 0;
  for (int tj = 0; tj < p.tiles_b; ++tj)
    for (int ti = 0; ti < p.tiles_a; ++ti)
      if (!herm || ti <= tj) p.n_tiles++;
  // slabs of 2048 nodes; where that leaves fewer (slab, tile) items than two rounds of
  // work-groups on every CU (four for small outputs), shorter slabs down to 256 nodes
  const int64_t items_min = (int64_t)(((int64_t)na * nb <= 1024) ? 4 : 2) * std::max(n_cu, 1);
  int64_t s = N / 2048;
  if (s * p.n_tiles < items_min) s = std::min<int64_t>((items_min + p.n_tiles - 1) / p.n_tiles, N / 256);
  if (slabs > 0) s = slabs;  // a tuned count
  s = std::max<int64_t>(1, std::min<int64_t>(gram_cap(na, nb), s));
  p.slab_len = (N + s - 1) / s;
  p.slab_len = ((p.slab_len + 15) / 16) * 16;
  p.n_slab = (int)((N + p.slab_len - 1) / p.slab_len);
  return p;
}

size_t gram_work_bytes(int64_t N, int32_t n_a, int32_t n_b, sparc_dtype dt) {
  (void)N;
  return (size_t)gram_cap(n_a, n_b) * n_a * n_b * 8 * (dtype_complex(dt) ? 2 : 1);
}

// tile edge of the native products: the smallest of 32, 64 and the type's full tile that
// covers the larger dimension of the output (less padding in the MFMA blocks)
template <typename E>
static int native_tile(int na, int nb) {
  const int m = std::max(na, nb);
  if (m <= 32) return 32;
  if (m <= 64 || elem<E>::is_cplx) return 64;
  return 128;
}

template <typename E, int T>
static void gram_native_launch(hipStream_t s, int grid, int64_t N, int na, int nb, const E* A, int64_t lda,
                               const E* B, int64_t ldb, const GramPlan& p, int herm, double* part, int remap,
                               int vec) {
  gram_kernel<E, T, 16><<<grid, 256, 0, s>>>(N, na, nb, A, lda, B, ldb, p.n_slab, p.slab_len, p.tiles_a, p.n_tiles,
                                              herm, part, remap, vec);
}

// one product with tile edge T and (when slabs > 0) that many slabs
template <typename E>
static int gram_launch(hipStream_t s, int64_t N, int na, int nb, const E* A, int64_t lda, const E* B, int64_t ldb,
                       void* C, int ldc, void* work, size_t work_bytes, int n_cu, bool herm, sparc_gemm_mode mode, int T,
                       int64_t slabs) {
  GramPlan p = gram_plan(N, na, nb, herm, n_cu, T, slabs);
  // persistent grid: two work-groups per CU (a multiple of 8), at most one per item
  const int items = p.n_slab * p.n_tiles;
  int grid = std::min(items, 2 * n_cu);
  if (grid >= 8) grid -= grid % 8;
  const bool cplx = elem<E>::is_cplx;
  size_t part_bytes = (size_t)p.n_slab * na * nb * 8 * (cplx ? 2 : 1);
  if (part_bytes > work_bytes) return fail(SPARC_ENOMEM, "gram: workspace %zu < %zu bytes", work_bytes, part_bytes);
  double* part = (double*)work;
  int remap = (grid % 8 == 0) ? 1 : 0;
  int tmr = timer_begin(g_timer_ctx, "gram");
  const int vec = (lda % 2 == 0 && ldb % 2 == 0 && ((uintptr_t)A % 16) == 0 && ((uintptr_t)B % 16) == 0) ? 1 : 0;
  bool launched = false;
  if constexpr (sizeof(typename elem<E>::real) == 4) {
    constexpr int TS = gram_tile<E>::T;
    if (mode == SPARC_GEMM_BF16X3) {
      gram_split_kernel<E, TS, 32, 2><<<grid, 256, 0, s>>>(N, na, nb, A, lda, B, ldb, p.n_slab, p.slab_len, p.tiles_a,
                                                            p.n_tiles, herm ? 1 : 0, part, remap, vec);
      launched = true;
    } else if (mode == SPARC_GEMM_BF16X6) {
      gram_split_kernel<E, TS, 32, 3><<<grid, 256, 0, s>>>(N, na, nb, A, lda, B, ldb, p.n_slab, p.slab_len, p.tiles_a,
                                                            p.n_tiles, herm ? 1 : 0, part, remap, vec);
      launched = true;
    }
  }
  if (!launched) {
    if (T == 32) gram_native_launch<E, 32>(s, grid, N, na, nb, A, lda, B, ldb, p, herm ? 1 : 0, part, remap, vec);
    else if (T == 64) gram_native_launch<E, 64>(s, grid, N, na, nb, A, lda, B, ldb, p, herm ? 1 : 0, part, remap, vec);
    else if constexpr (!elem<E>::is_cplx)
      gram_native_launch<E, 128>(s, grid, N, na, nb, A, lda, B, ldb, p, herm ? 1 : 0, part, remap, vec);
  }
  timer_end(g_timer_ctx, tmr);
  SPARC_TRY(check_launch("gram_kernel"));
  int64_t ne = (int64_t)na * nb;
  if (ne <= 4096 && p.n_slab > 64)
    gram_reduce_wave_kernel<<<(unsigned)((ne + 3) / 4), 256, 0, s>>>(na, nb, p.n_slab, part, (double*)C, ldc,
                                                                     cplx ? 1 : 0, herm ? 1 : 0);
  else if (herm && na == nb && nb <= 65535)
    gram_reduce_herm_kernel<<<dim3((unsigned)((na + 255) / 256), (unsigned)nb), 256, 0, s>>>(na, p.n_slab, part,
                                                                                           (double*)C, ldc,
                                                                                           cplx ? 1 : 0);
  else
    gram_reduce_kernel<<<(unsigned)((ne + 255) / 256), 256, 0, s>>>(na, nb, p.n_slab, part, (double*)C, ldc,
                                                                    cplx ? 1 : 0, herm ? 1 : 0);
  return check_launch("gram_reduce_kernel");
}

// ------------------------------------------------------------ GEMM shape tuner
// With a context that autotunes, the first product of a new shape (N, n_a, n_b, type,
// Hermitian, one or two operands) times the tile edges next to the heuristic's
// (32 / 64 / 128) and, for the Gram, slab counts of half, one and two times the plan's,
// each launch once to warm up and twice timed with HIP events, and keeps the fastest;
// the heuristic's own choice is among the candidates.  Later products of that shape
// reuse it.
struct GemmChoice { int T; int64_t slabs; };
static std::mutex g_gemm_tune_mu;
static std::map<std::tuple<int64_t, int, int, int, int, int>, GemmChoice> g_gemm_tune;

static bool gemm_lookup(const std::tuple<int64_t, int, int, int, int, int>& key, GemmChoice* c) {
  std::lock_guard<std::mutex> lk(g_gemm_tune_mu);
  auto it = g_gemm_tune.find(key);
  if (it == g_gemm_tune.end()) return false;
  *c = it->second;
  return true;
}

static void gemm_store(const std::tuple<int64_t, int, int, int, int, int>& key, GemmChoice c) {
  std::lock_guard<std::mutex> lk(g_gemm_tune_mu);
  g_gemm_tune[key] = c;
}

template <typename E>
static std::vector<int> tile_candidates(int T0) {
  std::vector<int> v;
  for (int T : {32, 64, 128}) {
    if (T == 128 && elem<E>::is_cplx) continue;
    if (T >= T0 / 2 && T <= T0 * 2) v.push_back(T);
  }
  return v;
}

// times fn() (one warm-up, then the best of two timed calls) on stream s; -1 on failure
template <typename F>
static float time_best(hipStream_t s, hipEvent_t e0, hipEvent_t e1, F&& fn) {
  if (fn() != SPARC_OK) return -1.0f;
  float best = 1e30f;
  for (int r = 0; r < 2; ++r) {
    hipEventRecord(e0, s);
    if (fn() != SPARC_OK) return -1.0f;
    hipEventRecord(e1, s);
    hipEventSynchronize(e1);
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    best = std::min(best, ms);
  }
  return best;
}

template <typename E>
static int gram_t(hipStream_t s, int64_t N, int na, int nb, const E* A, int64_t lda, const E* B, int64_t ldb, void* C,
                  int ldc, void* work, size_t work_bytes, int n_cu, bool herm_result,
                  sparc_gemm_mode mode = SPARC_GEMM_NATIVE, sparc_ctx* tune = nullptr) {
  const bool herm = (na == nb) && (herm_result || ((A == B) && (lda == ldb)));
  const bool split = mode != SPARC_GEMM_NATIVE;
  if constexpr (sizeof(typename elem<E>::real) == 8)
    if (split) return fail(SPARC_EINVAL, "gram: split-BF16 modes take FP32 blocks");
  GemmChoice c{split ? gram_tile<E>::T : native_tile<E>(na, nb), 0};
  if (split || !tune || !tune->autotune)
    return gram_launch<E>(s, N, na, nb, A, lda, B, ldb, C, ldc, work, work_bytes, n_cu, herm, mode, c.T, c.slabs);
  // kind 0: one operand (A^H A), 2: two (they read twice the data)
  const int kind = (A == B && lda == ldb) ? 0 : 2;
  const auto key = std::make_tuple(N, na, nb, (int)(sizeof(E) * 2 + (elem<E>::is_cplx ? 1 : 0)), herm ? 1 : 0, kind);
  if (!gemm_lookup(key, &c)) {
    hipEvent_t e0, e1;
    SPARC_HIP(hipEventCreate(&e0));
    SPARC_HIP(hipEventCreate(&e1));
    const bool timing = tune->timing;
    tune->timing = false;
    const int cap_bytes_slabs = (int)std::min<int64_t>(gram_cap(na, nb),
                                                       (int64_t)(work_bytes / ((size_t)na * nb * 8 *
                                                                               (elem<E>::is_cplx ? 2 : 1))));
    float best = 1e30f;
    GemmChoice pick = c;
    for (int T : tile_candidates<E>(c.T)) {
      const int64_t s0 = gram_plan(N, na, nb, herm, n_cu, T).n_slab;
      for (int64_t sl : {s0, s0 / 2, s0 * 2}) {
        if (sl < 1 || sl > cap_bytes_slabs || (sl != s0 && N / sl < 64)) continue;
        const float ms = time_best(s, e0, e1, [&]() {
          return gram_launch<E>(s, N, na, nb, A, lda, B, ldb, C, ldc, work, work_bytes, n_cu, herm, mode, T, sl);
        });
        if (ms >= 0 && ms < best) { best = ms; pick = GemmChoice{T, sl}; }
      }
    }
    tune->timing = timing;
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    c = pick;
    gemm_store(key, c);
  }
  return gram_launch<E>(s, N, na, nb, A, lda, B, ldb, C, ldc, work, work_bytes, n_cu, herm, mode, c.T, c.slabs);
}

int gram(hipStream_t s, sparc_dtype dt, int64_t N, int32_t na, int32_t nb, const void* A, int64_t lda, const void* B,
         int64_t ldb, void* C, int32_t ldc, void* work, size_t work_bytes, sparc_gemm_mode mode, int n_cu,
         bool herm_result, sparc_ctx* tune) {
  switch (dt) {
    case SPARC_R64: return gram_t<double>(s, N, na, nb, (const double*)A, lda, (const double*)B, ldb, C, ldc, work, work_bytes, n_cu, herm_result, mode, tune);
    case SPARC_R32: return gram_t<float>(s, N, na, nb, (const float*)A, lda, (const float*)B, ldb, C, ldc, work, work_bytes, n_cu, herm_result, mode, tune);
    case SPARC_C128: return gram_t<cd>(s, N, na, nb, (const cd*)A, lda, (const cd*)B, ldb, C, ldc, work, work_bytes, n_cu, herm_result, mode, tune);
    case SPARC_C64: return gram_t<cf>(s, N, na, nb, (const cf*)A, lda, (const cf*)B, ldb, C, ldc, work, work_bytes, n_cu, herm_result, mode, tune);
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
                                                     int64_t total, int q_upper, int vec, int qvec) {
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
  // A loader: pairs of consecutive rows, T/2 lanes per column (whole cache lines per wave);
  // Q loader: pairs of consecutive k of one column j, KC/2 lanes per column
  constexpr int APAIRS = T * KC / 2 / 256;
  constexpr int QPAIRS = T * KC / 2 / 256;
  // an upper-triangular Q has no entries below row j0 + T - 1 in this column tile
  const int k_stop = q_upper ? min(n_in, j0 + T) : n_in;
  E ra0[APAIRS], ra1[APAIRS];
  double qr0[QPAIRS], qr1[QPAIRS], qi0[QPAIRS], qi1[QPAIRS];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < APAIRS; ++u) {
      const int q = tid + 256 * u;
      const int k = k0 + q / (T / 2);
      const int64_t m = m0 + (q % (T / 2)) * 2;
      ra0[u] = zero<E>();
      ra1[u] = zero<E>();
      if (k < n_in) {
        const E* p = A + m + (int64_t)k * lda;
        bool done = false;
        if constexpr (!elem<E>::is_cplx && sizeof(E) == 8) {
          if (vec && m + 1 < N) {
            double2 t = *(const double2*)p;
            ra0[u] = t.x;
            ra1[u] = t.y;
            done = true;
          }
        }
        if (!done) {
          if (m < N) ra0[u] = p[0];
          if (m + 1 < N) ra1[u] = p[1];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < QPAIRS; ++u) {
      const int q = tid + 256 * u;
      const int j = j0 + q / (KC / 2), kq = k0 + (q % (KC / 2)) * 2;
      qr0[u] = qr1[u] = qi0[u] = qi1[u] = 0;
      if (j < n_out) {
        if constexpr (CPX) {
          const double* p = Q + 2 * (kq + (int64_t)j * ldq);
          if (kq < n_in) { qr0[u] = p[0]; qi0[u] = p[1]; }
          if (kq + 1 < n_in) { qr1[u] = p[2]; qi1[u] = p[3]; }
        } else {
          const double* p = Q + kq + (int64_t)j * ldq;
          if (qvec && kq + 1 < n_in) {
            double2 t = *(const double2*)p;
            qr0[u] = t.x;
            qr1[u] = t.y;
          } else {
            if (kq < n_in) qr0[u] = p[0];
            if (kq + 1 < n_in) qr1[u] = p[1];
          }
        }
      }
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < k_stop; k0 += KC) {
#pragma unroll
    for (int u = 0; u < APAIRS; ++u) {
      const int q = tid + 256 * u;
      const int k = q / (T / 2), m = (q % (T / 2)) * 2;
      R vr, vi;
      split<E>(ra0[u], vr, vi);
      As[0][k][m] = vr;
      if constexpr (CPX) As[1][k][m] = vi;
      split<E>(ra1[u], vr, vi);
      As[0][k][m + 1] = vr;
      if constexpr (CPX) As[1][k][m + 1] = vi;
    }
#pragma unroll
    for (int u = 0; u < QPAIRS; ++u) {
      const int q = tid + 256 * u;
      const int jj = q / (KC / 2), kk = (q % (KC / 2)) * 2;
      Qs[0][kk][jj] = (R)qr0[u];
      Qs[0][kk + 1][jj] = (R)qr1[u];
      if constexpr (CPX) {
        Qs[1][kk][jj] = (R)qi0[u];
        Qs[1][kk + 1][jj] = (R)qi1[u];
      }
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

template <typename E, int T>
static void rotate_launch(hipStream_t s, int64_t total, int64_t N, int n_in, int n_out, const E* A, int64_t lda,
                          const double* Q, int ldq, E* Out, int64_t ldo, int tiles_n, int remap, int q_upper, int vec,
                          int qvec) {
  rotate_kernel<E, T><<<(unsigned)total, 256, 0, s>>>(N, n_in, n_out, A, lda, Q, ldq, Out, ldo, tiles_n, remap,
                                                       total, q_upper, vec, qvec);
}

template <typename E>
static int rotate_run(hipStream_t s, int64_t N, int n_in, int n_out, const E* A, int64_t lda, const double* Q, int ldq,
                      E* Out, int64_t ldo, int q_upper, int T) {
  int tiles_n = (n_out + T - 1) / T;
  int64_t tiles_m = (N + T - 1) / T;
  int64_t total = tiles_m * tiles_n;
  if (total > (int64_t)INT32_MAX) return fail(SPARC_ESHAPE, "rotate: too many tiles");
  int remap = (total % 8 == 0) ? 1 : 0;
  int tmr = timer_begin(g_timer_ctx, "rotate");
  const int vec = (lda % 2 == 0 && ((uintptr_t)A % 16) == 0) ? 1 : 0;
  const int qvec = (ldq % 2 == 0 && ((uintptr_t)Q % 16) == 0) ? 1 : 0;
  if (T == 32) rotate_launch<E, 32>(s, total, N, n_in, n_out, A, lda, Q, ldq, Out, ldo, tiles_n, remap, q_upper, vec, qvec);
  else if (T == 64) rotate_launch<E, 64>(s, total, N, n_in, n_out, A, lda, Q, ldq, Out, ldo, tiles_n, remap, q_upper, vec, qvec);
  else if constexpr (!elem<E>::is_cplx)
    rotate_launch<E, 128>(s, total, N, n_in, n_out, A, lda, Q, ldq, Out, ldo, tiles_n, remap, q_upper, vec, qvec);
  timer_end(g_timer_ctx, tmr);
  return check_launch("rotate_kernel");
}

template <typename E>
static int rotate_t(hipStream_t s, int64_t N, int n_in, int n_out, const E* A, int64_t lda, const double* Q, int ldq,
                    E* Out, int64_t ldo, int q_upper, sparc_ctx* tune) {
  // tile edge from the output width (rows of A per work-group = output columns per tile);
  // tuned like the Gram's when the context asks for it (Out is rewritten by every candidate)
  int T = n_out <= 32 ? 32 : (n_out <= 64 || elem<E>::is_cplx) ? 64 : 128;
  if (tune && tune->autotune) {
    const auto key = std::make_tuple(N, n_in, n_out, (int)(sizeof(E) * 2 + (elem<E>::is_cplx ? 1 : 0)), q_upper, 1);
    GemmChoice c{T, 0};
    if (!gemm_lookup(key, &c)) {
      hipEvent_t e0, e1;
      SPARC_HIP(hipEventCreate(&e0));
      SPARC_HIP(hipEventCreate(&e1));
      const bool timing = tune->timing;
      tune->timing = false;
      float best = 1e30f;
      for (int Tc : tile_candidates<E>(T)) {
        const float ms = time_best(s, e0, e1, [&]() {
          return rotate_run<E>(s, N, n_in, n_out, A, lda, Q, ldq, Out, ldo, q_upper, Tc);
        });
        if (ms >= 0 && ms < best) { best = ms; c.T = Tc; }
      }
      tune->timing = timing;
      hipEventDestroy(e0);
      hipEventDestroy(e1);
      gemm_store(key, c);
    }
    T = c.T;
  }
  return rotate_run<E>(s, N, n_in, n_out, A, lda, Q, ldq, Out, ldo, q_upper, T);
}

// ---------------------------------------------------------------- rotate, split-BF16 (x3) from pre-split pieces
// The FP32 block is split once into two bf16 pieces laid out for the B operand of
// v_mfma_f32_16x16x16_bf16: pieces[t][c][k/4][m][k%4] (t piece, c real/imaginary part,
// k column of A, m row), so a lane's four k values of row m are one 8-byte load; Q
// (FP64, rounded to FP32) likewise as Qp[t][c][k/4][j][k%4].  The rotation then
// reads its operands straight from global memory (L2) in MFMA layout, without LDS, and
// sums the three piece products with p + q < 2.  n_in must be a multiple of 16.
template <typename E>
__global__ __launch_bounds__(256) void split_block_kernel(int64_t N, int n, const E* __restrict__ A, int64_t lda,
                                                          unsigned short* __restrict__ out) {
  constexpr int NCP = elem<E>::is_cplx ? 2 : 1;
  const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int kb = blockIdx.y, KB = gridDim.y;
  if (m >= N) return;
  unsigned short pc[2][NCP][4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int k = 4 * kb + q;
    float vr = 0.0f, vi = 0.0f;
    if (k < n) split<E>(A[m + (int64_t)k * lda], vr, vi);
    unsigned short t2[2];
    bf16_pieces<2>(vr, t2);
    pc[0][0][q] = t2[0];
    pc[1][0][q] = t2[1];
    if constexpr (NCP == 2) {
      bf16_pieces<2>(vi, t2);
      pc[0][1][q] = t2[0];
      pc[1][1][q] = t2[1];
    }
  }
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int c = 0; c < NCP; ++c) {
      v4s v = {(short)pc[t][c][0], (short)pc[t][c][1], (short)pc[t][c][2], (short)pc[t][c][3]};
      *(v4s*)&out[((((int64_t)t * NCP + c) * KB + kb) * N + m) * 4] = v;
    }
}

template <bool CPX>
__global__ void split_q_kernel(int n_in, int n_out, const double* __restrict__ Q, int ldq,
                               unsigned short* __restrict__ out) {
  constexpr int NCP = CPX ? 2 : 1;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)n_in * n_out) return;
  const int k = (int)(i % n_in), j = (int)(i / n_in);
#pragma unroll
  for (int c = 0; c < NCP; ++c) {
    const double q = CPX ? Q[2 * (k + (int64_t)j * ldq) + c] : Q[k + (int64_t)j * ldq];
    unsigned short t2[2];
    bf16_pieces<2>((float)q, t2);
#pragma unroll
    for (int t = 0; t < 2; ++t) out[((((int64_t)t * NCP + c) * (n_in / 4) + k / 4) * n_out + j) * 4 + k % 4] = t2[t];
  }
}

template <typename E, int T>
__global__ __launch_bounds__(256) void rotate_pieces_kernel(int64_t N, int n_in, int n_out,
                                                            const unsigned short* __restrict__ Ap,
                                                            const unsigned short* __restrict__ Qp,
                                                            E* __restrict__ Out, int64_t ldo, int tiles_n,
                                                            int xcd_remap, int64_t total, int q_upper) {
  constexpr bool CPX = elem<E>::is_cplx;
  constexpr int NCP = CPX ? 2 : 1;
  constexpr int WB = T / 32;
  typedef mfma_t<float> M;
  int64_t bid = blockIdx.x;
  if (xcd_remap) bid = (bid % 8) * (total / 8) + bid / 8;
  const int tn = (int)(bid % tiles_n);
  const int64_t m0 = (bid / tiles_n) * T;
  const int j0 = tn * T;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wj = (wv & 1) * (T / 2), wm = (wv >> 1) * (T / 2);
  const int r16 = lane & 15;
  const int KB = n_in / 4;
  typename M::acc acc_r[WB][WB], acc_i[WB][WB];
#pragma unroll
  for (int a = 0; a < WB; ++a)
#pragma unroll
    for (int b = 0; b < WB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) { acc_r[a][b][v] = 0; if constexpr (CPX) acc_i[a][b][v] = 0; }
  const int k_stop = q_upper ? min(n_in, j0 + T) : n_in;  // a multiple of 16
  const v4s zero4 = {0, 0, 0, 0};
  for (int k0 = 0; k0 < k_stop; k0 += 16) {
    const int kq = k0 + 4 * (lane >> 4);
    v4s q_[NCP][2][WB], a_[NCP][2][WB];
#pragma unroll
    for (int c = 0; c < NCP; ++c)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int a = 0; a < WB; ++a) {
          const int j = j0 + wj + 16 * a + r16;
          const int64_t m = m0 + wm + 16 * a + r16;
          q_[c][t][a] = j < n_out ? *(const v4s*)&Qp[((((int64_t)t * NCP + c) * KB + kq / 4) * n_out + j) * 4] : zero4;
          a_[c][t][a] = m < N ? *(const v4s*)&Ap[((((int64_t)t * NCP + c) * KB + kq / 4) * N + m) * 4] : zero4;
        }
#pragma unroll
    for (int a = 0; a < WB; ++a)
#pragma unroll
      for (int b = 0; b < WB; ++b)
#pragma unroll
        for (int tq = 1; tq >= 0; --tq)
#pragma unroll
          for (int ta = 1 - tq; ta >= 0; --ta) {
            acc_r[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(q_[0][tq][a], a_[0][ta][b], acc_r[a][b], 0, 0, 0);
            if constexpr (CPX) {
              // (A Q): re = Ar Qr - Ai Qi ; im = Ar Qi + Ai Qr
              acc_r[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(neg_bf16(q_[1][tq][a]), a_[1][ta][b], acc_r[a][b], 0, 0, 0);
              acc_i[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(q_[1][tq][a], a_[0][ta][b], acc_i[a][b], 0, 0, 0);
              acc_i[a][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(q_[0][tq][a], a_[1][ta][b], acc_i[a][b], 0, 0, 0);
            }
          }
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
static int rotate_x3_t(hipStream_t s, int64_t N, int n_in, int n_out, const E* A, int64_t lda, const double* Q,
                       int ldq, E* Out, int64_t ldo, int q_upper, void* a_pieces, void* q_pieces) {
  constexpr int T = gram_tile<E>::T;
  constexpr bool CPX = elem<E>::is_cplx;
  int tmr = timer_begin(g_timer_ctx, "rotate");
  split_block_kernel<E><<<dim3((unsigned)((N + 255) / 256), (unsigned)(n_in / 4)), 256, 0, s>>>(
      N, n_in, A, lda, (unsigned short*)a_pieces);
  split_q_kernel<CPX><<<(unsigned)(((int64_t)n_in * n_out + 255) / 256), 256, 0, s>>>(n_in, n_out, Q, ldq,
                                                                                     (unsigned short*)q_pieces);
  const int tiles_n = (n_out + T - 1) / T;
  const int64_t total = ((N + T - 1) / T) * tiles_n;
  if (total > (int64_t)INT32_MAX) return fail(SPARC_ESHAPE, "rotate: too many tiles");
  const int remap = (total % 8 == 0) ? 1 : 0;
  rotate_pieces_kernel<E, T><<<(unsigned)total, 256, 0, s>>>(N, n_in, n_out, (const unsigned short*)a_pieces,
                                                              (const unsigned short*)q_pieces, Out, ldo, tiles_n,
                                                              remap, total, q_upper);
  timer_end(g_timer_ctx, tmr);
  return check_launch("rotate_pieces_kernel");
}

int rotate_split_x3(hipStream_t s, sparc_dtype dt, int64_t N, int32_t n_in, int32_t n_out, const void* A,
                    int64_t lda, const void* Q, int32_t ldq, void* Out, int64_t ldo, int q_upper, void* a_pieces,
                    void* q_pieces) {
  if (n_in % 16 != 0) return fail(SPARC_EINVAL, "rotate_split_x3: n_in=%d is not a multiple of 16", n_in);
  if (n_in / 4 > 65535) return fail(SPARC_ESHAPE, "rotate_split_x3: n_in=%d too large", n_in);
  switch (dt) {
    case SPARC_R32: return rotate_x3_t<float>(s, N, n_in, n_out, (const float*)A, lda, (const double*)Q, ldq, (float*)Out, ldo, q_upper, a_pieces, q_pieces);
    case SPARC_C64: return rotate_x3_t<cf>(s, N, n_in, n_out, (const cf*)A, lda, (const double*)Q, ldq, (cf*)Out, ldo, q_upper, a_pieces, q_pieces);
    default: break;
  }
  return fail(SPARC_EINVAL, "rotate_split_x3: FP32 / complex64 blocks only");
}

int rotate(hipStream_t s, sparc_dtype dt, int64_t N, int32_t n_in, int32_t n_out, const void* A, int64_t lda,
           const void* Q, int32_t ldq, void* Out, int64_t ldo, int q_upper, sparc_ctx* tune) {
  switch (dt) {
    case SPARC_R64: return rotate_t<double>(s, N, n_in, n_out, (const double*)A, lda, (const double*)Q, ldq, (double*)Out, ldo, q_upper, tune);
    case SPARC_R32: return rotate_t<float>(s, N, n_in, n_out, (const float*)A, lda, (const double*)Q, ldq, (float*)Out, ldo, q_upper, tune);
    case SPARC_C128: return rotate_t<cd>(s, N, n_in, n_out, (const cd*)A, lda, (const double*)Q, ldq, (cd*)Out, ldo, q_upper, tune);
    case SPARC_C64: return rotate_t<cf>(s, N, n_in, n_out, (const cf*)A, lda, (const double*)Q, ldq, (cf*)Out, ldo, q_upper, tune);
  }
  return fail(SPARC_EINVAL, "rotate: bad dtype");
}

}  // namespace sparc
