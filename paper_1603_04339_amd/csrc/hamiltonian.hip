// Application of the finite-difference Hamiltonian to a block of orbitals:
// the fused stencil + local potential + non-local scatter step that every H*X,
// Chebyshev recurrence step and Lanczos step runs, and the non-local gather
// (projections of the orbitals onto the Kleinman-Bylander projectors).
//
// Stencil step (one work-group = one TX x TY column tile of one orbital, a
// chunk of z planes): the tile streams along z.  Each thread keeps the 2*NO+1
// values of its own (x, y) column around the current plane in registers
// (z-direction taps); the current plane, with NO-wide x and y halos, is staged
// in LDS (double-buffered, one barrier per plane) for the x and y taps.  Loads
// are x-fastest and coalesced; nodes outside the cell are fetched from their
// periodic image with the Bloch factor e^{i k_s L_s w}.
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "devmath.hpp"

namespace sparc {

template <typename E>
struct StepArgs {
  typedef typename elem<E>::real R;
  int n1, n2, n3;
  int tiles_x, zchunk;
  int tiles, nz;     // tiles per plane, z chunks
  int ns;            // orbitals
  int64_t ldx, ldz, ldo;
  const E* __restrict__ x;
  const E* z;
  E* out;
  const R* __restrict__ veff;
  R centre;        // a * centre coefficient of -1/2 Lap_h
  R tx[8], ty[8], tz[8];
  R va, vb, zc;    // out = lap*a + (a V + b) x + zc z
  double kl[3];    // k_s L_s
};

template <typename E>
__device__ __forceinline__ void bloch_factor(const double* kl, int wx, int wy, int wz, typename elem<E>::real& c,
                                             typename elem<E>::real& s) {
  if constexpr (elem<E>::is_cplx) {
    double th = kl[0] * wx + kl[1] * wy + kl[2] * wz;
    if (th == 0.0) {
      c = 1;
      s = 0;
    } else {
      double sn, cs;
      sincos(th, &sn, &cs);
      c = (typename elem<E>::real)cs;
      s = (typename elem<E>::real)sn;
    }
  } else {
    c = 1;
    s = 0;
  }
}

template <typename E, int TX, int TY, int NO>
__device__ __forceinline__ void hstep_body(const StepArgs<E>& A, int tile, int n, int zi,
                                           E (&plane)[2][(TY + 2 * NO) * (TX + 2 * NO)]) {
  typedef typename elem<E>::real R;
  constexpr int NT = TX * TY;
  constexpr int PX = TX + 2 * NO;
  constexpr int HC = 2 * NO * (TX + TY);         // halo cells of one plane (no corners)
  constexpr int HM = (HC + NT - 1) / NT;         // halo cells per thread

  const int tid = threadIdx.x;
  const int hx = tid % TX, hy = tid / TX;
  const int x0 = (tile % A.tiles_x) * TX, y0 = (tile / A.tiles_x) * TY;
  const int zb = zi * A.zchunk;
  const int ze = min(A.n3, zb + A.zchunk);
  const int n1 = A.n1, n2 = A.n2, n3 = A.n3;
  const int64_t plane_sz = (int64_t)n1 * n2;

  const E* __restrict__ xc = A.x + (int64_t)n * A.ldx;
  // own column: extended coordinates, periodic source and Bloch factor in x, y
  const int ex = x0 + hx, ey = y0 + hy;
  const int wx = floordiv_i(ex, n1), wy = floordiv_i(ey, n2);
  const int col = (ex - wx * n1) + n1 * (ey - wy * n2);
  const bool inside = (ex < n1) && (ey < n2);
  R cxy = 1, sxy = 0;
  bloch_factor<E>(A.kl, wx, wy, 0, cxy, sxy);
  const int own = (hy + NO) * PX + hx + NO;

  // halo cells owned by this thread: LDS slot, offset inside a plane, Bloch factor
  int h_lds[HM], h_off[HM];
  R h_c[HM], h_s[HM];
#pragma unroll
  for (int u = 0; u < HM; ++u) {
    const int c = tid + u * NT;
    h_lds[u] = -1;
    h_off[u] = 0;
    h_c[u] = 1;
    h_s[u] = 0;
    if (c < HC) {
      int cx, cy;
      if (c < 2 * NO * TY) {  // x strips
        const int r = c / (2 * NO), k = c % (2 * NO);
        cy = r;
        cx = (k < NO) ? (k - NO) : (TX + k - NO);
      } else {  // y strips
        const int c2 = c - 2 * NO * TY;
        const int r = c2 / TX, k = c2 % TX;
        cx = k;
        cy = (r < NO) ? (r - NO) : (TY + r - NO);
      }
      const int gx = x0 + cx, gy = y0 + cy;
      const int hwx = floordiv_i(gx, n1), hwy = floordiv_i(gy, n2);
      h_off[u] = (gx - hwx * n1) + n1 * (gy - hwy * n2);
      h_lds[u] = (cy + NO) * PX + cx + NO;
      bloch_factor<E>(A.kl, hwx, hwy, 0, h_c[u], h_s[u]);
    }
  }

  // z-direction register queue q[d] = x(column, z - NO + d); the plane index of the
  // next load and its number of cell wraps are advanced without divisions
  int zl = zb - NO;
  int wz = floordiv_i(zl, n3);
  int sz = zl - wz * n3;
  auto load_next = [&]() -> E {
    E v = xc[col + plane_sz * sz];
    if constexpr (elem<E>::is_cplx) {
      if (wz != 0 || cxy != 1 || sxy != 0) {
        R c = cxy, s = sxy;
        if (wz != 0) {
          R cz, szn;
          bloch_factor<E>(A.kl, wx, wy, wz, cz, szn);
          c = cz;
          s = szn;
        }
        v = rot(v, c, s);
      }
    }
    if (++sz == n3) {
      sz = 0;
      ++wz;
    }
    return v;
  };

  E q[2 * NO + 1];
#pragma unroll
  for (int d = 0; d < 2 * NO; ++d) q[d] = load_next();

  // software pipeline: the column value and halo cells of plane z+1 are loaded while
  // plane z is computed (their latency is hidden behind one plane of work)
  const E* __restrict__ pz = xc + plane_sz * zb;
  E qn = load_next();
  E hn[HM];
#pragma unroll
  for (int u = 0; u < HM; ++u) {
    hn[u] = zero<E>();
    if (h_lds[u] >= 0 && zb < ze) hn[u] = pz[h_off[u]];
  }
  int64_t g = col + plane_sz * zb;
  const R* __restrict__ vp = A.veff;
  const E* __restrict__ zp = A.z ? A.z + (int64_t)n * A.ldz : nullptr;
  E* __restrict__ op = A.out + (int64_t)n * A.ldo;
  int step = 0;
  for (int z = zb; z < ze; ++z, ++step, g += plane_sz) {
    q[2 * NO] = qn;
    E* __restrict__ pl = plane[step & 1];
    pl[own] = q[NO];
#pragma unroll
    for (int u = 0; u < HM; ++u) {
      if (h_lds[u] >= 0) {
        E v = hn[u];
        if constexpr (elem<E>::is_cplx) v = rot(v, h_c[u], h_s[u]);
        pl[h_lds[u]] = v;
      }
    }
    // issue the loads of the next plane and of this plane's point data
    pz += plane_sz;
    if (z + 1 < ze) {
      qn = load_next();
#pragma unroll
      for (int u = 0; u < HM; ++u)
        if (h_lds[u] >= 0) hn[u] = pz[h_off[u]];
    }
    R v = 0;
    E zv = zero<E>();
    if (inside) {
      v = vp[g];
      if (zp) zv = nt_load(zp + g);
    }
    __syncthreads();
    if (inside) {
      E lap = scale(A.centre, q[NO]);
#pragma unroll
      for (int p = 1; p <= NO; ++p) {
        lap = fmar(lap, A.tz[p - 1], q[NO + p] + q[NO - p]);
        lap = fmar(lap, A.tx[p - 1], pl[own + p] + pl[own - p]);
        lap = fmar(lap, A.ty[p - 1], pl[own + p * PX] + pl[own - p * PX]);
      }
      E r = fmar(lap, (R)(A.va * v + A.vb), q[NO]);
      if (zp) r = fmar(r, A.zc, zv);
      nt_store(r, op + g);
    }
#pragma unroll
    for (int d = 0; d < 2 * NO; ++d) q[d] = q[d + 1];
  }
}

// Work-groups are dispatched round-robin over the 8 XCDs, each with its own L2.  The
// dispatch index is renumbered so that every XCD receives one contiguous range of the
// logical order (tiles fastest, then orbitals, then z chunks): the tiles of one
// (orbital, z chunk) then run side by side on one XCD and read each other's halo
// columns from its L2, and the orbitals that follow reuse the same V_eff planes.
__device__ __forceinline__ int64_t xcd_order(int64_t L, int64_t G) {
  const int64_t q = G >> 3, r = G & 7;
  const int64_t xcd = L & 7, slot = L >> 3;
  return xcd * q + (xcd < r ? xcd : r) + slot;
}

template <typename E, int TX, int TY, int NO>
__device__ __forceinline__ void hstep_local(const StepArgs<E>& A, int64_t local,
                                            E (&plane)[2][(TY + 2 * NO) * (TX + 2 * NO)]) {
  const int tile = (int)(local % A.tiles);
  const int64_t rest = local / A.tiles;
  const int n = (int)(rest % A.ns);
  const int zi = (int)(rest / A.ns);
  hstep_body<E, TX, TY, NO>(A, tile, n, zi, plane);
}

template <typename E, int TX, int TY, int NO>
__global__ __launch_bounds__(TX* TY) void hstep_kernel(StepArgs<E> A) {
  __shared__ E plane[2][(TY + 2 * NO) * (TX + 2 * NO)];
  hstep_local<E, TX, TY, NO>(A, xcd_order(blockIdx.x, gridDim.x), plane);
}

// Several (cell, k) problems in one launch: work-group b (in XCD order) belongs to the
// problem p with wg_off[p] <= b < wg_off[p+1]; inside it, the logical order of a
// single-problem launch.
template <typename E, int TX, int TY, int NO>
__global__ __launch_bounds__(TX* TY) void hstep_batched_kernel(const StepArgs<E>* __restrict__ probs,
                                                               const int* __restrict__ wg_off, int n_probs) {
  __shared__ E plane[2][(TY + 2 * NO) * (TX + 2 * NO)];
  const int b = (int)xcd_order(blockIdx.x, gridDim.x);
  int lo = 0, hi = n_probs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (wg_off[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const StepArgs<E> A = probs[lo];
  hstep_local<E, TX, TY, NO>(A, b - wg_off[lo], plane);
}

// Non-local scatter: y(g, n) += a * sum_{entries e at g} gamma_p chi~_p(g) alpha[p][n] over the
// nodes that carry projector support (point-major CSR).  One thread per node and
// block of NB orbitals; alpha is projector-major with the orbitals contiguous
// (leading dimension lda, a multiple of NB), so each entry reads NB coefficients
// in one vector load.
template <typename E, int NB>
__global__ __launch_bounds__(256) void nl_scatter_kernel(int n_pts, const int32_t* __restrict__ pts,
                                                         const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ ent_proj,
                                                         const E* __restrict__ ent_coef,
                                                         const E* __restrict__ alpha, int lda, int n_s,
                                                         typename elem<E>::real a, const double* a_dev,
                                                         E* __restrict__ y, int64_t ldy) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_pts) return;
  if (a_dev) a = (typename elem<E>::real)(*a_dev);
  const int nb0 = blockIdx.y * NB;
  const int64_t g = pts[i];
  const int e0 = ptr[i], ne = ptr[i + 1] - e0;
  E acc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j] = zero<E>();
  for (int u = 0; u < ne; ++u) {
    const E c = ent_coef[e0 + u];
    const E* __restrict__ ap = alpha + (int64_t)ent_proj[e0 + u] * lda + nb0;
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = fmae(acc[j], c, ap[j]);
  }
  E yv[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (nb0 + j < n_s) yv[j] = y[g + (int64_t)(nb0 + j) * ldy];
#pragma unroll
  for (int j = 0; j < NB; ++j)
    if (nb0 + j < n_s) y[g + (int64_t)(nb0 + j) * ldy] = fmar(yv[j], a, acc[j]);
}

// Non-local gather: alpha[p][n] = dV * sum_{t in supp(atom)} conj(chi~_p(t)) x(g_t, n)
// One work-group per (atom, block of NB orbitals).
template <typename E, int MAXP, int NB>
__global__ __launch_bounds__(256) void nl_gather_kernel(const E* __restrict__ x, int64_t ldx, int n_s,
                                                        const int32_t* __restrict__ sup_ptr,
                                                        const int32_t* __restrict__ sup_idx,
                                                        const int32_t* __restrict__ atom_pbeg,
                                                        const int64_t* __restrict__ proj_voff,
                                                        const E* __restrict__ pval, double dV,
                                                        E* __restrict__ alpha, int lda) {
  typedef typename elem<E>::real R;
  constexpr int NV = elem<E>::is_cplx ? 2 : 1;
  const int a = blockIdx.x;
  const int nb0 = blockIdx.y * NB;
  const int t0 = sup_ptr[a], t1 = sup_ptr[a + 1];
  const int pb = atom_pbeg[a], np = atom_pbeg[a + 1] - pb;
  E acc[MAXP][NB];
#pragma unroll
  for (int p = 0; p < MAXP; ++p)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[p][j] = zero<E>();
  int64_t voff[MAXP];
#pragma unroll
  for (int p = 0; p < MAXP; ++p) voff[p] = (p < np) ? proj_voff[pb + p] : 0;
#pragma unroll 2
  for (int t = t0 + (int)threadIdx.x; t < t1; t += blockDim.x) {
    const int64_t g = sup_idx[t];
    E chi[MAXP];
#pragma unroll
    for (int p = 0; p < MAXP; ++p) chi[p] = (p < np) ? pval[voff[p] + (t - t0)] : zero<E>();
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      if (nb0 + j < n_s) {
        E xv = x[g + (int64_t)(nb0 + j) * ldx];
#pragma unroll
        for (int p = 0; p < MAXP; ++p) acc[p][j] = fmac(acc[p][j], chi[p], xv);
      }
    }
  }
  // block reduction: wave butterflies, then across the 4 waves through LDS
  __shared__ R red[4][MAXP * NB * NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int p = 0; p < MAXP; ++p)
#pragma unroll
    for (int j = 0; j < NB; ++j) {
      const R* comp = (const R*)&acc[p][j];
#pragma unroll
      for (int c = 0; c < NV; ++c) {
        R s = wave_sum(comp[c]);
        if (lane == 0) red[wv][(p * NB + j) * NV + c] = s;
      }
    }
  __syncthreads();
  for (int i = threadIdx.x; i < MAXP * NB * NV; i += blockDim.x) {
    int pj = i / NV, c = i % NV;
    int p = pj / NB, j = pj % NB;
    if (p < np && nb0 + j < n_s) {
      R s = red[0][i] + red[1][i] + red[2][i] + red[3][i];
      ((R*)&alpha[(int64_t)(pb + p) * lda + nb0 + j])[c] = (R)(dV * (double)s);
    }
  }
}

// projections are stored [projector][orbital] with the orbital count padded to a multiple of 8
static inline int alpha_ld(int32_t n_s) { return ((n_s + 7) / 8) * 8; }

size_t alpha_bytes(const sparc_ham* H, int32_t n_s) {
  return (size_t)std::max(H->n_proj, 1) * (size_t)alpha_ld(n_s) * elem_bytes(H->dtype);
}

template <typename E>
static int nl_project_t(sparc_ham* H, const void* x, int64_t ldx, int32_t n_s, void* alpha) {
  if (H->n_proj == 0) return SPARC_OK;
  hipStream_t st = H->ctx->stream;
  constexpr int NB = elem<E>::is_cplx ? 4 : 8;
  dim3 grid(H->n_atoms_nl, (n_s + NB - 1) / NB);
  int t = timer_begin(H->ctx, "nl_gather");
  struct End { sparc_ctx* c; int t; ~End() { timer_end(c, t); } } end_{H->ctx, t};
  if (H->max_proj_per_atom <= 1)
    nl_gather_kernel<E, 1, NB><<<grid, 256, 0, st>>>((const E*)x, ldx, n_s, H->sup_ptr, H->sup_idx, H->atom_pbeg,
                                                     H->proj_voff, (const E*)H->pval, H->dV, (E*)alpha, alpha_ld(n_s));
  else if (H->max_proj_per_atom <= 4)
    nl_gather_kernel<E, 4, NB><<<grid, 256, 0, st>>>((const E*)x, ldx, n_s, H->sup_ptr, H->sup_idx, H->atom_pbeg,
                                                     H->proj_voff, (const E*)H->pval, H->dV, (E*)alpha, alpha_ld(n_s));
  else
    return fail(SPARC_EINVAL, "nl_project: more than 4 projector functions on one atom");
  return check_launch("nl_gather_kernel");
}

int nl_project(sparc_ham* H, const void* x, int64_t ldx, int32_t n_s, void* alpha) {
  switch (H->dtype) {
    case SPARC_R64: return nl_project_t<double>(H, x, ldx, n_s, alpha);
    case SPARC_R32: return nl_project_t<float>(H, x, ldx, n_s, alpha);
    case SPARC_C128: return nl_project_t<cd>(H, x, ldx, n_s, alpha);
    case SPARC_C64: return nl_project_t<cf>(H, x, ldx, n_s, alpha);
  }
  return fail(SPARC_EINVAL, "nl_project: bad dtype");
}

// ------------------------------------------------------------ launch planning
// Tile shapes (TX x TY threads).  Without autotuning the choice is the shape with
// the least idle work (tiles that divide n1, n2) weighted by its halo overhead;
// SPARC_HSTEP_TILE (an index into this list) overrides it.
struct TileShape { int tx, ty; };
static const TileShape kTiles[] = {{32, 8}, {32, 16}, {64, 4}, {64, 8}, {16, 16}, {24, 8}, {48, 8}, {32, 32}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

int heuristic_tile(int n1, int n2) {
  const char* env = getenv("SPARC_HSTEP_TILE");
  if (env) {
    int t = atoi(env);
    if (t >= 0 && t < kNumTiles) return t;
  }
  int best = 0;
  double best_cost = 1e30;
  for (int t = 0; t < kNumTiles; ++t) {
    const int tx = kTiles[t].tx, ty = kTiles[t].ty;
    if (tx * ty > 512) continue;
    const double waste = (double)((n1 + tx - 1) / tx * tx) / n1 * ((n2 + ty - 1) / ty * ty) / n2;
    const double halo = 1.0 + 12.0 * (tx + ty) / (double)(tx * ty) * 0.25;
    const double cost = waste * halo;
    if (cost < best_cost - 1e-12) { best_cost = cost; best = t; }
  }
  return best;
}

// per-problem grid bookkeeping for a tile shape; returns the number of work-groups
template <typename E>
static int64_t plan_problem(StepArgs<E>& A, int tx, int ty, int no, int n_s, int n_cu) {
  A.tiles_x = (A.n1 + tx - 1) / tx;
  const int tiles_y = (A.n2 + ty - 1) / ty;
  A.tiles = A.tiles_x * tiles_y;
  // z chunks: enough work-groups to fill the chip, at least 4 n_o planes per chunk
  const int64_t base = (int64_t)A.tiles * n_s;
  int nz = 1;
  const int64_t want = 8 * (int64_t)n_cu;
  while (base * nz < want && A.n3 / (nz * 2) >= 4 * no) nz *= 2;
  A.zchunk = (A.n3 + nz - 1) / nz;
  A.nz = (A.n3 + A.zchunk - 1) / A.zchunk;
  A.ns = n_s;
  return (int64_t)A.tiles * A.nz * n_s;
}

template <typename E, int TX, int TY, int NO>
static int launch_single_t(sparc_ctx* ctx, StepArgs<E>& A, int32_t n_s) {
  const int64_t G = plan_problem(A, TX, TY, NO, n_s, ctx->n_cu);
  if (G > (int64_t)INT32_MAX) return fail(SPARC_ESHAPE, "stencil step: too many work-groups");
  int t = timer_begin(ctx, "hstep");
  hstep_kernel<E, TX, TY, NO><<<(unsigned)G, TX * TY, 0, ctx->stream>>>(A);
  timer_end(ctx, t);
  return check_launch("hstep_kernel");
}

template <typename E, int TX, int TY, int NO>
static int launch_batched_t(sparc_ctx* ctx, const void* dprobs, const int* dwg, int n_probs, int64_t total_wg) {
  if (total_wg <= 0) return SPARC_OK;
  if (total_wg > (int64_t)INT32_MAX) return fail(SPARC_ESHAPE, "batched step: too many work-groups");
  int t = timer_begin(ctx, "hstep");
  hstep_batched_kernel<E, TX, TY, NO><<<(unsigned)total_wg, TX * TY, 0, ctx->stream>>>(
      (const StepArgs<E>*)dprobs, dwg, n_probs);
  timer_end(ctx, t);
  return check_launch("hstep_batched_kernel");
}

// run `F::template run<TX, TY>()` for tile index t
#define SPARC_TILE_SWITCH(t, CALL)        \
  switch (t) {                            \
    case 0: return CALL(32, 8);           \
    case 1: return CALL(32, 16);          \
    case 2: return CALL(64, 4);           \
    case 3: return CALL(64, 8);           \
    case 4: return CALL(16, 16);          \
    case 5: return CALL(24, 8);           \
    case 6: return CALL(48, 8);           \
    default: return CALL(32, 32);         \
  }

template <typename E, int NO>
static int single_tile(sparc_ctx* ctx, StepArgs<E>& A, int32_t n_s, int t) {
#define CALL(tx, ty) launch_single_t<E, tx, ty, NO>(ctx, A, n_s)
  SPARC_TILE_SWITCH(t, CALL)
#undef CALL
}

template <typename E>
static int single_no(sparc_ctx* ctx, StepArgs<E>& A, int32_t n_s, int no, int t) {
  switch (no) {
    case 1: return single_tile<E, 1>(ctx, A, n_s, t);
    case 2: return single_tile<E, 2>(ctx, A, n_s, t);
    case 3: return single_tile<E, 3>(ctx, A, n_s, t);
    case 4: return single_tile<E, 4>(ctx, A, n_s, t);
    case 5: return single_tile<E, 5>(ctx, A, n_s, t);
    case 6: return single_tile<E, 6>(ctx, A, n_s, t);
    case 7: return single_tile<E, 7>(ctx, A, n_s, t);
    case 8: return single_tile<E, 8>(ctx, A, n_s, t);
  }
  return fail(SPARC_EINVAL, "ham_step: n_o=%d unsupported", no);
}

template <typename E, int NO>
static int batched_tile(sparc_ctx* ctx, const void* dprobs, const int* dwg, int n_probs, int64_t total, int t) {
#define CALL(tx, ty) launch_batched_t<E, tx, ty, NO>(ctx, dprobs, dwg, n_probs, total)
  SPARC_TILE_SWITCH(t, CALL)
#undef CALL
}

// ------------------------------------------------------------ autotuner
// The first non-in-place step for a new (grid, states, type, stencil) key times every
// tile shape once (after one warm-up launch) with HIP events on the context's stream
// and keeps the fastest; later steps with that key reuse the choice.
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int, int, int>, int> g_tune_cache;

static bool tune_lookup(const std::tuple<int, int, int, int, int, int>& key, int* t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune_cache.find(key);
  if (it == g_tune_cache.end()) return false;
  *t = it->second;
  return true;
}

int tuned_tile(sparc_ham* H, int32_t n_s, int* t) {
  return tune_lookup(std::make_tuple(H->grid.n[0], H->grid.n[1], H->grid.n[2], n_s, (int)H->dtype, H->grid.n_o), t)
             ? 1 : 0;
}

template <typename E>
static int autotune(sparc_ham* H, StepArgs<E>& A, int32_t n_s, int* best) {
  sparc_ctx* ctx = H->ctx;
  hipEvent_t e0, e1;
  SPARC_HIP(hipEventCreate(&e0));
  SPARC_HIP(hipEventCreate(&e1));
  const bool timing = ctx->timing;
  ctx->timing = false;
  float best_ms = 1e30f;
  *best = heuristic_tile(A.n1, A.n2);
  int rc = SPARC_OK;
  for (int t = 0; t < kNumTiles && rc == SPARC_OK; ++t) {
    if (kTiles[t].tx * kTiles[t].ty > 1024) continue;
    StepArgs<E> B = A;
    rc = single_no<E>(ctx, B, n_s, H->grid.n_o, t);  // warm-up
    if (rc != SPARC_OK) break;
    hipEventRecord(e0, ctx->stream);
    B = A;
    rc = single_no<E>(ctx, B, n_s, H->grid.n_o, t);
    hipEventRecord(e1, ctx->stream);
    if (rc != SPARC_OK) break;
    hipEventSynchronize(e1);
    float ms = 0;
    hipEventElapsedTime(&ms, e0, e1);
    if (ms < best_ms) { best_ms = ms; *best = t; }
  }
  ctx->timing = timing;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != SPARC_OK) return rc;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[std::make_tuple(A.n1, A.n2, A.n3, n_s, (int)H->dtype, H->grid.n_o)] = *best;
  return SPARC_OK;
}

template <typename E>
static int nl_scatter_t(sparc_ham* H, const void* alpha, int32_t n_s, double a, const double* a_dev, void* out,
                        int64_t ldo) {
  typedef typename elem<E>::real R;
  if (H->n_proj == 0 || H->n_nlpts == 0) return SPARC_OK;
  constexpr int NB = 8;
  dim3 grid((unsigned)((H->n_nlpts + 255) / 256), (unsigned)((n_s + NB - 1) / NB));
  int t = timer_begin(H->ctx, "nl_scatter");
  nl_scatter_kernel<E, NB><<<grid, 256, 0, H->ctx->stream>>>(
      (int)H->n_nlpts, H->nl_pts, H->nl_ptr, H->ent_proj, (const E*)H->ent_coef, (const E*)alpha, alpha_ld(n_s), n_s,
      (R)a, a_dev, (E*)out, ldo);
  timer_end(H->ctx, t);
  return check_launch("nl_scatter_kernel");
}

int nl_scatter(sparc_ham* H, const void* alpha, int32_t n_s, double a, const double* a_dev, void* out, int64_t ldo) {
  switch (H->dtype) {
    case SPARC_R64: return nl_scatter_t<double>(H, alpha, n_s, a, a_dev, out, ldo);
    case SPARC_R32: return nl_scatter_t<float>(H, alpha, n_s, a, a_dev, out, ldo);
    case SPARC_C128: return nl_scatter_t<cd>(H, alpha, n_s, a, a_dev, out, ldo);
    case SPARC_C64: return nl_scatter_t<cf>(H, alpha, n_s, a, a_dev, out, ldo);
  }
  return fail(SPARC_EINVAL, "nl_scatter: bad dtype");
}

template <typename E>
static int ham_step_t(sparc_ham* H, const void* x, int64_t ldx, const void* z, int64_t ldz, void* out, int64_t ldo,
                      int32_t n_s, double a, double b, double c, const void* alpha, int flags) {
  typedef typename elem<E>::real R;
  StepArgs<E> A;
  A.n1 = H->grid.n[0];
  A.n2 = H->grid.n[1];
  A.n3 = H->grid.n[2];
  A.ldx = ldx;
  A.ldz = ldz;
  A.ldo = ldo;
  A.x = (const E*)x;
  A.z = (const E*)z;
  A.out = (E*)out;
  if constexpr (sizeof(R) == 8) A.veff = (const R*)H->veff;
  else A.veff = (const R*)H->veff32;
  A.centre = (R)(a * H->centre);
  for (int p = 0; p < 8; ++p) {
    A.tx[p] = (R)(a * H->tap[0][p]);
    A.ty[p] = (R)(a * H->tap[1][p]);
    A.tz[p] = (R)(a * H->tap[2][p]);
  }
  A.va = (flags & STEP_NO_VEFF) ? (R)0 : (R)a;
  A.vb = (R)b;
  A.zc = (R)c;
  for (int s = 0; s < 3; ++s) A.kl[s] = H->grid.kpt[s] * H->grid.L[s];
  int t = heuristic_tile(A.n1, A.n2);
  if (H->ctx->autotune && !tuned_tile(H, n_s, &t) && z == nullptr && out != x) SPARC_TRY(autotune(H, A, n_s, &t));
  int rc = single_no<E>(H->ctx, A, n_s, H->grid.n_o, t);
  if (rc != SPARC_OK || H->n_proj == 0 || H->n_nlpts == 0 || (flags & STEP_NO_NONLOCAL)) return rc;
  if (!alpha) return fail(SPARC_EINVAL, "ham_step: projections missing");
  return nl_scatter(H, alpha, n_s, a, nullptr, out, ldo);
}

// ------------------------------------------------------------ batched step tables
template <typename E>
static void fill_args(sparc_ham* H, const StepDesc& d, StepArgs<E>& A) {
  typedef typename elem<E>::real R;
  A.n1 = H->grid.n[0];
  A.n2 = H->grid.n[1];
  A.n3 = H->grid.n[2];
  A.ldx = d.ldx;
  A.ldz = d.ldz;
  A.ldo = d.ldo;
  A.x = (const E*)d.x;
  A.z = (const E*)d.z;
  A.out = (E*)d.out;
  if constexpr (sizeof(R) == 8) A.veff = (const R*)H->veff;
  else A.veff = (const R*)H->veff32;
  A.centre = (R)(d.a * H->centre);
  for (int p = 0; p < 8; ++p) {
    A.tx[p] = (R)(d.a * H->tap[0][p]);
    A.ty[p] = (R)(d.a * H->tap[1][p]);
    A.tz[p] = (R)(d.a * H->tap[2][p]);
  }
  A.va = (R)d.a;
  A.vb = (R)d.b;
  A.zc = (R)d.c;
  for (int s = 0; s < 3; ++s) A.kl[s] = H->grid.kpt[s] * H->grid.L[s];
}

size_t step_args_bytes(sparc_dtype dt) {
  switch (dt) {
    case SPARC_R64: return sizeof(StepArgs<double>);
    case SPARC_R32: return sizeof(StepArgs<float>);
    case SPARC_C128: return sizeof(StepArgs<cd>);
    case SPARC_C64: return sizeof(StepArgs<cf>);
  }
  return 0;
}

template <typename E>
static int64_t build_t(sparc_ham* const* H, const StepDesc* d, int n, int tile, void* table, int* wg) {
  StepArgs<E>* T = (StepArgs<E>*)table;
  int64_t total = 0;
  for (int p = 0; p < n; ++p) {
    fill_args<E>(H[p], d[p], T[p]);
    wg[p] = (int)total;
    total += plan_problem(T[p], kTiles[tile].tx, kTiles[tile].ty, H[p]->grid.n_o, d[p].n_s, H[p]->ctx->n_cu);
  }
  wg[n] = (int)total;
  return total;
}

int64_t step_table_build(sparc_ham* const* H, const StepDesc* d, int n, int tile, void* table, int* wg) {
  switch (H[0]->dtype) {
    case SPARC_R64: return build_t<double>(H, d, n, tile, table, wg);
    case SPARC_R32: return build_t<float>(H, d, n, tile, table, wg);
    case SPARC_C128: return build_t<cd>(H, d, n, tile, table, wg);
    case SPARC_C64: return build_t<cf>(H, d, n, tile, table, wg);
  }
  return -1;
}

template <typename E>
static int launch_tab_t(sparc_ctx* ctx, int no, int tile, const void* table, const int* wg, int n, int64_t total) {
  switch (no) {
    case 1: return batched_tile<E, 1>(ctx, table, wg, n, total, tile);
    case 2: return batched_tile<E, 2>(ctx, table, wg, n, total, tile);
    case 3: return batched_tile<E, 3>(ctx, table, wg, n, total, tile);
    case 4: return batched_tile<E, 4>(ctx, table, wg, n, total, tile);
    case 5: return batched_tile<E, 5>(ctx, table, wg, n, total, tile);
    case 6: return batched_tile<E, 6>(ctx, table, wg, n, total, tile);
    case 7: return batched_tile<E, 7>(ctx, table, wg, n, total, tile);
    case 8: return batched_tile<E, 8>(ctx, table, wg, n, total, tile);
  }
  return fail(SPARC_EINVAL, "batched step: n_o=%d unsupported", no);
}

int step_table_launch(sparc_ctx* ctx, sparc_dtype dt, int no, int tile, const void* dev_table, const int* dev_wg,
                      int n, int64_t total) {
  switch (dt) {
    case SPARC_R64: return launch_tab_t<double>(ctx, no, tile, dev_table, dev_wg, n, total);
    case SPARC_R32: return launch_tab_t<float>(ctx, no, tile, dev_table, dev_wg, n, total);
    case SPARC_C128: return launch_tab_t<cd>(ctx, no, tile, dev_table, dev_wg, n, total);
    case SPARC_C64: return launch_tab_t<cf>(ctx, no, tile, dev_table, dev_wg, n, total);
  }
  return fail(SPARC_EINVAL, "batched step: bad dtype");
}

int ham_step(sparc_ham* H, const void* x, int64_t ldx, const void* z, int64_t ldz, void* out, int64_t ldo,
             int32_t n_s, double a, double b, double c, const void* alpha, int flags) {
  switch (H->dtype) {
    case SPARC_R64: return ham_step_t<double>(H, x, ldx, z, ldz, out, ldo, n_s, a, b, c, alpha, flags);
    case SPARC_R32: return ham_step_t<float>(H, x, ldx, z, ldz, out, ldo, n_s, a, b, c, alpha, flags);
    case SPARC_C128: return ham_step_t<cd>(H, x, ldx, z, ldz, out, ldo, n_s, a, b, c, alpha, flags);
    case SPARC_C64: return ham_step_t<cf>(H, x, ldx, z, ldz, out, ldo, n_s, a, b, c, alpha, flags);
  }
  return fail(SPARC_EINVAL, "ham_step: bad dtype");
}

}  // namespace sparc
