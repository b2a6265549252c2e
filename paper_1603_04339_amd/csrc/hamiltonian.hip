// Application of the finite-difference Hamiltonian to a block of orbitals: the
// non-local gather (projections of the orbitals onto the Kleinman-Bylander
// projectors) and scatter kernels, the stencil-step launch logic (tile choice,
// autotuner, batched step tables) and the H*X entry point.  The stencil step
// kernels themselves are in hstep_impl.hpp.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "hstep_api.hpp"

namespace sparc {

// Non-local scatter: y(g, n) += a * sum_{entries e at g} gamma_p chi~_p(g) alpha[p][n] over the
// nodes that carry projector support (point-major CSR).  One thread per node and
// block of NB orbitals; alpha is projector-major with the orbitals contiguous
// (leading dimension lda, a multiple of NB), so each entry reads NB coefficients
// in one vector load.
template <typename E, int NB>
__device__ __forceinline__ void nl_scatter_body(int i, int nb0, int n_pts, const int32_t* __restrict__ pts,
                                                const int32_t* __restrict__ ptr,
                                                const int32_t* __restrict__ ent_proj,
                                                const E* __restrict__ ent_coef, const E* __restrict__ alpha,
                                                int lda, int n_s, typename elem<E>::real a, E* __restrict__ y,
                                                int64_t ldy) {
  if (i >= n_pts) return;
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

template <typename E, int NB>
__global__ __launch_bounds__(256) void nl_scatter_kernel(int n_pts, const int32_t* __restrict__ pts,
                                                         const int32_t* __restrict__ ptr,
                                                         const int32_t* __restrict__ ent_proj,
                                                         const E* __restrict__ ent_coef,
                                                         const E* __restrict__ alpha, int lda, int n_s,
                                                         typename elem<E>::real a, const double* a_dev,
                                                         E* __restrict__ y, int64_t ldy) {
  // orbital groups fastest in the grid: consecutive work-groups share the same nodes'
  // entry lists (from L2)
  if (a_dev) a = (typename elem<E>::real)(*a_dev);
  nl_scatter_body<E, NB>(blockIdx.y * blockDim.x + threadIdx.x, blockIdx.x * NB, n_pts, pts, ptr, ent_proj, ent_coef,
                         alpha, lda, n_s, a, y, ldy);
}

// Several problems in one launch (work-group b of problem p as in nl_gather_batched_kernel;
// inside it the single-problem order, orbital blocks fastest); the scale comes from the
// device step table (a_dev[p]), so one captured launch serves every pass
template <typename E, int NB>
__global__ __launch_bounds__(256) void nl_scatter_batched_kernel(const NlBatchArgs* __restrict__ probs,
                                                                 const int* __restrict__ off, int n_probs,
                                                                 const double* __restrict__ a_dev) {
  const int b = blockIdx.x;
  int lo = 0, hi = n_probs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (off[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const NlBatchArgs& P = probs[lo];
  const int local = b - off[lo];
  const int groups = (P.n_s + NB - 1) / NB;
  nl_scatter_body<E, NB>((local / groups) * 256 + (int)threadIdx.x, (local % groups) * NB, P.n_pts, P.pts, P.ptr,
                         P.ent_proj, (const E*)P.ent_coef, (const E*)P.alpha, P.lda, P.n_s,
                         (typename elem<E>::real)a_dev[P.slot], (E*)P.y, P.ldy);
}

// Non-local gather: alpha[p][n] = dV * sum_{t in supp(atom)} conj(chi~_p(t)) x(g_t, n)
// One work-group per (atom, block of NB orbitals).
template <typename E, int MAXP, int NB>
__device__ __forceinline__ void nl_gather_body(int a, int nb0, const E* __restrict__ x, int64_t ldx, int n_s,
                                               const int32_t* __restrict__ sup_ptr,
                                               const int32_t* __restrict__ sup_idx,
                                               const int32_t* __restrict__ atom_pbeg,
                                               const int64_t* __restrict__ proj_voff, const E* __restrict__ pval,
                                               double dV, E* __restrict__ alpha, int lda) {
  typedef typename elem<E>::real R;
  constexpr int NV = elem<E>::is_cplx ? 2 : 1;
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

template <typename E, int MAXP, int NB>
__global__ __launch_bounds__(256) void nl_gather_kernel(const E* __restrict__ x, int64_t ldx, int n_s,
                                                        const int32_t* __restrict__ sup_ptr,
                                                        const int32_t* __restrict__ sup_idx,
                                                        const int32_t* __restrict__ atom_pbeg,
                                                        const int64_t* __restrict__ proj_voff,
                                                        const E* __restrict__ pval, double dV,
                                                        E* __restrict__ alpha, int lda) {
  nl_gather_body<E, MAXP, NB>(blockIdx.x, blockIdx.y * NB, x, ldx, n_s, sup_ptr, sup_idx, atom_pbeg, proj_voff, pval,
                              dV, alpha, lda);
}

// Several problems in one launch: work-group b belongs to the problem p with
// off[p] <= b < off[p+1], and inside it to (atom, orbital block) in the order of the
// single-problem grid (atoms fastest).
template <typename E, int MAXP, int NB>
__global__ __launch_bounds__(256) void nl_gather_batched_kernel(const NlBatchArgs* __restrict__ probs,
                                                                const int* __restrict__ off, int n_probs) {
  const int b = blockIdx.x;
  int lo = 0, hi = n_probs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (off[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const NlBatchArgs& P = probs[lo];
  const int local = b - off[lo];
  nl_gather_body<E, MAXP, NB>(local % P.n_atoms, (local / P.n_atoms) * NB, (const E*)P.x, P.ldx, P.n_s, P.sup_ptr,
                              P.sup_idx, P.atom_pbeg, P.proj_voff, (const E*)P.pval, P.dV, (E*)P.alpha, P.lda);
}

// projections are stored [projector][orbital] with the orbital count padded to a multiple of 16
size_t alpha_bytes(const sparc_ham* H, int32_t n_s) {
  return (size_t)std::max(H->n_proj, 1) * (size_t)alpha_ld(n_s) * elem_bytes(H->dtype);
}

template <typename E, int MAXP, int NB>
static void nl_gather_launch(sparc_ham* H, const void* x, int64_t ldx, int32_t n_s, void* alpha) {
  dim3 grid(H->n_atoms_nl, (n_s + NB - 1) / NB);
  nl_gather_kernel<E, MAXP, NB><<<grid, 256, 0, H->ctx->stream>>>(
      (const E*)x, ldx, n_s, H->sup_ptr, H->sup_idx, H->atom_pbeg, H->proj_voff, (const E*)H->pval, H->dV, (E*)alpha,
      alpha_ld(n_s));
}

// One work-group per (atom, NB orbitals): NB = 4 (measured on the c2 block: 362 us per
// launch against 385 with 8, 387 with 2 and 491 with 16), or 2 (1 complex) when 4 would
// leave fewer than two work-groups per CU (few atoms and orbitals: the SCF cells), which
// spreads each atom's sums over more CUs
template <typename E>
static int nl_project_t(sparc_ham* H, const void* x, int64_t ldx, int32_t n_s, void* alpha) {
  if (H->n_proj == 0) return SPARC_OK;
  constexpr int NBW = 4, NBN = elem<E>::is_cplx ? 1 : 2;
  const bool narrow = (int64_t)H->n_atoms_nl * ((n_s + NBW - 1) / NBW) < 2 * (int64_t)H->ctx->n_cu;
  int t = timer_begin(H->ctx, "nl_gather");
  struct End { sparc_ctx* c; int t; ~End() { timer_end(c, t); } } end_{H->ctx, t};
  if (H->max_proj_per_atom <= 1) {
    if (narrow) nl_gather_launch<E, 1, NBN>(H, x, ldx, n_s, alpha);
    else nl_gather_launch<E, 1, NBW>(H, x, ldx, n_s, alpha);
  } else if (H->max_proj_per_atom <= 4) {
    if (narrow) nl_gather_launch<E, 4, NBN>(H, x, ldx, n_s, alpha);
    else nl_gather_launch<E, 4, NBW>(H, x, ldx, n_s, alpha);
  } else {
    return fail(SPARC_EINVAL, "nl_project: more than 4 projector functions on one atom");
  }
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

// ------------------------------------------------------------ non-local scatter inside the step
// Per tile shape: the atoms whose support meets each column tile (its "slots", in atom
// order) and the entries of every (tile, plane), node-major within the plane, with the
// slot-projector index resolved.
int nl_tables_build(sparc_ham* H, const std::vector<int32_t>& sup_ptr, const std::vector<int32_t>& sup_idx,
                    const std::vector<int32_t>& nodes, const std::vector<int32_t>& ptr,
                    const std::vector<int32_t>& key, const std::vector<double>& cre,
                    const std::vector<double>& cim) {
  const int n1 = H->grid.n[0], n2 = H->grid.n[1], n3 = H->grid.n[2];
  const int na = H->n_atoms_nl;
  const int64_t n12 = (int64_t)n1 * n2;
  for (int t = 0; t < kNumTiles; ++t) {
    NlTileTable& T = H->nlt[t];
    const int tx = kTiles[t].tx, ty = kTiles[t].ty;
    const int tiles_x = (n1 + tx - 1) / tx, tiles = tiles_x * ((n2 + ty - 1) / ty);
    T.tiles = tiles;
    T.smax = 0;
    // slots: the atoms of each tile, and the slot of (tile, atom)
    std::vector<std::vector<int32_t>> tile_atoms(tiles);
    std::vector<int> stamp(tiles, -1);
    for (int a = 0; a < na; ++a)
      for (int q = sup_ptr[a]; q < sup_ptr[a + 1]; ++q) {
        const int64_t g = sup_idx[q];
        const int tl = (int)(g % n1) / tx + tiles_x * ((int)((g / n1) % n2) / ty);
        if (stamp[tl] != a) {
          stamp[tl] = a;
          tile_atoms[tl].push_back(a);
        }
      }
    int smax = 0;
    for (const auto& v : tile_atoms) smax = std::max(smax, (int)v.size());
    if (smax == 0 || smax > kNlMaxSlots) continue;  // this shape keeps the separate scatter
    auto slot_of = [&](int tl, int a) {
      const auto& v = tile_atoms[tl];
      return (int)(std::lower_bound(v.begin(), v.end(), a) - v.begin());
    };
    // entries, one per (node, atom), bucketed by (tile, plane); nodes ascend in g, so
    // within a bucket they come out in ascending tile-local node order
    const int pw = 4;  // chi~ values per entry (zero past the atom's own projectors)
    std::vector<int32_t> tpp((size_t)tiles * n3 + 1, 0);
    std::vector<int32_t> bucket(nodes.size());
    size_t n_grp = 0;
    for (size_t i = 0; i < nodes.size(); ++i) {
      const int64_t g = nodes[i];
      const int x = (int)(g % n1), y = (int)((g / n1) % n2), z = (int)(g / n12);
      bucket[i] = (x / tx + tiles_x * (y / ty)) * n3 + z;
      int groups = 0;
      for (int e = ptr[i]; e < ptr[i + 1]; ++e)
        if (e == ptr[i] || (key[e] >> 2) != (key[e - 1] >> 2)) ++groups;
      tpp[bucket[i] + 1] += groups;
      n_grp += groups;
    }
    for (size_t b = 0; b + 1 < tpp.size(); ++b) tpp[b + 1] += tpp[b];
    int maxb = 0;
    for (size_t b = 0; b + 1 < tpp.size(); ++b) maxb = std::max(maxb, tpp[b + 1] - tpp[b]);
    std::vector<int32_t> fill(tpp.begin(), tpp.end() - 1), ent(n_grp);
    std::vector<double> vre(n_grp * pw, 0.0), vim(n_grp * pw, 0.0);
    for (size_t i = 0; i < nodes.size(); ++i) {
      const int64_t g = nodes[i];
      const int x = (int)(g % n1), y = (int)((g / n1) % n2);
      const int tl = bucket[i] / n3;
      const int local = (x - (tl % tiles_x) * tx) + tx * (y - (tl / tiles_x) * ty);
      int o = -1;
      for (int e = ptr[i]; e < ptr[i + 1]; ++e) {
        const int a = key[e] >> 2, p = key[e] & 3;
        if (e == ptr[i] || a != (key[e - 1] >> 2)) {
          o = fill[bucket[i]]++;
          ent[o] = local | (slot_of(tl, a) << 16);
        }
        vre[(size_t)o * pw + p] = cre[e];
        vim[(size_t)o * pw + p] = cim[e];
      }
    }
    std::vector<int32_t> slots((size_t)tiles * smax, -1);
    for (int tl = 0; tl < tiles; ++tl)
      for (size_t i = 0; i < tile_atoms[tl].size(); ++i) slots[(size_t)tl * smax + i] = tile_atoms[tl][i];
    const size_t n_val = n_grp * pw;
    std::vector<char> val;
    val.resize(n_val * elem_bytes(H->dtype));
    for (size_t e = 0; e < n_val; ++e) {
      switch (H->dtype) {
        case SPARC_R64: ((double*)val.data())[e] = vre[e]; break;
        case SPARC_R32: ((float*)val.data())[e] = (float)vre[e]; break;
        case SPARC_C128: ((cd*)val.data())[e] = cd{vre[e], vim[e]}; break;
        case SPARC_C64: ((cf*)val.data())[e] = cf{(float)vre[e], (float)vim[e]}; break;
      }
    }
    SPARC_HIP(hipMalloc((void**)&T.slots, slots.size() * 4));
    SPARC_HIP(hipMemcpy(T.slots, slots.data(), slots.size() * 4, hipMemcpyHostToDevice));
    SPARC_HIP(hipMalloc((void**)&T.tp_ptr, tpp.size() * 4));
    SPARC_HIP(hipMemcpy(T.tp_ptr, tpp.data(), tpp.size() * 4, hipMemcpyHostToDevice));
    SPARC_HIP(hipMalloc((void**)&T.tp_ent, std::max<size_t>(n_grp, 1) * 4));
    SPARC_HIP(hipMalloc(&T.tp_val, std::max<size_t>(val.size(), 16)));
    if (n_grp) {
      SPARC_HIP(hipMemcpy(T.tp_ent, ent.data(), n_grp * 4, hipMemcpyHostToDevice));
      SPARC_HIP(hipMemcpy(T.tp_val, val.data(), val.size(), hipMemcpyHostToDevice));
    }
    T.max_bucket = maxb;
    T.smax = smax;
  }
  return SPARC_OK;
}

void nl_tables_free(sparc_ham* H) {
  for (int t = 0; t < kNlTileShapes; ++t) {
    NlTileTable& T = H->nlt[t];
    for (void* p : {(void*)T.slots, (void*)T.tp_ptr, (void*)T.tp_ent, T.tp_val})
      if (p) hipFree(p);
    T = NlTileTable();
  }
}

// the plane buffers and the fused rows of tile shape t fit the work-group's LDS
static bool nl_lds_fits(const sparc_ham* H, int t) {
  const int tx = kTiles[t].tx, ty = kTiles[t].ty, no = H->grid.n_o;
  const size_t eb = elem_bytes(H->dtype);
  const size_t plane = 2 * (size_t)(tx + 2 * no) * (ty + 2 * no) * eb;
  const size_t rows = ((size_t)H->nlt[t].smax * 4 * eb + 15) / 16 * 16 + 2 * (size_t)tx * ty * eb +
                      ((size_t)H->grid.n[2] + 1) * 4;
  return plane + rows <= kNlMaxLds;
}

bool nl_step_fused(const sparc_ham* H, int t) {
  return H->nl_fused && H->n_proj > 0 && H->n_nlpts > 0 && H->nlt[t].smax > 0 && nl_lds_fits(H, t);
}

// sets the fused non-local fields of a step (tile shape t); false when the step keeps
// the separate scatter (no projectors, no tables for this shape, no projections given)
template <typename E>
static bool nl_fill(sparc_ham* H, StepArgs<E>& A, int t, double a, const void* alpha, int32_t n_s) {
  typedef typename elem<E>::real R;
  A.nl_val = nullptr;
  if (!alpha || !nl_step_fused(H, t)) return false;
  const NlTileTable& T = H->nlt[t];
  A.nl_tpp = T.tp_ptr;
  A.nl_ent = T.tp_ent;
  A.nl_val = (const E*)T.tp_val;
  A.nl_slots = T.slots;
  A.nl_smax = T.smax;
  A.atom_pbeg = H->atom_pbeg;
  A.gamma = (const R*)H->gamma_d;
  A.alpha = (const E*)alpha;
  A.lda = alpha_ld(n_s);
  A.nla = (R)a;
  return true;
}

template <typename E>
static constexpr int gather_nb() { return elem<E>::is_cplx ? 4 : 8; }
constexpr int kScatterNB = 16;

void nl_batch_args(const sparc_ham* H, const void* x, int64_t ldx, void* y, int64_t ldy, int n_s, void* alpha,
                   int slot, NlBatchArgs* o, int* gather_wg, int* scatter_wg) {
  o->x = x;
  o->ldx = ldx;
  o->y = y;
  o->ldy = ldy;
  o->n_s = n_s;
  o->lda = alpha_ld(n_s);
  o->n_atoms = H->n_atoms_nl;
  o->n_pts = (int)H->n_nlpts;
  o->slot = slot;
  o->sup_ptr = H->sup_ptr;
  o->sup_idx = H->sup_idx;
  o->atom_pbeg = H->atom_pbeg;
  o->proj_voff = H->proj_voff;
  o->pval = H->pval;
  o->dV = H->dV;
  o->alpha = alpha;
  o->pts = H->nl_pts;
  o->ptr = H->nl_ptr;
  o->ent_proj = H->ent_proj;
  o->ent_coef = H->ent_coef;
  const int gnb = dtype_complex(H->dtype) ? 4 : 8;
  const bool any = H->n_proj > 0 && H->n_nlpts > 0;
  *gather_wg = any ? H->n_atoms_nl * ((n_s + gnb - 1) / gnb) : 0;
  *scatter_wg = any ? (int)((H->n_nlpts + 255) / 256) * ((n_s + kScatterNB - 1) / kScatterNB) : 0;
}

template <typename E>
static int gather_batched_t(sparc_ctx* ctx, int maxp, const NlBatchArgs* tab, const int* off, int n, int64_t total) {
  if (total <= 0) return SPARC_OK;
  if (total > INT32_MAX) return fail(SPARC_ESHAPE, "batched projections: too many work-groups");
  int t = timer_begin(ctx, "nl_gather");
  if (maxp <= 1) nl_gather_batched_kernel<E, 1, gather_nb<E>()><<<(unsigned)total, 256, 0, ctx->stream>>>(tab, off, n);
  else nl_gather_batched_kernel<E, 4, gather_nb<E>()><<<(unsigned)total, 256, 0, ctx->stream>>>(tab, off, n);
  timer_end(ctx, t);
  return check_launch("nl_gather_batched_kernel");
}

int nl_gather_batched(sparc_ctx* ctx, sparc_dtype dt, int maxp, const NlBatchArgs* tab, const int* off, int n,
                      int64_t total) {
  if (maxp > 4) return fail(SPARC_EINVAL, "batched projections: more than 4 projector functions on one atom");
  switch (dt) {
    case SPARC_R64: return gather_batched_t<double>(ctx, maxp, tab, off, n, total);
    case SPARC_R32: return gather_batched_t<float>(ctx, maxp, tab, off, n, total);
    case SPARC_C128: return gather_batched_t<cd>(ctx, maxp, tab, off, n, total);
    case SPARC_C64: return gather_batched_t<cf>(ctx, maxp, tab, off, n, total);
  }
  return fail(SPARC_EINVAL, "batched projections: bad dtype");
}

template <typename E>
static int scatter_batched_t(sparc_ctx* ctx, const NlBatchArgs* tab, const int* off, int n, int64_t total,
                             const double* a_dev) {
  if (total <= 0) return SPARC_OK;
  if (total > INT32_MAX) return fail(SPARC_ESHAPE, "batched scatter: too many work-groups");
  int t = timer_begin(ctx, "nl_scatter");
  nl_scatter_batched_kernel<E, kScatterNB><<<(unsigned)total, 256, 0, ctx->stream>>>(tab, off, n, a_dev);
  timer_end(ctx, t);
  return check_launch("nl_scatter_batched_kernel");
}

int nl_scatter_batched(sparc_ctx* ctx, sparc_dtype dt, const NlBatchArgs* tab, const int* off, int n, int64_t total,
                       const double* a_dev) {
  switch (dt) {
    case SPARC_R64: return scatter_batched_t<double>(ctx, tab, off, n, total, a_dev);
    case SPARC_R32: return scatter_batched_t<float>(ctx, tab, off, n, total, a_dev);
    case SPARC_C128: return scatter_batched_t<cd>(ctx, tab, off, n, total, a_dev);
    case SPARC_C64: return scatter_batched_t<cf>(ctx, tab, off, n, total, a_dev);
  }
  return fail(SPARC_EINVAL, "batched scatter: bad dtype");
}

int heuristic_tile(int n1, int n2, size_t elem_size) {
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
    // rows shorter than 128 bytes split the tile's loads into short segments
    const double seg = (tx * elem_size < 128) ? 1.5 : 1.0;
    const double cost = waste * halo * seg;
    if (cost < best_cost - 1e-12) { best_cost = cost; best = t; }
  }
  return best;
}

// ------------------------------------------------------------ autotuner
// The first non-in-place step for a new (grid, states, type, stencil) key times every
// tile shape the way the filter runs it: recurrence steps (two blocks read, one written:
// out = a H x + b x + 0 * out) three times back to back after a warm-up, best of two
// such runs, with HIP events on the context's stream, and keeps the fastest.  x is only
// read; out (the caller's output block) is overwritten by the real launch that follows.
// Later steps with that key reuse the choice.
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

void tune_store(sparc_ham* H, int32_t n_s, int t) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[std::make_tuple(H->grid.n[0], H->grid.n[1], H->grid.n[2], n_s, (int)H->dtype, H->grid.n_o)] = t;
}

int tile_shape_count() { return kNumTiles; }
int tile_shape_threads(int t) { return (t >= 0 && t < kNumTiles) ? kTiles[t].tx * kTiles[t].ty : 0; }

constexpr int kTuneBurst = 3;  // launches timed back to back
constexpr int kTuneRuns = 2;   // best of

template <typename E>
static int autotune(sparc_ham* H, StepArgs<E>& A, int32_t n_s, int* best, double a, const void* alpha) {
  sparc_ctx* ctx = H->ctx;
  hipEvent_t e0, e1;
  SPARC_HIP(hipEventCreate(&e0));
  SPARC_HIP(hipEventCreate(&e1));
  const bool timing = ctx->timing;
  ctx->timing = false;
  float best_ms = 1e30f;
  *best = heuristic_tile(A.n1, A.n2, sizeof(E));
  int rc = SPARC_OK;
  for (int t = 0; t < kNumTiles && rc == SPARC_OK; ++t) {
    if (kTiles[t].tx * kTiles[t].ty > 1024) continue;
    StepArgs<E> B = A;
    B.z = A.out;  // the recurrence operand: read as the filter reads Y_{j-1}
    B.ldz = A.ldo;
    B.zc = 0;
    nl_fill(H, B, t, a, alpha, n_s);
    const StepArgs<E> B0 = B;
    rc = hstep_single<E>(ctx, B, n_s, H->grid.n_o, t);  // warm-up
    float t_best = 1e30f;
    for (int r = 0; r < kTuneRuns && rc == SPARC_OK; ++r) {
      hipEventRecord(e0, ctx->stream);
      for (int q = 0; q < kTuneBurst && rc == SPARC_OK; ++q) {
        B = B0;
        rc = hstep_single<E>(ctx, B, n_s, H->grid.n_o, t);
      }
      hipEventRecord(e1, ctx->stream);
      if (rc != SPARC_OK) break;
      hipEventSynchronize(e1);
      float ms = 0;
      hipEventElapsedTime(&ms, e0, e1);
      t_best = std::min(t_best, ms);
    }
    if (rc == SPARC_OK && t_best < best_ms) { best_ms = t_best; *best = t; }
  }
  ctx->timing = timing;
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != SPARC_OK) return rc;
  tune_store(H, n_s, *best);
  return SPARC_OK;
}

template <typename E, int NB>
static void nl_scatter_launch(sparc_ham* H, const void* alpha, int32_t n_s, double a, const double* a_dev, void* out,
                              int64_t ldo) {
  typedef typename elem<E>::real R;
  dim3 grid((unsigned)((n_s + NB - 1) / NB), (unsigned)((H->n_nlpts + 255) / 256));
  nl_scatter_kernel<E, NB><<<grid, 256, 0, H->ctx->stream>>>(
      (int)H->n_nlpts, H->nl_pts, H->nl_ptr, H->ent_proj, (const E*)H->ent_coef, (const E*)alpha, alpha_ld(n_s), n_s,
      (R)a, a_dev, (E*)out, ldo);
}

// 16 orbitals per thread, or 4 when that would leave fewer than four work-groups per CU
// (small cells: shorter per-thread chains of loads)
template <typename E>
static int nl_scatter_t(sparc_ham* H, const void* alpha, int32_t n_s, double a, const double* a_dev, void* out,
                        int64_t ldo) {
  if (H->n_proj == 0 || H->n_nlpts == 0) return SPARC_OK;
  if ((H->n_nlpts + 255) / 256 > 65535) return fail(SPARC_ESHAPE, "nl_scatter: too many projector nodes");
  const int64_t wide = (int64_t)((n_s + 15) / 16) * ((H->n_nlpts + 255) / 256);
  int t = timer_begin(H->ctx, "nl_scatter");
  if (wide < 4 * (int64_t)H->ctx->n_cu) nl_scatter_launch<E, 4>(H, alpha, n_s, a, a_dev, out, ldo);
  else nl_scatter_launch<E, 16>(H, alpha, n_s, a, a_dev, out, ldo);
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

// ------------------------------------------------------------ small launches
// A step whose tiled launch would not give every CU a work-group (one orbital or a few
// on a small grid: the Poisson solves of the SCF, the Lanczos steps) runs one thread per
// (node, orbital) instead, every tap read straight from memory (the operand is
// L2-resident at these sizes), with the tiled kernel's arithmetic in the same order: the
// tiled form would march a handful of work-groups through all planes one after another.
// Periodic images carry the Bloch factor e^{i k_s L_s w}; taps past a Dirichlet face are
// zero.
template <typename E>
__device__ __forceinline__ E point_tap(const StepArgs<E>& A, const E* __restrict__ xc, int ii, int jj, int kk) {
  typedef typename elem<E>::real R;
  const int wx = floordiv_i(ii, A.n1), wy = floordiv_i(jj, A.n2), wz = floordiv_i(kk, A.n3);
  if (((A.dmask & 1) && wx != 0) || ((A.dmask & 2) && wy != 0) || ((A.dmask & 4) && wz != 0)) return zero<E>();
  E v = xc[(ii - wx * A.n1) + (int64_t)A.n1 * ((jj - wy * A.n2) + (int64_t)A.n2 * (kk - wz * A.n3))];
  if constexpr (elem<E>::is_cplx) {
    const double th = A.kl[0] * wx + A.kl[1] * wy + A.kl[2] * wz;
    if (th != 0.0) {
      double sn, cs;
      sincos(th, &sn, &cs);
      v = rot(v, (R)cs, (R)sn);
    }
  }
  return v;
}

template <typename E, int NO>
__global__ __launch_bounds__(256) void hstep_point_kernel(StepArgs<E> A, int n_s) {
  typedef typename elem<E>::real R;
  const int64_t nd = (int64_t)A.n1 * A.n2 * A.n3;
  const int64_t t = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (t >= nd * n_s) return;
  const int n = (int)(t / nd);
  const int64_t g = t - (int64_t)n * nd;
  const int i = (int)(g % A.n1), j = (int)((g / A.n1) % A.n2), k = (int)(g / ((int64_t)A.n1 * A.n2));
  const E* __restrict__ xc = A.x + (int64_t)n * A.ldx;
  const E x0 = xc[g];
  E lap = scale(A.centre, x0);
#pragma unroll
  for (int p = 1; p <= NO; ++p) {
    lap = fmar(lap, A.tz[p - 1], point_tap(A, xc, i, j, k + p) + point_tap(A, xc, i, j, k - p));
    lap = fmar(lap, A.tx[p - 1], point_tap(A, xc, i + p, j, k) + point_tap(A, xc, i - p, j, k));
    lap = fmar(lap, A.ty[p - 1], point_tap(A, xc, i, j + p, k) + point_tap(A, xc, i, j - p, k));
  }
  const R v = A.veff[g];
  E r = fmar(lap, (R)(A.va * v + A.vb), x0);
  if (A.z) r = fmar(r, A.zc, A.z[(int64_t)n * A.ldz + g]);
  A.out[(int64_t)n * A.ldo + g] = r;
}

template <typename E>
static int hstep_point(sparc_ctx* ctx, const StepArgs<E>& A, int32_t n_s, int no) {
  const int64_t total = (int64_t)A.n1 * A.n2 * A.n3 * n_s;
  const int64_t blocks = (total + 255) / 256;
  if (blocks > (int64_t)INT32_MAX) return fail(SPARC_ESHAPE, "stencil step: too many nodes");
  int t = timer_begin(ctx, "hstep");
  switch (no) {
#define CASE(K) case K: hstep_point_kernel<E, K><<<(unsigned)blocks, 256, 0, ctx->stream>>>(A, n_s); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: timer_end(ctx, t); return fail(SPARC_EINVAL, "stencil step: n_o=%d unsupported", no);
  }
  timer_end(ctx, t);
  return check_launch("hstep_point_kernel");
}

// whether a single-problem step is small enough for the point form: its tiled launch
// would have fewer work-groups than the chip has CUs (a forced tile shape keeps the
// tiled form)
template <typename E>
static bool use_point_form(const sparc_ham* H, const StepArgs<E>& A, int32_t n_s, int t) {
  if (getenv("SPARC_HSTEP_TILE")) return false;
  StepArgs<E> B = A;
  const int64_t G = plan_problem(B, kTiles[t].tx, kTiles[t].ty, H->grid.n_o, n_s, H->ctx->n_cu);
  return G < H->ctx->n_cu;
}

// ------------------------------------------------------------ conjugate-gradient iteration
// g = r.r and d = w.r from the block partials of the last cg_apply_kernel, added in the
// same fixed order by every block (so every block takes the same step)
__device__ __forceinline__ void cg_sums(const CgIter& C, double& g, double& d) {
  __shared__ double red[2][4];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < C.nparts; i += 256) {
    a += C.part[i];
    b += C.part[kCgBlocks + i];
  }
  a = wave_sum_dpp(a);
  b = wave_sum_dpp(b);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  g = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  d = red[1][0] + red[1][1] + red[1][2] + red[1][3];
}

// node-wise part of iteration it: the step scalars, then p = r + beta p, s = w + beta s,
// x += alpha p, r -= alpha s
__global__ __launch_bounds__(256) void cg_update_kernel(int64_t nd, CgIter C) {
  double g, d;
  cg_sums(C, g, d);
  double beta = 0.0, alpha = g / d;
  if (C.it > 0) {
    const double* pv = C.sc + 4 * ((C.it + 1) % 2);
    beta = g / pv[0];
    alpha = g / (d - beta * g / pv[2]);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    double* cv = C.sc + 4 * (C.it % 2);
    cv[0] = g;
    cv[1] = d;
    cv[2] = alpha;
  }
  const int64_t t = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (t >= nd) return;
  const double rt = C.r[t];
  const double pn = fma(beta, C.p[t], rt);
  const double sn = fma(beta, C.s[t], C.w[t]);
  C.p[t] = pn;
  C.s[t] = sn;
  C.x[t] = fma(alpha, pn, C.x[t]);
  C.r[t] = fma(-alpha, sn, rt);
}

// r.r of the current residual into sc[8] (for the convergence test)
__global__ __launch_bounds__(256) void cg_norm_kernel(CgIter C) {
  double g, d;
  cg_sums(C, g, d);
  if (threadIdx.x == 0) C.sc[8] = g;
}

// w = A r with the point-form taps; block partials of r.r and w.r
template <int NO>
__global__ __launch_bounds__(256) void cg_apply_kernel(StepArgs<double> A, CgIter C) {
  const int64_t nd = (int64_t)A.n1 * A.n2 * A.n3;
  const double* __restrict__ r = C.r;
  double a = 0.0, b = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)256 + threadIdx.x; t < nd; t += (int64_t)gridDim.x * 256) {
    const int i = (int)(t % A.n1), j = (int)((t / A.n1) % A.n2), k = (int)(t / ((int64_t)A.n1 * A.n2));
    const double r0 = r[t];
    double lap = A.centre * r0;
#pragma unroll
    for (int q = 1; q <= NO; ++q) {
      lap = fmar(lap, A.tz[q - 1], point_tap(A, r, i, j, k + q) + point_tap(A, r, i, j, k - q));
      lap = fmar(lap, A.tx[q - 1], point_tap(A, r, i + q, j, k) + point_tap(A, r, i - q, j, k));
      lap = fmar(lap, A.ty[q - 1], point_tap(A, r, i, j + q, k) + point_tap(A, r, i, j - q, k));
    }
    const double w0 = fmar(lap, A.vb, r0);
    C.w[t] = w0;
    a = fma(r0, r0, a);
    b = fma(w0, r0, b);
  }
  __shared__ double red[2][4];
  a = wave_sum_dpp(a);
  b = wave_sum_dpp(b);
  if ((threadIdx.x & 63) == 0) {
    red[0][threadIdx.x >> 6] = a;
    red[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    C.part[blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    C.part[kCgBlocks + blockIdx.x] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

static StepArgs<double> cg_args(const sparc_ham* H, double a, double b) {
  StepArgs<double> A{};
  A.n1 = H->grid.n[0];
  A.n2 = H->grid.n[1];
  A.n3 = H->grid.n[2];
  A.centre = a * H->centre;
  for (int p = 0; p < 8; ++p) {
    A.tx[p] = a * H->tap[0][p];
    A.ty[p] = a * H->tap[1][p];
    A.tz[p] = a * H->tap[2][p];
  }
  A.vb = b;
  A.dmask = dirichlet_mask(H->grid);
  return A;
}

bool cg_point_form(sparc_ham* H) {
  if (H->dtype != SPARC_R64) return false;
  StepArgs<double> A = cg_args(H, 1.0, 0.0);
  return use_point_form<double>(H, A, 1, heuristic_tile(A.n1, A.n2, sizeof(double)));
}

int cg_blocks(const sparc_ham* H) {
  const int64_t nd = (int64_t)H->grid.n[0] * H->grid.n[1] * H->grid.n[2];
  return (int)std::max<int64_t>(1, std::min<int64_t>(kCgBlocks, (nd + 255) / 256));
}

int cg_apply(sparc_ham* H, double a, double b, const CgIter& C) {
  if (H->dtype != SPARC_R64) return fail(SPARC_EINVAL, "cg_apply: FP64 operator only");
  if (C.nparts != cg_blocks(H)) return fail(SPARC_EINVAL, "cg_apply: nparts must be cg_blocks()");
  const StepArgs<double> A = cg_args(H, a, b);
  hipStream_t st = H->ctx->stream;
  const unsigned blocks = (unsigned)C.nparts;
  switch (H->grid.n_o) {
#define CASE(K) case K: cg_apply_kernel<K><<<blocks, 256, 0, st>>>(A, C); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return fail(SPARC_EINVAL, "cg_apply: n_o=%d unsupported", H->grid.n_o);
  }
  return check_launch("cg_apply_kernel");
}

int cg_iterate(sparc_ham* H, double a, double b, const CgIter& C) {
  const int64_t nd = (int64_t)H->grid.n[0] * H->grid.n[1] * H->grid.n[2];
  if ((nd + 255) / 256 > (int64_t)INT32_MAX) return fail(SPARC_ESHAPE, "cg_iterate: grid too large");
  cg_update_kernel<<<(unsigned)((nd + 255) / 256), 256, 0, H->ctx->stream>>>(nd, C);
  SPARC_TRY(check_launch("cg_update_kernel"));
  return cg_apply(H, a, b, C);
}

int cg_residual_norm(sparc_ham* H, const CgIter& C) {
  cg_norm_kernel<<<1, 256, 0, H->ctx->stream>>>(C);
  return check_launch("cg_norm_kernel");
}

template <typename E>
static int ham_step_t(sparc_ham* H, const void* x, int64_t ldx, const void* z, int64_t ldz, void* out, int64_t ldo,
                      int32_t n_s, double a, double b, double c, const void* alpha, int flags) {
  typedef typename elem<E>::real R;
  StepArgs<E> A{};
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
  A.dmask = dirichlet_mask(H->grid);
  A.zplane = (const E*)H->zplane;
  const bool nonlocal = H->n_proj > 0 && H->n_nlpts > 0 && !(flags & STEP_NO_NONLOCAL);
  if (nonlocal && !alpha) return fail(SPARC_EINVAL, "ham_step: projections missing");
  const void* al = nonlocal ? alpha : nullptr;
  int t = heuristic_tile(A.n1, A.n2, sizeof(E));
  if (use_point_form(H, A, n_s, t)) {
    SPARC_TRY(hstep_point<E>(H->ctx, A, n_s, H->grid.n_o));
    if (nonlocal) SPARC_TRY(nl_scatter(H, alpha, n_s, a, nullptr, out, ldo));
    return SPARC_OK;
  }
  if (H->ctx->autotune && !tuned_tile(H, n_s, &t) && !(flags & STEP_NO_TUNE) && z == nullptr && out != x)
    SPARC_TRY(autotune(H, A, n_s, &t, a, al));
  const bool fused = nl_fill(H, A, t, a, al, n_s);
  SPARC_TRY(hstep_single<E>(H->ctx, A, n_s, H->grid.n_o, t));
  if (nonlocal && !fused) SPARC_TRY(nl_scatter(H, alpha, n_s, a, nullptr, out, ldo));
  return SPARC_OK;
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
  A.dmask = dirichlet_mask(H->grid);
  A.zplane = (const E*)H->zplane;
  A.nl_val = nullptr;
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

// Builds the step table of n problems.  A problem whose StepDesc carries projections
// (alpha) applies its projectors inside the step when its Hamiltonian has tables for
// the tile shape.  *nl_lds: dynamic LDS bytes of the widest fused problem.
template <typename E>
static int64_t build_t(sparc_ham* const* H, const StepDesc* d, int n, int tile, void* table, int* wg,
                       size_t* nl_lds) {
  StepArgs<E>* T = (StepArgs<E>*)table;
  int64_t total = 0;
  size_t lds = 0;
  for (int p = 0; p < n; ++p) {
    fill_args<E>(H[p], d[p], T[p]);
    wg[p] = (int)total;
    total += plan_problem(T[p], kTiles[tile].tx, kTiles[tile].ty, H[p]->grid.n_o, d[p].n_s, H[p]->ctx->n_cu);
    if (d[p].alpha) nl_fill(H[p], T[p], tile, d[p].a, d[p].alpha, d[p].n_s);
    lds = std::max(lds, nl_lds_bytes(T[p], kTiles[tile].tx * kTiles[tile].ty));
  }
  wg[n] = (int)total;
  if (nl_lds) *nl_lds = lds;
  return total;
}

int64_t step_table_build(sparc_ham* const* H, const StepDesc* d, int n, int tile, void* table, int* wg,
                         size_t* nl_lds) {
  switch (H[0]->dtype) {
    case SPARC_R64: return build_t<double>(H, d, n, tile, table, wg, nl_lds);
    case SPARC_R32: return build_t<float>(H, d, n, tile, table, wg, nl_lds);
    case SPARC_C128: return build_t<cd>(H, d, n, tile, table, wg, nl_lds);
    case SPARC_C64: return build_t<cf>(H, d, n, tile, table, wg, nl_lds);
  }
  return -1;
}

int step_table_launch(sparc_ctx* ctx, sparc_dtype dt, int no, int tile, const void* dev_table, const int* dev_wg,
                      int n, int64_t total, int dir, size_t nl_lds) {
  switch (dt) {
    case SPARC_R64: return hstep_batched<double>(ctx, dev_table, dev_wg, n, total, no, tile, dir, nl_lds);
    case SPARC_R32: return hstep_batched<float>(ctx, dev_table, dev_wg, n, total, no, tile, dir, nl_lds);
    case SPARC_C128: return hstep_batched<cd>(ctx, dev_table, dev_wg, n, total, no, tile, dir, nl_lds);
    case SPARC_C64: return hstep_batched<cf>(ctx, dev_table, dev_wg, n, total, no, tile, dir, nl_lds);
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
