// Stencil step kernels (the fused stencil + local potential + recurrence step that
// every H*X, Chebyshev recurrence step and Lanczos step runs), instantiated once per
// element type in hstep_<type>.hip.
//
// One work-group = one TX x TY column tile of one orbital and a chunk of z planes;
// the tile streams along z.  Each thread keeps the 2*NO+1 values of its own (x, y)
// columns around the current plane in registers (z-direction taps); the current
// plane, with NO-wide x and y halos, is staged in LDS (double-buffered, one barrier
// per plane) for the x and y taps.  Loads are x-fastest and coalesced; nodes outside
// the cell are fetched from their periodic image with the Bloch factor e^{i k_s L_s w},
// or are zero along a direction with Dirichlet conditions.
#pragma once
#include <algorithm>
#include <cstdlib>

#include "hstep_api.hpp"

namespace sparc {


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

// one fused non-local entry e: the atom's projector terms at its node, added into the
// plane buffer nb
// the four chi~ values of an entry (zero past the atom's own projectors) as vector loads
__device__ __forceinline__ void nl_vals(const double* p, double (&v)[4]) {
  const double2 a = *(const double2*)p, b = *(const double2*)(p + 2);
  v[0] = a.x;
  v[1] = a.y;
  v[2] = b.x;
  v[3] = b.y;
}
__device__ __forceinline__ void nl_vals(const float* p, float (&v)[4]) {
  const float4 a = *(const float4*)p;
  v[0] = a.x;
  v[1] = a.y;
  v[2] = a.z;
  v[3] = a.w;
}
__device__ __forceinline__ void nl_vals(const cd* p, cd (&v)[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const double2 a = *(const double2*)(p + i);
    v[i] = cd{a.x, a.y};
  }
}
__device__ __forceinline__ void nl_vals(const cf* p, cf (&v)[4]) {
  const float4 a = *(const float4*)p, b = *(const float4*)(p + 2);
  v[0] = cf{a.x, a.y};
  v[1] = cf{a.z, a.w};
  v[2] = cf{b.x, b.y};
  v[3] = cf{b.z, b.w};
}

template <typename E>
__device__ __forceinline__ void nl_entry(const StepArgs<E>& A, int e, const E* alds, E* nb) {
  const int k = A.nl_ent[e];
  const E* al = alds + (k >> 16) * 4;
  E v[4];
  nl_vals(A.nl_val + (int64_t)e * 4, v);
  E c = zero<E>();
#pragma unroll
  for (int p = 0; p < 4; ++p) c = fmae(c, v[p], al[p]);
  lds_add(nb + (k & 0xffff), c);
}

// One recurrence step on one (tile, orbital, z chunk): out = a(-1/2 Lap_h) x + (a V + b) x + c z.
// Each thread owns one (x, y) column of the TX x TY tile and marches through the z
// chunk with a register queue of the 2 NO + 1 planes around the current one (z
// neighbours never touch LDS); each plane of the tile plus an NO-wide x/y halo is
// staged in LDS (double-buffered, one barrier per plane).  Threads whose column lies
// past the grid edge (partial tiles) load the periodic image, with the Bloch factor,
// so the LDS plane is always complete.
template <typename E, int TX, int TY, int NO, bool DIR, bool NL>
__device__ __forceinline__ void hstep_body(const StepArgs<E>& A, int tile, int n, int zi,
                                           E (&plane)[2][(TY + 2 * NO) * (TX + 2 * NO)], char* nl_lds) {
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
  // a column past a Dirichlet face holds zeros (it is read only as a halo); DIR is
  // false for launches without Dirichlet directions, which then compile without them
  const bool own_zero = DIR && (((A.dmask & 1) && wx != 0) || ((A.dmask & 2) && wy != 0));
  const bool dz = DIR && (A.dmask & 4) != 0;
  R cxy = 1, sxy = 0;
  bloch_factor<E>(A.kl, wx, wy, 0, cxy, sxy);
  const int own = (hy + NO) * PX + hx + NO;

  // halo cells owned by this thread: LDS slot, offset inside a plane, Bloch factor
  int h_lds[HM], h_off[HM];
  bool h_dz[HM];
  R h_c[HM], h_s[HM];
#pragma unroll
  for (int u = 0; u < HM; ++u) {
    const int c = tid + u * NT;
    h_lds[u] = -1;
    h_off[u] = 0;
    h_dz[u] = false;
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
      h_dz[u] = DIR && (((A.dmask & 1) && hwx != 0) || ((A.dmask & 2) && hwy != 0));   // Dirichlet: zero
    }
  }

  // z-direction register queue q[d] = x(column, z - NO + d); the plane index of the
  // next load and its number of cell wraps are advanced without divisions.  The Bloch
  // rotation of a value from a wrapped plane is computed when the load is issued and
  // applied where the value is consumed, so that issuing a prefetch never waits for its
  // data; planes past a Dirichlet z face are read from a plane of zeros, and the
  // Dirichlet zeros in x and y are applied at the LDS writes.
  int zl = zb - NO;
  int wz = floordiv_i(zl, n3);
  int sz = zl - wz * n3;
  R qc = cxy, qs = sxy;   // rotation of the pending column value
  auto issue_next = [&]() -> E {
    // a plane past a Dirichlet face in z is read from a plane of zeros: the choice is
    // uniform over the work-group and made on the address, never on loaded data
    const E* __restrict__ src = xc + plane_sz * sz;
    if constexpr (DIR) {
      if (dz && wz != 0) src = A.zplane;
    }
    E v = src[col];
    qc = cxy;
    qs = sxy;
    if constexpr (elem<E>::is_cplx) {
      if (wz != 0) bloch_factor<E>(A.kl, wx, wy, wz, qc, qs);
    }
    if (++sz == n3) {
      sz = 0;
      ++wz;
    }
    return v;
  };

  E q[2 * NO + 1];
#pragma unroll
  for (int d = 0; d < 2 * NO; ++d) {
    E v = issue_next();
    if constexpr (elem<E>::is_cplx) v = rot(v, qc, qs);
    q[d] = v;
  }

  // software pipeline: the column value and halo cells of plane z+1 are loaded while
  // plane z is computed.  For 4-byte elements V_eff and the recurrence operand of plane
  // z+1 are prefetched as well (no load is then consumed in the iteration that issues
  // it: the vector-memory counter completes in order); for wider elements they are
  // loaded in the iteration that uses them, which keeps the register count, and so the
  // number of resident waves, of the larger register queue down.
  constexpr bool PF = sizeof(E) <= 4;
  const E* __restrict__ pz = xc + plane_sz * zb;
  E qn = issue_next();
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
  R vn = 0;
  E zn = zero<E>();
  if (PF && inside && zb < ze) {
    vn = vp[g];
    if (zp) zn = nt_load(zp + g);
  }
  // Non-local operator: the projector term of plane z + 1 is accumulated in LDS during
  // step z (one atomic add per (node, atom) entry, entries spread over the threads)
  // and added by each node's owner before its store at step z + 1.  alds holds
  // nla * gamma_P * alpha_P of this orbital for the tile's slots; tpl the entry
  // offsets of the chunk's planes.  A step's entries are loaded before its plane
  // prefetch, so waiting for them never waits for the prefetch.
  E* alds = nullptr;
  E* nlb = nullptr;
  int* tpl = nullptr;
  if constexpr (NL) {
    const int smax4 = A.nl_smax * 4;
    const int32_t* slots = A.nl_slots + (int64_t)tile * A.nl_smax;
    alds = (E*)nl_lds;
    nlb = (E*)(nl_lds + ((size_t)smax4 * sizeof(E) + 15) / 16 * 16);
    tpl = (int*)(nlb + 2 * NT);
    for (int i = tid; i < smax4; i += NT) {
      const int a = slots[i >> 2], p = i & 3;
      E v = zero<E>();
      if (a >= 0) {
        const int pb = A.atom_pbeg[a];
        if (p < A.atom_pbeg[a + 1] - pb)
          v = scale((R)(A.nla * A.gamma[pb + p]), A.alpha[(int64_t)(pb + p) * A.lda + n]);
      }
      alds[i] = v;
    }
    const int32_t* tpp = A.nl_tpp + (int64_t)tile * n3 + zb;
    for (int i = tid; i <= ze - zb; i += NT) tpl[i] = tpp[i];
    nlb[tid] = zero<E>();
    nlb[NT + tid] = zero<E>();
    __syncthreads();
  }
  if constexpr (NL)
    for (int e = tpl[0] + tid; e < tpl[1]; e += NT) nl_entry(A, e, alds, nlb);
  int step = 0;
  for (int z = zb; z < ze; ++z, ++step, g += plane_sz) {
    if constexpr (elem<E>::is_cplx) q[2 * NO] = rot(qn, qc, qs);
    else q[2 * NO] = qn;
    E* __restrict__ pl = plane[step & 1];
    if constexpr (DIR) pl[own] = own_zero ? zero<E>() : q[NO];
    else pl[own] = q[NO];
#pragma unroll
    for (int u = 0; u < HM; ++u) {
      if (h_lds[u] >= 0) {
        E v = hn[u];
        if constexpr (elem<E>::is_cplx) v = rot(v, h_c[u], h_s[u]);
        if constexpr (DIR) {
          if (h_dz[u]) v = zero<E>();
        }
        pl[h_lds[u]] = v;
      }
    }
    R v = vn;
    E zv = zn;
    // issue the loads of the next plane (and, without prefetch, this plane's point data)
    pz += plane_sz;
    if (z + 1 < ze) {
      qn = issue_next();
#pragma unroll
      for (int u = 0; u < HM; ++u)
        if (h_lds[u] >= 0) hn[u] = pz[h_off[u]];
      if (PF && inside) {
        vn = vp[g + plane_sz];
        if (zp) zn = nt_load(zp + g + plane_sz);
      }
    }
    if (!PF && inside) {
      v = vp[g];
      if (zp) zv = nt_load(zp + g);
    }
    __syncthreads();
    // projector term of this node (complete since the barrier) and the first entry of
    // plane z + 1 for this thread, applied after the store
    E nlt = zero<E>();
    int ek = -1, e0 = 0, e1 = 0;
    E ev[4];
    if constexpr (NL) {
      E* nb = nlb + (step & 1) * NT;
      nlt = nb[tid];
      nb[tid] = zero<E>();
      if (z + 1 < ze) {
        e0 = __builtin_amdgcn_readfirstlane(tpl[z + 1 - zb]);
        e1 = __builtin_amdgcn_readfirstlane(tpl[z + 2 - zb]);
        if (e0 + tid < e1) {
          ek = A.nl_ent[e0 + tid];
          nl_vals(A.nl_val + (int64_t)(e0 + tid) * 4, ev);
        }
      }
    }
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
      if constexpr (NL) r = r + nlt;
      nt_store(r, op + g);
    }
    if constexpr (NL) {
      // projector terms of plane z + 1 into the other buffer (its owners cleared it
      // before this step's barrier; they read it after the next one).  Applied after
      // the store, where the loop waits for the plane prefetch anyway.
      E* nb = nlb + ((step + 1) & 1) * NT;
      if (ek >= 0) {
        const E* al = alds + (ek >> 16) * 4;
        E c = zero<E>();
#pragma unroll
        for (int p = 0; p < 4; ++p) c = fmae(c, ev[p], al[p]);
        lds_add(nb + (ek & 0xffff), c);
      }
      for (int e = e0 + tid + NT; e < e1; e += NT) nl_entry(A, e, alds, nb);
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

template <typename E, int TX, int TY, int NO, bool DIR, bool NL>
__device__ __forceinline__ void hstep_local(const StepArgs<E>& A, int64_t local,
                                            E (&plane)[2][(TY + 2 * NO) * (TX + 2 * NO)], char* nl_lds) {
  // tiles fastest (neighbouring tiles share halo columns in L2), then orbitals, then z chunks
  const int tile = (int)(local % A.tiles);
  const int64_t rest = local / A.tiles;
  const int n = (int)(rest % A.ns);
  const int zi = (int)(rest / A.ns);
  hstep_body<E, TX, TY, NO, DIR, NL>(A, tile, n, zi, plane, nl_lds);
}

template <typename E, int TX, int TY, int NO, bool DIR, bool NL>
__global__ __launch_bounds__(TX* TY) void hstep_kernel(StepArgs<E> A) {
  __shared__ __align__(16) E plane[2][(TY + 2 * NO) * (TX + 2 * NO)];
  extern __shared__ __align__(16) char nl_lds[];
  hstep_local<E, TX, TY, NO, DIR, NL>(A, xcd_order(blockIdx.x, gridDim.x), plane, nl_lds);
}

// Several (cell, k) problems in one launch: work-group b (in XCD order) belongs to the
// problem p with wg_off[p] <= b < wg_off[p+1]; inside it, the logical order of a
// single-problem launch.
template <typename E, int TX, int TY, int NO, bool DIR, bool NL>
__global__ __launch_bounds__(TX* TY) void hstep_batched_kernel(const StepArgs<E>* __restrict__ probs,
                                                                    const int* __restrict__ wg_off, int n_probs) {
  __shared__ __align__(16) E plane[2][(TY + 2 * NO) * (TX + 2 * NO)];
  extern __shared__ __align__(16) char nl_lds[];
  const int b = (int)xcd_order(blockIdx.x, gridDim.x);
  int lo = 0, hi = n_probs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (wg_off[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const StepArgs<E> A = probs[lo];
  if (NL && !A.nl_val) {
    hstep_local<E, TX, TY, NO, DIR, false>(A, b - wg_off[lo], plane, nl_lds);
    return;
  }
  hstep_local<E, TX, TY, NO, DIR, NL>(A, b - wg_off[lo], plane, nl_lds);
}

template <typename E, int TX, int TY, int NO>
static int launch_single_t(sparc_ctx* ctx, StepArgs<E>& A, int32_t n_s) {
  const int64_t G = plan_problem(A, TX, TY, NO, n_s, ctx->n_cu);
  if (G > (int64_t)INT32_MAX) return fail(SPARC_ESHAPE, "stencil step: too many work-groups");
  const size_t lds = nl_lds_bytes(A, TX * TY);
  int t = timer_begin(ctx, "hstep");
  if (A.nl_val) {
    if (A.dmask) hstep_kernel<E, TX, TY, NO, true, true><<<(unsigned)G, TX * TY, lds, ctx->stream>>>(A);
    else hstep_kernel<E, TX, TY, NO, false, true><<<(unsigned)G, TX * TY, lds, ctx->stream>>>(A);
  } else {
    if (A.dmask) hstep_kernel<E, TX, TY, NO, true, false><<<(unsigned)G, TX * TY, 0, ctx->stream>>>(A);
    else hstep_kernel<E, TX, TY, NO, false, false><<<(unsigned)G, TX * TY, 0, ctx->stream>>>(A);
  }
  timer_end(ctx, t);
  return check_launch("hstep_kernel");
}

template <typename E, int TX, int TY, int NO>
static int launch_batched_t(sparc_ctx* ctx, const void* dprobs, const int* dwg, int n_probs, int64_t total_wg,
                            int dir, size_t nl_lds) {
  if (total_wg <= 0) return SPARC_OK;
  if (total_wg > (int64_t)INT32_MAX) return fail(SPARC_ESHAPE, "batched step: too many work-groups");
  int t = timer_begin(ctx, "hstep");
  const StepArgs<E>* P = (const StepArgs<E>*)dprobs;
  const unsigned G = (unsigned)total_wg;
  if (nl_lds) {
    if (dir) hstep_batched_kernel<E, TX, TY, NO, true, true><<<G, TX * TY, nl_lds, ctx->stream>>>(P, dwg, n_probs);
    else hstep_batched_kernel<E, TX, TY, NO, false, true><<<G, TX * TY, nl_lds, ctx->stream>>>(P, dwg, n_probs);
  } else {
    if (dir) hstep_batched_kernel<E, TX, TY, NO, true, false><<<G, TX * TY, 0, ctx->stream>>>(P, dwg, n_probs);
    else hstep_batched_kernel<E, TX, TY, NO, false, false><<<G, TX * TY, 0, ctx->stream>>>(P, dwg, n_probs);
  }
  timer_end(ctx, t);
  return check_launch("hstep_batched_kernel");
}

// launch with the tile shape kTiles[t]
#define SPARC_TILE_SWITCH(t, CALL)        \
  switch (t) {                            \
    case 0: return CALL(32, 8);           \
    case 1: return CALL(32, 16);          \
    case 2: return CALL(64, 8);           \
    case 3: return CALL(16, 16);          \
    case 4: return CALL(48, 8);           \
    case 5: return CALL(32, 32);          \
    default: return CALL(40, 8);          \
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
static int batched_tile(sparc_ctx* ctx, const void* dprobs, const int* dwg, int n_probs, int64_t total, int t,
                        int dir, size_t nl_lds) {
#define CALL(tx, ty) launch_batched_t<E, tx, ty, NO>(ctx, dprobs, dwg, n_probs, total, dir, nl_lds)
  SPARC_TILE_SWITCH(t, CALL)
#undef CALL
}

template <typename E>
int hstep_single(sparc_ctx* ctx, StepArgs<E>& A, int32_t n_s, int no, int t) {
  return single_no<E>(ctx, A, n_s, no, t);
}

template <typename E>
int hstep_batched(sparc_ctx* ctx, const void* dprobs, const int* dwg, int n, int64_t total, int no, int t, int dir,
                  size_t nl_lds) {
  switch (no) {
    case 1: return batched_tile<E, 1>(ctx, dprobs, dwg, n, total, t, dir, nl_lds);
    case 2: return batched_tile<E, 2>(ctx, dprobs, dwg, n, total, t, dir, nl_lds);
    case 3: return batched_tile<E, 3>(ctx, dprobs, dwg, n, total, t, dir, nl_lds);
    case 4: return batched_tile<E, 4>(ctx, dprobs, dwg, n, total, t, dir, nl_lds);
    case 5: return batched_tile<E, 5>(ctx, dprobs, dwg, n, total, t, dir, nl_lds);
    case 6: return batched_tile<E, 6>(ctx, dprobs, dwg, n, total, t, dir, nl_lds);
    case 7: return batched_tile<E, 7>(ctx, dprobs, dwg, n, total, t, dir, nl_lds);
    case 8: return batched_tile<E, 8>(ctx, dprobs, dwg, n, total, t, dir, nl_lds);
  }
  return fail(SPARC_EINVAL, "batched step: n_o=%d unsupported", no);
}

}  // namespace sparc
