// Stencil step kernels: shared declarations (argument block, tile shapes, launch
// planning) between the launch code and the per-element-type kernel instances.
#pragma once
#include <cstdlib>

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
  int dmask;       // bit s: zero Dirichlet conditions along direction s
  const E* zplane; // one plane of zeros (read for planes past a Dirichlet z face)
  // Non-local operator applied inside the step (nl_val != nullptr): at every stored
  // node with projector support, out += nla * sum_P gamma_P chi~_P(g) alpha_P(x), from
  // the entry list of each (tile, plane), one entry per (node, atom)
  const int32_t* nl_tpp;    // [tiles * n3 + 1] first entry of (tile, plane)
  const int32_t* nl_ent;    // node | slot << 16
  const E* nl_val;          // [entry * 4 + p] chi~ of the slot's projector p at the node (0 past its own)
  const int32_t* nl_slots;  // [tiles * nl_smax] atoms meeting each column tile (-1: none)
  int nl_smax;              // slots per tile
  const int32_t* atom_pbeg; // first projector of each projector-carrying atom
  const R* gamma;           // [projectors] gamma_P
  const E* alpha;           // projections of x: alpha[P * lda + orbital] (dV included)
  int lda;
  R nla;                    // scale of the projector term (the step's a)
};

// dynamic LDS bytes of a fused step launch (after plan_problem): the tile's scaled
// projections of the work-group's orbital, two planes of projector terms (the next
// plane's are accumulated while the current one is computed) and the entry offsets of
// the chunk's planes
template <typename E>
inline size_t nl_lds_bytes(const StepArgs<E>& A, int threads) {
  if (!A.nl_val) return 0;
  const size_t rows = ((size_t)A.nl_smax * 4 * sizeof(E) + 15) / 16 * 16;
  return rows + 2 * (size_t)threads * sizeof(E) + ((size_t)A.zchunk + 1) * 4;
}

// ------------------------------------------------------------ launch planning
// Tile shapes (TX x TY threads).  Without autotuning the choice is the shape with
// the least idle work (tiles that divide n1, n2) weighted by its halo overhead;
// SPARC_HSTEP_TILE (an index into this list) overrides it.
struct TileShape { int tx, ty; };
static const TileShape kTiles[] = {{32, 8}, {32, 16}, {64, 8}, {16, 16}, {48, 8}, {32, 32}, {40, 8}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

// z chunks of one orbital's column tile: enough work-groups to fill the chip, at least
// 4 n_o planes per chunk (2 n_o when the step's three blocks, `step_bytes`, stay
// cache-resident, so that the 2 n_o extra planes each chunk reads come from the cache);
// returns the chunk length (the chunk count is ceil(n3 / length))
inline int plan_zchunk(int n3, int64_t tiles, int no, int n_s, int n_cu, double step_bytes = 1e300) {
  const int64_t base = tiles * n_s;
  int nz = 1;
  const int64_t want = 8 * (int64_t)n_cu;
  const int min_len = step_bytes <= 128e6 ? 2 * no : 4 * no;
  while (base * nz < want && n3 / (nz * 2) >= min_len) nz *= 2;
  return (n3 + nz - 1) / nz;
}

// per-problem grid bookkeeping for a tile shape; returns the number of work-groups
template <typename E>
inline int64_t plan_problem(StepArgs<E>& A, int tx, int ty, int no, int n_s, int n_cu) {
  A.tiles_x = (A.n1 + tx - 1) / tx;
  const int tiles_y = (A.n2 + ty - 1) / ty;
  A.tiles = A.tiles_x * tiles_y;
  A.zchunk = plan_zchunk(A.n3, A.tiles, no, n_s, n_cu, 3.0 * A.n1 * A.n2 * A.n3 * n_s * sizeof(E));
  A.nz = (A.n3 + A.zchunk - 1) / A.zchunk;
  A.ns = n_s;
  return (int64_t)A.tiles * A.nz * n_s;
}

// one stencil step launch (single problem) with stencil order no and tile shape t
template <typename E>
int hstep_single(sparc_ctx* ctx, StepArgs<E>& A, int32_t n_s, int no, int t);
// one batched stencil step launch over a device table of n problems (dir: some problem
// has a Dirichlet direction; nl_lds: dynamic LDS bytes of the widest fused problem, 0
// when no problem applies its projectors inside the step)
template <typename E>
int hstep_batched(sparc_ctx* ctx, const void* dprobs, const int* dwg, int n, int64_t total, int no, int t, int dir,
                  size_t nl_lds);

}  // namespace sparc
