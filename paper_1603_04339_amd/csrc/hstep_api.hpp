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
};

// ------------------------------------------------------------ launch planning
// Tile shapes (TX x TY threads).  Without autotuning the choice is the shape with
// the least idle work (tiles that divide n1, n2) weighted by its halo overhead;
// SPARC_HSTEP_TILE (an index into this list) overrides it.
struct TileShape { int tx, ty; };
static const TileShape kTiles[] = {{32, 8}, {32, 16}, {64, 8}, {16, 16}, {48, 8}, {32, 32}};
constexpr int kNumTiles = sizeof(kTiles) / sizeof(kTiles[0]);

// per-problem grid bookkeeping for a tile shape; returns the number of work-groups
template <typename E>
inline int64_t plan_problem(StepArgs<E>& A, int tx, int ty, int no, int n_s, int n_cu) {
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

// one stencil step launch (single problem) with stencil order no and tile shape t
template <typename E>
int hstep_single(sparc_ctx* ctx, StepArgs<E>& A, int32_t n_s, int no, int t);
// one batched stencil step launch over a device table of n problems (dir: some problem
// has a Dirichlet direction)
template <typename E>
int hstep_batched(sparc_ctx* ctx, const void* dprobs, const int* dwg, int n, int64_t total, int no, int t, int dir);

}  // namespace sparc
