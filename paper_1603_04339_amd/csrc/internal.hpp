// Internal declarations of libsparc_hip (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/sparc_hip.h"

namespace sparc {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
int fail(int status, const char* fmt, ...);

#define SPARC_HIP(call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return ::sparc::fail(SPARC_EDEVICE, "%s failed: %s (%s:%d)", #call,                \
                           hipGetErrorString(e_), __FILE__, __LINE__);                   \
  } while (0)

#define SPARC_TRY(expr)          \
  do {                           \
    int s_ = (expr);             \
    if (s_ != SPARC_OK) return s_; \
  } while (0)

// ---------------------------------------------------------------- element types
template <typename T>
struct cplx {
  T re, im;
};
typedef cplx<double> cd;
typedef cplx<float> cf;

template <typename E> struct elem;
template <> struct elem<double> { typedef double real; static constexpr bool is_cplx = false; };
template <> struct elem<float> { typedef float real; static constexpr bool is_cplx = false; };
template <> struct elem<cd> { typedef double real; static constexpr bool is_cplx = true; };
template <> struct elem<cf> { typedef float real; static constexpr bool is_cplx = true; };

inline size_t elem_bytes(sparc_dtype d) {
  switch (d) {
    case SPARC_R64: return 8;
    case SPARC_R32: return 4;
    case SPARC_C128: return 16;
    case SPARC_C64: return 8;
  }
  return 0;
}
inline bool dtype_complex(sparc_dtype d) { return d == SPARC_C128 || d == SPARC_C64; }
inline bool dtype_single(sparc_dtype d) { return d == SPARC_R32 || d == SPARC_C64; }

// ---------------------------------------------------------------- handles
}  // namespace sparc

struct sparc_ctx {
  int device;
  hipStream_t stream;
  int n_cu;
  double* scalars;  // device scratch for scalar results (64 doubles), owned by the context
  bool autotune = false;  // time the stencil tile shapes on first use of a problem shape
  // optional kernel timing: HIP events recorded around launches on `stream`
  bool timing = false;
  struct TimeRec {
    std::string name;
    hipEvent_t a, b;
  };
  std::vector<TimeRec> recs;
  std::vector<hipEvent_t> pool;
};

// bit s set: zero Dirichlet conditions along direction s
inline int dirichlet_mask(const sparc_grid& g) { return (g.bc[0] == 1 ? 1 : 0) | (g.bc[1] == 1 ? 2 : 0) | (g.bc[2] == 1 ? 4 : 0); }

// z-chunks of the local-force box per atom (partial sums reduced in a fixed order)
constexpr int kForceChunks = 8;

// Tables of the non-local scatter applied inside the stencil step: the step adds
// V_nl x to its output at the nodes with projector support, from entry lists per
// (column tile, z plane).  Limits of the fused form; beyond them a cell uses the
// separate scatter kernel.
constexpr int kNlMaxSlots = 64;       // atoms whose support meets one column tile
constexpr int kNlTileShapes = 7;      // the stencil tile shapes (kTiles)
constexpr size_t kNlMaxLds = 65536;   // LDS bytes of one fused work-group (planes + rows)

// per stencil tile shape: the atoms ("slots") whose projector support meets each
// column tile, and the entries of each (tile, plane): one per (node, atom) with the
// tile-local node index and the slot packed as node | slot << 16, and the atom's
// four chi~ values at the node (zero past the atom's own projectors)
struct NlTileTable {
  int32_t tiles = 0;          // column tiles of the shape
  int32_t smax = 0;           // slots per tile (the widest tile); 0: no tables for this shape
  int32_t max_bucket = 0;     // entries of the fullest (tile, plane)
  int32_t* slots = nullptr;   // [tiles * smax] atom index, -1 past the tile's own count
  int32_t* tp_ptr = nullptr;  // [tiles * n3 + 1] first entry of (tile, plane)
  int32_t* tp_ent = nullptr;  // [entries] node | slot << 16, ascending node within a bucket
  void* tp_val = nullptr;     // [entries * 4] chi~ (element type)
};

struct sparc_ham {
  sparc_ctx* ctx;
  sparc_grid grid;
  sparc_dtype dtype;
  int64_t n_d;
  double h[3];
  double dV;
  // kinetic stencil coefficients of -1/2 Lap_h: centre and per-direction taps p = 1..n_o
  double centre;
  double tap[3][8];
  // Bloch factors e^{i k_s L_s} per direction
  double ph_re[3], ph_im[3];
  bool gamma;
  // potentials (device)
  double* vloc;       // [n_d]
  double* veff;       // [n_d] FP64
  float* veff32;      // [n_d] FP32 copy (single-precision dtypes)
  // non-local projector table (device)
  int32_t n_atoms_nl;   // atoms carrying projectors
  int32_t n_proj;       // projector functions
  int32_t max_proj_per_atom;
  int64_t n_sup;        // support points summed over atoms
  int64_t n_ent;        // (point, projector) entries
  int32_t* sup_ptr;     // [n_atoms_nl+1] offsets into sup_idx
  int32_t* sup_idx;     // [n_sup] grid index of support points (ascending per atom)
  int32_t* atom_pbeg;   // [n_atoms_nl+1] first projector of each atom
  int64_t* proj_voff;   // [n_proj] offset of the projector's values in pval
  void* pval;           // [sum over projectors of support size] chi~ values (element type)
  void* gamma_d;        // [n_proj] gamma per projector (real of the element precision)
  int64_t n_nlpts;      // grid nodes carrying projector support
  int32_t* nl_pts;      // [n_nlpts] those nodes (ascending grid index)
  int32_t* nl_ptr;      // [n_nlpts+1] CSR: entries of each such node
  int32_t* ent_proj;    // [n_ent] projector of the entry
  void* ent_coef;       // [n_ent] gamma_p * chi~_p(g) (element type)
  // atoms (device), kept for the atomic forces
  int32_t n_atoms;
  double* atom_R;       // [3 n_atoms]
  double* atom_D;       // [n_atoms] well depths
  double* atom_W;       // [n_atoms] well widths
  double* force_part;   // [n_atoms * kForceChunks * 3] partial sums of the local force
  int32_t* nl_atom;     // [n_atoms_nl] atom index of each projector-carrying atom
  void* zplane;         // [n1 n2] zero elements (Dirichlet z only; read for planes past a face)
  double gtap[3][8];    // FD gradient weights w~_p / h_s per direction, p = 1..n_o
  bool nl_fused;        // the stencil step applies the projectors (tables built)
  NlTileTable nlt[kNlTileShapes];
};

namespace sparc {

// ---------------------------------------------------------------- launch helpers
inline int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SPARC_EDEVICE, "launch of %s failed: %s", what, hipGetErrorString(e));
  return SPARC_OK;
}

// kernel timing (setup.hip): begin returns a record index (or -1 when timing is off)
int timer_begin(sparc_ctx* c, const char* name);
void timer_end(sparc_ctx* c, int idx);
// context whose timer records the GEMM launches (set by the calls that issue them)
extern sparc_ctx* g_timer_ctx;

// Hamiltonian application kernels (hamiltonian.hip)
//   out = a*(H x) + b*x + c*z ; z may alias out (in-place recurrence), x must not.
//   Runs the stencil/potential/recurrence kernel, then the non-local scatter into out.
//   alpha: projections [n_s][n_proj] of x (already scaled by dV), from nl_project.
//   flags: STEP_NO_VEFF drops the potential term, STEP_NO_NONLOCAL the projector term
//   (both together give a * (-1/2 Lap_h x) + b x + c z, used by the Poisson solver);
//   STEP_NO_TUNE keeps the heuristic tile (or an already tuned one) where the autotuner
//   would time the shapes (it creates events and synchronises).
//   With tables for the chosen tile shape the projector term is applied inside the
//   stencil kernel; otherwise the scatter kernel runs after it.
enum { STEP_NO_VEFF = 1, STEP_NO_NONLOCAL = 2, STEP_NO_TUNE = 4 };
int ham_step(sparc_ham* H, const void* x, int64_t ldx, const void* z, int64_t ldz, void* out, int64_t ldo,
             int32_t n_s, double a, double b, double c, const void* alpha, int flags = 0);
int nl_project(sparc_ham* H, const void* x, int64_t ldx, int32_t n_s, void* alpha);
// argument checks shared by the entry points (api.hip)
int check_ham(const sparc_ham* H, const char* who);
int check_block(const sparc_ham* H, const void* X, int64_t ldx, int32_t n_s, const char* who);
// device address of this library's static scratch on `device` (noalloc.hip); called with
// the device current when a context is created
int noalloc_scratch_init(int device);
//   out += a * V_nl-scatter(alpha); a from a device scalar when a_dev != nullptr
int nl_scatter(sparc_ham* H, const void* alpha, int32_t n_s, double a, const double* a_dev, void* out, int64_t ldo);
int heuristic_tile(int n1, int n2, size_t elem_size);
// Conjugate gradients on A = a (-1/2 Lap_h) + b (FP64, one orbital) in two launches per
// iteration, for grids whose stencil step runs in point form (cg_point_form).  In the
// Chronopoulos-Gear arrangement, which needs one reduction phase per iteration: from
// g = r.r, d = w.r (w = A r) of the current residual and g, alpha of the previous
// iteration, beta = g / g_prev (0 on the first iteration) and
// alpha = g / (d - beta g / alpha_prev) (g / d on the first); then, node by node,
//   p = r + beta p,  s = w + beta s,  x += alpha p,  r -= alpha s,
// and w = A r with the block partials of the new g and d (cg_apply).  All vectors are
// updated in place (s = A p).  part: 2 * kCgBlocks doubles of block partials (nparts =
// cg_blocks() of them used); sc: two slots of four doubles (g, d, alpha, unused) written
// by iteration it into slot it % 2, and sc[8] for cg_residual_norm.  The first iteration
// needs r, w = cg_apply(r) (which leaves its partials) and p = s = 0.
constexpr int kCgBlocks = 1024;
struct CgIter {
  double* r;
  double* w;
  double* s;
  double* p;
  double* x;
  double* sc;
  double* part;
  int nparts;
  int it;
};
bool cg_point_form(sparc_ham* H);
int cg_blocks(const sparc_ham* H);
int cg_apply(sparc_ham* H, double a, double b, const CgIter& C);
int cg_iterate(sparc_ham* H, double a, double b, const CgIter& C);
int cg_residual_norm(sparc_ham* H, const CgIter& C);
// projections and scatters of several problems in one launch each (hamiltonian.hip): one
// argument block per problem in a device table, work-group offsets per problem
struct NlBatchArgs {
  const void* x;      // gather input block
  int64_t ldx;
  void* y;            // scatter output block
  int64_t ldy;
  int n_s, lda, n_atoms, n_pts, slot;  // slot: index of the problem's scatter scale
  const int32_t *sup_ptr, *sup_idx, *atom_pbeg;
  const int64_t* proj_voff;
  const void* pval;
  double dV;
  void* alpha;
  const int32_t *pts, *ptr, *ent_proj;
  const void* ent_coef;
};
//   argument block of one problem; *gather_wg / *scatter_wg: its work-groups in each launch
void nl_batch_args(const sparc_ham* H, const void* x, int64_t ldx, void* y, int64_t ldy, int n_s, void* alpha,
                   int slot, NlBatchArgs* out, int* gather_wg, int* scatter_wg);
int nl_gather_batched(sparc_ctx* ctx, sparc_dtype dt, int maxp, const NlBatchArgs* dev_tab, const int* dev_off,
                      int n, int64_t total);
int nl_scatter_batched(sparc_ctx* ctx, sparc_dtype dt, const NlBatchArgs* dev_tab, const int* dev_off, int n,
                       int64_t total, const double* a_dev);
// non-local scatter inside the stencil step (hamiltonian.hip): per tile shape tables
// from the node-major entries (nodes ascending, entries of node i in [ptr[i], ptr[i+1]),
// key 4 atom + p, chi~ as (re, im))
int nl_tables_build(sparc_ham* H, const std::vector<int32_t>& sup_ptr, const std::vector<int32_t>& sup_idx,
                    const std::vector<int32_t>& nodes, const std::vector<int32_t>& ptr,
                    const std::vector<int32_t>& key, const std::vector<double>& cre,
                    const std::vector<double>& cim);
void nl_tables_free(sparc_ham* H);
// whether the batched plan's problems apply their projectors inside the step
bool nl_step_fused(const sparc_ham* H, int tile);
// batched stencil steps over several Hamiltonians (same dtype and n_o): a host table of
// per-problem step arguments and work-group offsets is built, uploaded by the caller, and
// launched as one kernel
struct StepDesc {
  const void* x;
  int64_t ldx;
  const void* z;
  int64_t ldz;
  void* out;
  int64_t ldo;
  int n_s;
  double a, b, c;
  const void* alpha;  // projections of x (the projectors are applied inside the step), or nullptr
};
size_t step_args_bytes(sparc_dtype dt);
//   nl_lds: dynamic LDS bytes of the launch (the widest fused problem)
int64_t step_table_build(sparc_ham* const* H, const StepDesc* d, int n, int tile, void* table, int* wg,
                         size_t* nl_lds = nullptr);
int step_table_launch(sparc_ctx* ctx, sparc_dtype dt, int no, int tile, const void* dev_table, const int* dev_wg,
                      int n, int64_t total, int dir, size_t nl_lds = 0);
int tuned_tile(sparc_ham* H, int32_t n_s, int* t);
// stencil tile shapes (hstep_api.hpp): count and threads per work-group of shape t
int tile_shape_count();
int tile_shape_threads(int t);
size_t alpha_bytes(const sparc_ham* H, int32_t n_s);
// partial sums of the non-local force (forces.hip)
size_t force_nl_part_bytes(const sparc_ham* H, int32_t n_s);
// leading dimension (orbitals, padded to 16) of the projections alpha[projector][orbital]
inline int alpha_ld(int32_t n_s) { return ((n_s + 15) / 16) * 16; }

// GEMMs (gemm.hip)
//   gram:   C[n_a x n_b] (FP64 or complex FP64, column-major, ldc) = A^H B, A: N x n_a, B: N x n_b
//           in the orbital element type; split over N with a deterministic reduction.
//           herm_result: the caller knows C is Hermitian (A^H H A with H Hermitian): only
//           the upper triangle is computed and the lower one is its conjugate mirror (this
//           is automatic when A and B are the same block).
//           tune: a context whose autotune flag selects timed tile / slab choices per shape
//           (gram and rotate; nullptr or autotune off: the size heuristic).
size_t gram_work_bytes(int64_t N, int32_t n_a, int32_t n_b, sparc_dtype dt);
int gram(hipStream_t s, sparc_dtype dt, int64_t N, int32_t n_a, int32_t n_b, const void* A, int64_t lda,
         const void* B, int64_t ldb, void* C, int32_t ldc, void* work, size_t work_bytes,
         sparc_gemm_mode mode, int n_cu, bool herm_result = false, sparc_ctx* tune = nullptr);
//   rotate: Out[N x n_out] = A[N x n_in] * Q[n_in x n_out] (Q FP64 / complex FP64, column-major ldq)
//   q_upper: Q is upper triangular (entries below the diagonal are not read).
int rotate(hipStream_t s, sparc_dtype dt, int64_t N, int32_t n_in, int32_t n_out, const void* A, int64_t lda,
           const void* Q, int32_t ldq, void* Out, int64_t ldo, int q_upper = 0, sparc_ctx* tune = nullptr);
// Out = A Q with split-BF16 (x3) products from pre-split operands (FP32 / complex64
// blocks, n_in a multiple of 16): a_pieces holds N * n_in * 2 pieces of 2 bytes per
// real part (the size of one FP32 / complex64 N x n_in block), q_pieces 2 * n_in * n_out
// pieces per real part.
int rotate_split_x3(hipStream_t s, sparc_dtype dt, int64_t N, int32_t n_in, int32_t n_out, const void* A,
                    int64_t lda, const void* Q, int32_t ldq, void* Out, int64_t ldo, int q_upper, void* a_pieces,
                    void* q_pieces);

// Dense N_s x N_s FP64 linear algebra (dense.hip); complex when cplx = true.
//   scaled Cholesky: M = D S D with D = diag(M)^{1/2}; S = R^H R; T = D^{-1} R^{-1} (upper)
//   so that (A T) has orthonormal columns when M = A^H A. info (device int) = failing col+1 or 0.
//   shift: added to the unit diagonal of S before factorising (0 for plain Cholesky-QR);
//   min_rel_diag: fail when a diagonal entry of M is below this fraction of the largest.
int chol_orth(hipStream_t s, bool cplx, int32_t n, const void* M, void* T, int32_t* info_dev, void* work,
              double shift, double min_rel_diag = 0.0);
size_t chol_orth_work_bytes(int32_t n, bool cplx);
// after chol_orth(M -> T) with the same work: *out_dev (device double) = estimated
// condition number of the column-scaled M (1e300 after a failed factorisation)
int chol_cond_est(hipStream_t s, bool cplx, int32_t n, const void* M, const void* T, const int32_t* info_dev,
                  void* work, double* out_dev);
//   symmetric / Hermitian eigensolve: A (n x n, overwritten) -> ascending w, eigenvectors Z (n x n)
int heev(hipStream_t s, bool cplx, int32_t n, void* A, double* w, void* Z, void* work);
size_t heev_work_bytes(int32_t n, bool cplx);
//   small products: C = op(A) * B for n x n FP64 (or complex) matrices; opA: 0 none, 1 conj-transpose
int small_gemm(hipStream_t s, bool cplx, int32_t n, int opA, const void* A, const void* B, void* C, void* work,
               size_t work_bytes, int n_cu);

}  // namespace sparc
