/* sparc_hip.h — C ABI of libsparc_hip: the Chebyshev-filtered subspace
 * iteration (CheFSI) of the real-space finite-difference Kohn–Sham method for
 * periodic systems (Ghosh & Suryanarayana, "SPARC ... Extended systems"), on
 * one AMD MI355X (gfx950).
 *
 * Conventions shared by every entry point
 *   - Status: every int-returning call returns SPARC_OK (0) or a negative
 *     sparc_status.  Argument errors are detected on the host before anything
 *     is launched; device errors are reported by the call that sees them or by
 *     sparc_ctx_sync.  sparc_last_error() gives a message for the calling thread.
 *   - Streams: all device work of a call is enqueued on the stream of its
 *     context and is asynchronous unless the call returns host scalars (stated).
 *   - Memory: "device" pointers are HIP device memory owned by the caller; the
 *     library never frees caller memory.  Handles own only their own tables.
 *     Workspace is passed in by the caller (sizes from sparc_workspace_bytes);
 *     hot calls allocate nothing.
 *   - Grid layout (Sec. 3.1): nodes (i,j,k), 0-based, flattened x-fastest,
 *     g = i + n1*(j + n2*k); N_d = n1*n2*n3.
 *   - Orbital blocks (Sec. 3.1, dense U(k) with orbitals as columns): column-
 *     major N_d x N_s with leading dimension ld >= N_d; complex values are
 *     interleaved (re, im).  Element type by the Hamiltonian's dtype: SPARC_R64
 *     double, SPARC_R32 float (Gamma point, real), SPARC_C128 complex double,
 *     SPARC_C64 complex float (any k).
 *   - Orbitals are Euclidean-orthonormal (X^H X = I); densities carry 1/(h1h2h3).
 *   - Bloch form: the operator acts on psi = e^{ik.x}u with the periodic index
 *     map psi(i + n_s) = e^{i k_s L_s} psi(i) (Sec. 2 Kohn–Sham equations with
 *     Bloch's theorem, Sec. 3.1 periodic boundary conditions).
 */
#ifndef SPARC_HIP_H
#define SPARC_HIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  SPARC_OK = 0,
  SPARC_EINVAL = -1,   /* bad argument (null pointer, bad enum, bad count)         */
  SPARC_ESHAPE = -2,   /* inconsistent sizes (ld < N_d, n_s < 1, n_s > limits)     */
  SPARC_ENOMEM = -3,   /* workspace too small, or a handle allocation failed       */
  SPARC_ENOTSPD = -4,  /* Gram matrix not positive definite; info = failing column */
  SPARC_ENOCONV = -5,  /* iteration limit reached without convergence              */
  SPARC_EDEVICE = -6,  /* HIP runtime error                                        */
  SPARC_ENAN = -7      /* NaN or Inf detected in a result                          */
} sparc_status;

typedef enum { SPARC_R64 = 0, SPARC_R32 = 1, SPARC_C128 = 2, SPARC_C64 = 3 } sparc_dtype;

/* Precision of the N_d-long Rayleigh–Ritz contractions; the Cholesky factors,
 * the subspace eigensolve and all N_s x N_s work stay in FP64.
 * NATIVE: the contractions run on MFMA in the element type of the orbitals (FP64 or
 * FP32, FP32 accumulation for FP32).
 * BF16X3 / BF16X6 (FP32 and complex64 blocks only, else EINVAL): the Gram contractions
 * X^H X and X^H (H X) split every FP32 operand into 2 (x3) or 3 (x6) bfloat16 pieces,
 * x = x_0 + x_1 (+ x_2) with each piece the round-to-nearest bf16 of the remainder, and
 * sum the piece products x_p y_q with p + q < 2 (three products: about 16 significant
 * bits) or p + q < 3 (six products: FP32 accuracy) on bf16 MFMA with FP32 accumulation.
 * With BF16X3 and n_s a multiple of 16 the two N_d-long rotations X Q use three split
 * products too (the block is split once into the Rayleigh–Ritz workspace); otherwise
 * the rotations stay FP32 MFMA.  Other values: EINVAL. */
typedef enum {
  SPARC_GEMM_NATIVE = 0,
  SPARC_GEMM_BF16X3 = 1,
  SPARC_GEMM_BF16X6 = 2
} sparc_gemm_mode;

/* Uniform grid on an axis-aligned cuboid (Sec. 3.1): n grid points and L lengths
 * (bohr) per direction, stencil half-width n_o (12th order: 6), Bloch wavevector
 * kpt (bohr^-1), and per direction the boundary condition bc: 0 Bloch-periodic,
 * 1 zero Dirichlet (Sec. 3.1: every value at an index outside the grid is zero; the
 * cell is not repeated across that direction, so atoms have no images there and kpt
 * must be 0 in it).  Zero-initialise bc for a periodic cell. */
typedef struct {
  int32_t n[3];
  double L[3];
  int32_t n_o;
  double kpt[3];
  int32_t bc[3];
} sparc_grid;

/* Synthetic atoms (host pointers, read during sparc_ham_create only).
 * Local potential V_loc(x) = -sum_J sum_images D_J exp(-|x-R_J-L|^2/(2 w_J^2)),
 * every image within 10 w_J.  Projector channel c belongs to atom chan_atom[c],
 * has angular momentum chan_l[c] (0: one s function; 1: three real p functions
 * x, y, z), energy chan_gamma[c] (Ha) and cutoff radius chan_rc[c] (bohr):
 * chi_s = c exp(-r^2/(2 s^2)), chi_p,m = c (r_m/s) exp(-r^2/(2 s^2)) for r <= rc,
 * s = rc/4, c normalising h1h2h3 * sum over the unwrapped grid of chi^2 to 1.
 * Z: valence charge per atom (used for the atomic-superposition density and the
 * pseudocharges).  psd_rc / psd_rc_ref: cutoffs of the Coulomb-tailed local
 * pseudopotential and of its reference potential, read only by the pseudocharge
 * calls and the pseudocharge SCF (may be NULL otherwise; see sparc_pseudocharge). */
typedef struct {
  int32_t n_atoms;
  const double* R;          /* [3*n_atoms], bohr                */
  const double* vloc_depth; /* [n_atoms] D_J, Ha                */
  const double* vloc_width; /* [n_atoms] w_J, bohr              */
  int32_t n_chan;
  const int32_t* chan_atom; /* [n_chan]                         */
  const int32_t* chan_l;    /* [n_chan] 0 or 1                  */
  const double* chan_gamma; /* [n_chan]                         */
  const double* chan_rc;    /* [n_chan]                         */
  const double* Z;          /* [n_atoms]                        */
  const double* psd_rc;     /* [n_atoms] rc_J, bohr, or NULL    */
  const double* psd_rc_ref; /* [n_atoms] rc~_J, bohr, or NULL   */
} sparc_atoms;

typedef struct sparc_ctx sparc_ctx; /* device + stream                                    */
typedef struct sparc_ham sparc_ham; /* one (cell, k, dtype): weights, V_eff, projector table */

/* Context on device `device` enqueuing on `hip_stream` (a hipStream_t, or NULL
 * for the default stream).  Returns SPARC_EDEVICE if the device is missing. */
int sparc_ctx_create(int device, void* hip_stream, sparc_ctx** out);
void sparc_ctx_destroy(sparc_ctx* ctx);
/* Blocks until the context's stream is idle; returns the first pending device
 * error as SPARC_EDEVICE. */
int sparc_ctx_sync(sparc_ctx* ctx);
/* Kernel timing by HIP events recorded on the context's stream around each
 * launch of the named kernels ("hstep": the fused stencil/potential/non-local
 * step; "nl_gather": the projections).  set_timing clears earlier records;
 * kernel_time synchronises the stream and returns the summed milliseconds and
 * the number of launches recorded since. */
int sparc_ctx_set_timing(sparc_ctx* ctx, int enable);
int sparc_ctx_kernel_time(sparc_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches);
/* Message describing the last error of the calling thread (never NULL). */
const char* sparc_last_error(void);
const char* sparc_status_string(int status);

/* Builds the Hamiltonian of Sec. 2 / Sec. 3.1 for one cell at grid->kpt:
 * FD weights (Sec. 3.1, weights of the Laplacian), the local potential on the
 * grid (kept as V_loc) and the Bloch-phased projector table chi~_J(x) =
 * sum_L e^{ik.L} chi_J(x - R_J - L) (Sec. 2, non-local operator; Sec. 3.1,
 * discrete form with the trapezoidal rule).  V_eff starts equal to V_loc.
 * dtype: SPARC_R64/SPARC_R32 need kpt = 0.  Synchronous.
 * Errors: EINVAL (null, n_o outside 1..8, l outside {0,1}, R64/R32 with k != 0,
 * bc outside {0,1}, k != 0 in a Dirichlet direction),
 * ESHAPE (n outside 1..4096, N_d >= 2^31). */
int sparc_ham_create(sparc_ctx* ctx, const sparc_grid* grid, const sparc_atoms* atoms,
                     sparc_dtype dtype, sparc_ham** out);
void sparc_ham_destroy(sparc_ham* ham);
/* Sets V_eff (Sec. 2: V_eff = V_xc + phi, here V_loc + V_H + V_x) from a
 * device array of N_d doubles; copied (and rounded for FP32 dtypes). */
int sparc_ham_set_veff(sparc_ham* ham, const double* veff_dev);
/* Writes the local potential V_loc (N_d doubles) into a device array. */
int sparc_ham_get_vloc(const sparc_ham* ham, double* vloc_dev);
/* Host query: N_d, number of projector functions, total support entries. */
int sparc_ham_info(const sparc_ham* ham, int64_t* n_d, int32_t* n_proj, int64_t* n_entries);

/* Operation codes for sparc_workspace_bytes. */
enum { SPARC_OP_APPLY = 0, SPARC_OP_FILTER = 1, SPARC_OP_RR = 2, SPARC_OP_LANCZOS = 3, SPARC_OP_FORCES = 4 };
/* Bytes of device workspace an operation needs for n_s states (0 for none). */
size_t sparc_workspace_bytes(const sparc_ham* ham, int32_t n_s, int32_t op);

/* Y = H X for n_s orbitals (Sec. 2 Hamiltonian in Bloch form, discretised by
 * Sec. 3.1): Y = -1/2 Lap_h X + V_eff X + h1h2h3 sum_J gamma_J chi~_J (chi~_J^H X).
 * X, Y device, column-major, ldx, ldy >= N_d, no aliasing.  work: workspace of
 * SPARC_OP_APPLY bytes (projections).  Errors: EINVAL, ESHAPE, ENOMEM. */
int fd_hamiltonian_apply(sparc_ham* ham, const void* X, int64_t ldx, void* Y, int64_t ldy,
                         int32_t n_s, void* work, size_t work_bytes);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): Y = H X as fd_hamiltonian_apply,
 * with the projections held in a static device array of this library
 * (fd_hamiltonian_apply_noalloc_max_bytes() = 16 MiB; one copy per device, resident
 * until the process ends, its address looked up by sparc_ctx_create) instead of a
 * workspace.  Allocates nothing, creates no events and never synchronises; the stencil
 * tile is the heuristic one, or one the context's autotuner has already chosen.
 * Every call on one device shares that array: calls that overlap on one device (two
 * streams, two threads) race and must be ordered by the caller.  Errors: as
 * fd_hamiltonian_apply; ENOMEM when the projections (SPARC_OP_APPLY bytes of
 * sparc_workspace_bytes) exceed the array, EDEVICE if the array was not found. */
size_t fd_hamiltonian_apply_noalloc_max_bytes(void);
int fd_hamiltonian_apply_noalloc(sparc_ham* ham, const void* X, int64_t ldx, void* Y, int64_t ldy,
                                 int32_t n_s);

/* Chebyshev filter (Sec. 3.4, Eq. of the filter): X <- C_m((H - c)/e) X with
 * c = (lambda_max + lambda_cut)/2, e = (lambda_max - lambda_cut)/2, by the
 * three-term recurrence Y_1 = (H - c)X/e, Y_{j+1} = 2(H - c)Y_j/e - Y_{j-1}
 * (unscaled; m = degree >= 1 applications of H).  In place on X (device,
 * ld >= N_d).  work: SPARC_OP_FILTER bytes (one N_d x n_s block + projections).
 * Errors: EINVAL (degree < 1, lambda_max <= lambda_cut), ESHAPE, ENOMEM. */
int chebyshev_filter(sparc_ham* ham, void* X, int64_t ldx, int32_t n_s, int32_t degree,
                     double lambda_cut, double lambda_max, void* work, size_t work_bytes);

/* Rayleigh–Ritz step of CheFSI (Sec. 3.4: projected pencil H~ = U_f^H H U_f,
 * M~ = U_f^H U_f, generalized eigenproblem, rotation U = U_f Y).  The pencil is
 * reduced by two Cholesky-QR passes of the column-scaled block (an orthonormal
 * basis Q of span(U_f), then Q^H H Q), the N_s x N_s problem is solved in FP64
 * on the GPU (Householder tridiagonalisation, bisection, inverse iteration),
 * and X is overwritten with the rotated orbitals (Euclidean-orthonormal Ritz
 * vectors).  ritz_dev: device, n_s doubles, ascending.  mode: precision of the
 * N_d-long contractions (sparc_gemm_mode; the split-BF16 modes only with SPARC_R32 /
 * SPARC_C64 Hamiltonians).  info (host, may be NULL): failing column + 1 on
 * ENOTSPD.  work: SPARC_OP_RR bytes.  Errors: ENOTSPD (rank-deficient block),
 * EINVAL (also an unknown mode, or a split mode with an FP64 dtype), ESHAPE, ENOMEM.
 * Synchronous (reads back the Cholesky status). */
int rayleigh_ritz(sparc_ham* ham, void* X, int64_t ldx, int32_t n_s, sparc_gemm_mode mode,
                  double* ritz_dev, void* work, size_t work_bytes, int32_t* info);

/* Lanczos estimate of the extremal eigenvalues of H (Sec. 4, Lanczos for the
 * filter bounds): `steps` steps with full reorthogonalisation from the device
 * start vector v0 (N_d elements of the element type).  lmin = smallest Ritz
 * value; lmax = largest Ritz value + |beta_k s_k| (its residual bound), enlarged
 * by 1% of its magnitude.  Host outputs; synchronous.  work: SPARC_OP_LANCZOS
 * bytes for `steps` (pass steps as n_s to sparc_workspace_bytes). */
int lanczos_bounds(sparc_ham* ham, const void* v0, int32_t steps, void* work, size_t work_bytes,
                   double* lmin, double* lmax);

/* Electron density (Sec. 3.4): rho_g = (2/dV) sum_b sum_n occ_w[b*n_s+n]
 * |X_b(g,n)|^2 with occ_w = w_b g_nb (device, n_k*n_s doubles).  X: host array
 * of n_k device pointers, ldx host array; dtype of all blocks; rho_dev device,
 * n_d doubles (overwritten).  FP64 accumulation for every dtype. */
int density_from_orbitals(sparc_ctx* ctx, int32_t n_k, const void* const* X, const int64_t* ldx,
                          int32_t n_s, sparc_dtype dtype, const double* occ_w, int64_t n_d,
                          double dV, double* rho_dev);

/* Measurement: the streaming rate of the recurrence's memory pattern alone, the
 * practical HBM ceiling of the stencil step (which reads two blocks and writes one per
 * recurrence step, Sec. 3.4 Chebyshev filter).  c = 2 a - b over n doubles (device,
 * 16-byte aligned, n even; a, b read, c written), one warm-up launch then reps timed
 * launches on the context's stream; *ms_per_launch (host) gets the mean launch time.
 * Synchronous.  Bytes moved per launch: 24 n. */
int sparc_stream_triad(sparc_ctx* ctx, const double* a, const double* b, double* c, int64_t n, int32_t reps,
                       double* ms_per_launch);

/* Fermi level and occupations (Sec. 3.4 electron-count constraint; Sec. 2
 * Fermi-Dirac occupations): mu with 2 sum_b w_b sum_n g_nb = n_elec by Brent's
 * method (the paper's Fermi-level solver, Sec. 4) on the bracket
 * [min lambda - 40 kT - 1, max lambda + 40 kT + 1], to 1e-13 relative charge,
 * g = (1 - tanh((lambda - mu)/(2 kT)))/2.
 * lambda_dev: device [n_k*n_s]; wk host [n_k]; occ_w_dev (out, device, may be
 * NULL): w_b g_nb; mu (host out).  Synchronous. */
int sparc_fermi(sparc_ctx* ctx, int32_t n_k, int32_t n_s, const double* lambda_dev, const double* wk,
                double n_elec, double kT, double* occ_w_dev, double* mu);

/* ---- batched forms: several (cell, k) problems advanced together --------------------
 * A filter plan binds n_prob Hamiltonians (same context, dtype and stencil order) to
 * their orbital blocks X[p] (ld ldx[p], n_s[p] states) and filter degrees.  Each
 * recurrence step of every problem is one launch of the projections of all problems,
 * one stencil launch covering all problems and one launch of the projector scatters
 * of all problems (per-problem arguments in device tables).  With use_graph the whole sequence is captured once into a HIP graph
 * (on a private stream) and replayed by sparc_filter_plan_run; the coefficients,
 * which depend on the bounds, are uploaded to device tables before each replay.
 * Results equal those of chebyshev_filter on each problem.  work: caller-owned,
 * sparc_filter_plan_workspace_bytes bytes, kept until the plan is destroyed.
 * sparc_filter_plan_run is synchronous.  Errors: EINVAL (mixed dtypes/orders/contexts,
 * degree < 1, bad bounds), ESHAPE, ENOMEM, EDEVICE (graph capture). */
typedef struct sparc_filter_plan sparc_filter_plan;
size_t sparc_filter_plan_workspace_bytes(int32_t n_prob, sparc_ham* const* H, const int32_t* n_s,
                                         const int32_t* degree);
int sparc_filter_plan_create(sparc_ctx* ctx, int32_t n_prob, sparc_ham* const* H, void* const* X,
                             const int64_t* ldx, const int32_t* n_s, const int32_t* degree, int32_t use_graph,
                             void* work, size_t work_bytes, sparc_filter_plan** out);
int sparc_filter_plan_run(sparc_filter_plan* plan, const double* lambda_cut, const double* lambda_max);
void sparc_filter_plan_destroy(sparc_filter_plan* plan);
/* One-shot batched filter (plan without graph, run once). */
int chebyshev_filter_batched(sparc_ctx* ctx, int32_t n_prob, sparc_ham* const* H, void* const* X,
                             const int64_t* ldx, const int32_t* n_s, const int32_t* degree,
                             const double* lambda_cut, const double* lambda_max, void* work, size_t work_bytes);
/* Rayleigh–Ritz of every problem with one shared workspace of
 * sparc_rr_batched_workspace_bytes bytes; ritz_dev[p]: device, n_s[p] doubles. */
size_t sparc_rr_batched_workspace_bytes(int32_t n_prob, sparc_ham* const* H, const int32_t* n_s);
int rayleigh_ritz_batched(sparc_ctx* ctx, int32_t n_prob, sparc_ham* const* H, void* const* X,
                          const int64_t* ldx, const int32_t* n_s, sparc_gemm_mode mode,
                          double* const* ritz_dev, void* work, size_t work_bytes);
/* Stencil tile autotuning: when enabled, the first non-in-place stencil step of a new
 * (grid, n_s, dtype, n_o) shape times every tile shape once (HIP events on the
 * context's stream) and the fastest is cached for the process. */
int sparc_ctx_set_autotune(sparc_ctx* ctx, int enable);

/* Minimal self-consistent field (Sec. 2 SCF fixed point with mixing, Sec. 3.4
 * CheFSI schedule, Sec. 3.5 free energy) at the Gamma point in the reduced
 * model: V_eff = V_loc + V_H + V_x (Slater exchange), -Lap_h V_H =
 * 4 pi (rho - mean rho) solved by conjugate gradients on the FD Laplacian (warm-started
 * from the previous V_H, to a relative residual of max(poisson_tol, min(1e-4, 1e-3 x the
 * last density residual)): loose while the density is far from self-consistent,
 * poisson_tol near the fixed point),
 * density mixing (linear, or Anderson with relaxation `mix` and history
 * `mix_history`; with kerker_k0 > 0 the mixed residual f is Kerker-preconditioned,
 * f - k0^2 g with (-Lap_h + k0^2) g = f solved by conjugate gradients, which damps the
 * long-wavelength charge sloshing of the density iteration), Harris–Foulkes energy at
 * the input density, stop when
 * ||rho_out - rho_in|| / ||rho_in|| < tol.  The first step runs n_first_passes
 * CheFSI passes from X0 before forming the density.
 * electrostatics = SPARC_ELEC_PSEUDOCHARGE replaces the jellium form by the paper's
 * (Sec. 2 electrostatic reformulation, Sec. 3.2, Sec. 3.5): the pseudocharge b, E_self^h
 * and E_c^h are set up once (sparc_psd_boxes with eps_b, then sparc_pseudocharge),
 * V_eff = phi + V_x with -Lap_h phi = 4 pi (rho + b) (mean removed, phi with zero mean),
 * V_loc is not used, and the free energy is
 *   2 sum g lambda + h^3 sum [eps_x rho - V_x rho + 1/2 (b - rho) phi] - E_self^h + E_c^h
 *   + entropy.
 */
enum { SPARC_ELEC_JELLIUM = 0, SPARC_ELEC_PSEUDOCHARGE = 1 };
typedef struct {
  int32_t n_s, degree, n_first_passes, max_iter, lanczos_steps;
  int32_t mix_history;         /* 0: linear mixing; m > 0: Anderson extrapolation with m
                                  previous iterates (the SCF acceleration of Sec. 4)      */
  double kT, mix, tol, n_elec, poisson_tol;
  sparc_dtype filt;            /* SPARC_R64, or SPARC_R32 for an FP32 filter          */
  sparc_gemm_mode rr;          /* contraction precision for FP32 passes              */
  int32_t final_fp64_pass;     /* with an FP32 filter: finish with FP64 passes        */
  const double* rho_init_dev;  /* device [N_d] start density (NULL: superposition of
                                  atomic Gaussians of width w_J and charge Z_J)        */
  const double* x0_dev;        /* device [N_d*n_s] FP64 start orbitals (column-major) */
  const double* lanczos_v0_dev;/* device [N_d] FP64 Lanczos start vector              */
  int32_t electrostatics;      /* SPARC_ELEC_JELLIUM (0) or SPARC_ELEC_PSEUDOCHARGE   */
  double eps_b;                /* pseudocharge truncation tolerance (0: 1e-8)         */
  double kerker_k0;            /* Kerker wavenumber of the mixing (bohr^-1; 0: none)  */
} sparc_scf_params;

typedef struct {
  double energy, mu;
  int32_t iterations, converged;
  double* rho_dev;     /* caller-provided device [N_d]: final input density (out)   */
  double* ritz_dev;    /* caller-provided device [n_s]: final Ritz values (out)      */
  double* x_dev;       /* caller-provided device [N_d*n_s] FP64: final orbitals (out, may be NULL) */
  double* history;     /* caller-provided host [3*max_iter]: (energy, rho_err, t_s) per iteration (may be NULL) */
  double* phi_dev;     /* caller-provided device [N_d]: V_H (jellium) or phi (pseudocharges) of the final
                          input density (out, may be NULL)                                        */
} sparc_scf_result;

/* Runs the SCF; synchronous.  Periodic cells only (the jellium electrostatics have
 * no Dirichlet form): a grid with a Dirichlet direction is rejected with EINVAL.
 * Errors: ENOCONV (max_iter reached; result holds the last iterate), ENOTSPD, ENAN,
 * EINVAL, ESHAPE, ENOMEM. */
int sparc_scf_run(sparc_ctx* ctx, const sparc_grid* grid, const sparc_atoms* atoms,
                  const sparc_scf_params* params, sparc_scf_result* result);

/* Superposition of atomic densities, the SCF start density (Sec. 4): rho(x) =
 * sum_J Z_J (2 pi w_J^2)^{-3/2} exp(-|x - R_J - L|^2 / (2 w_J^2)) over the images
 * L within 10 w_J, with w_J = atoms->vloc_width[J] and Z_J = atoms->Z[J] (2 when
 * Z is NULL), renormalised to h^3 sum rho = n_elec.  rho_dev: device, N_d doubles
 * (x fastest).  Synchronous.  Errors: EINVAL, ESHAPE, ENAN (no charge), ENOMEM. */
int sparc_sad_density(sparc_ctx* ctx, const sparc_grid* grid, const sparc_atoms* atoms, double n_elec,
                      double* rho_dev);

/* ---- atomic forces ----------------------------------------------------------------
 * f_J = -dF/dR_J (Sec. 2, atomic forces), split as in Sec. 3.6 into a local and a
 * non-local component.  F_dev: device [n_atoms][3] FP64 (Ha/bohr, atoms in the order
 * of sparc_atoms); both calls ADD to it (zero it first; call the non-local part once
 * per k-point with that k-point's Hamiltonian).  Asynchronous on the context's stream.
 *
 * Local component.  The Gaussian wells are an external potential (jellium
 * electrostatics, no pseudocharges, so no overlap correction), and the component is
 * the exact derivative of the trapezoidal-rule local energy h1h2h3 sum_g rho_g V_loc(x_g):
 *   f_J,loc = h1h2h3 sum_g rho_g sum_L D_J exp(-r^2/(2 w_J^2)) (x_g - R_J - L) / w_J^2,
 * r = |x_g - R_J - L| <= 10 w_J.  rho_dev: device FP64 density [N_d] (h1h2h3 sum rho =
 * N_e).  Errors: EINVAL. */
int sparc_forces_local(sparc_ham* ham, const double* rho_dev, double* F_dev);

/* Non-local component (Sec. 3.6, discrete non-local force with Y and W; Algorithm 3),
 * the derivative moved from the projectors onto the orbitals and taken with the FD
 * gradient of Sec. 3.1 (weights w~_p, Bloch-periodic index map):
 *   f_J,nloc = -4 sum_n occ_n sum_{p of J} gamma_p Re[conj(alpha_pn) beta_pn] / h1h2h3,
 *   alpha_pn = h1h2h3 sum_g conj(chi~_p(g)) X(g,n),
 *   beta_pn  = h1h2h3 sum_g conj(chi~_p(g)) (grad_h X)(g,n),
 * i.e. the paper's -4 sum w_b g_nb gamma Re[Y W] for Euclidean-orthonormal columns.
 * X: device block (the Hamiltonian's dtype, column-major, ldx >= N_d); occ_dev: device
 * FP64 [n_s] = w_b g_nb (states with zero weight are skipped); work: SPARC_OP_FORCES
 * bytes.  Errors: EINVAL, ESHAPE, ENOMEM. */
int sparc_forces_nonlocal(sparc_ham* ham, const void* X, int64_t ldx, int32_t n_s, const double* occ_dev,
                          double* F_dev, void* work, size_t work_bytes);

/* ---- band structure and density of states ----------------------------------------
 * Band structure at the electronic ground state (Sec. 4): at every k-point the CheFSI
 * steps of Sec. 3.4 are repeated, with the potential V_eff fixed, until the lowest
 * n_bands Ritz values move by less than tol (Ha, max over the bands) between two
 * passes.  All k-points are filtered together (one batched plan, HIP graph when
 * use_graph) and Rayleigh–Ritz'd per k; filter bounds per k: lambda_max by Lanczos
 * (20 steps from the first column of X[b]), lambda_cut the midpoint of the Lanczos
 * interval for the first pass, then the largest Ritz value of the previous pass.
 * grid: the cell (its kpt is ignored); kpts: host [3*n_k] (bohr^-1); veff_dev: device
 * FP64 [N_d]; X: host array of n_k device complex128 blocks (N_d x n_s, ld = N_d): the
 * start vectors (linearly independent), overwritten by the Ritz vectors.  eig_out:
 * host [n_k*n_bands] ascending per k; passes_out: host [n_k] passes used (max_passes
 * where not converged).  Synchronous; allocates its own Hamiltonians and workspace.
 * Errors: ENOCONV (outputs hold the last pass), ENAN, ENOTSPD, EINVAL, ESHAPE, ENOMEM. */
int sparc_band_structure(sparc_ctx* ctx, const sparc_grid* grid, const sparc_atoms* atoms, const double* veff_dev,
                         int32_t n_k, const double* kpts, void* const* X, int32_t n_s, int32_t n_bands,
                         int32_t degree, int32_t max_passes, double tol, int32_t use_graph, double* eig_out,
                         int32_t* passes_out);

/* Density of states (Sec. 4): D(E) = 2 sum_b wk[b] sum_n g(E - eig[b*n_bands+n]) with g
 * the normalised Gaussian of width sigma (the broadened delta function), at n_e
 * energies.  Host arrays; host computation.  Errors: EINVAL, ESHAPE. */
int sparc_dos(int32_t n_k, int32_t n_bands, const double* eig, const double* wk, int32_t n_e, const double* energies,
              double sigma, double* dos_out);

/* ---- pseudocharge electrostatics ---------------------------------------------------
 * The paper's local electrostatics (Sec. 2, electrostatic reformulation: pseudocharges
 * b_I = -Lap V_I / (4 pi), self energy, overlap correction E_c; Sec. 3.2, Algorithm 1;
 * Appendix A).  Sign convention: electrons carry positive density rho, the pseudocharge
 * is negative (h1h2h3 sum b = -N_e), and phi, the potential energy of an electron,
 * solves -Lap_h phi = 4 pi (rho + b).
 * Local pseudopotential of atom J, valence charge Z_J = atoms->Z[J] > 0, cutoff
 * rc_J = atoms->psd_rc[J] > 0: the potential of the charge -Z 315/(64 pi rc^3)
 * (1 - r^2/rc^2)^3 (zero beyond rc),
 *   V_J(r) = -Z/r for r >= rc,  -(Z/rc)(315 - 420 s^2 + 378 s^4 - 180 s^6 + 35 s^8)/128,
 *   s = r/rc, inside.
 * Reference potential V~_J of the overlap correction: the same form with cutoff
 * rc~_J = atoms->psd_rc_ref[J] > 0.  Atoms have images across periodic directions
 * only.  All three calls are synchronous and allocate their own scratch.
 *
 * Truncation boxes (Sec. 3.2, the choice of r^b from eps_b): per atom and direction the
 * box half-width r^b_s = m_s h_s, m_s = ceil(rc/h_s) + t, with t >= 0 the smallest
 * step for which the discrete pseudocharge of all nodes x with |x_s - R_s| <= m_s h_s
 * (on the unbounded grid, i.e. all images inside the cell) sums to within eps_b Z of -Z;
 * at most 16 steps.  boxes: host int32 [n_atoms][6], (m1, m2, m3) for the pseudocharge
 * then (m1, m2, m3) for the reference charge.  Errors: EINVAL (null, a value <= 0,
 * eps_b outside (0,1), n_o outside 1..8, bc outside {0,1}), ESHAPE, ENOCONV (no box within
 * 16 steps), ENAN, ENOMEM, EDEVICE. */
int sparc_psd_boxes(sparc_ctx* ctx, const sparc_grid* grid, const sparc_atoms* atoms, double eps_b, int32_t* boxes);

/* Algorithm 1 and the discrete overlap correction (Appendix A, E_c^h), for the boxes
 * of sparc_psd_boxes (host [n_atoms][6], each 0..1024).  For every image J' of every atom
 * and every node x of its box, b_J'(x) = -(1/4pi) Lap_h V_J'(x) (the FD Laplacian of
 * Sec. 3.1 applied to V_J' evaluated in closed form at x and its stencil neighbours);
 * likewise b~_J' on the reference box, and V_c(x) = sum_J' (V~_J' - V_J')(x).
 * Outputs: device FP64 [N_d] each (x fastest) b_dev = sum b_J', bref_dev = sum b~_J',
 * vc_dev = V_c; host energies[3] = { E_self^h = 1/2 h^3 sum_J' sum_box b_J' V_J',
 * E~_self^h (the same for the reference), E_c^h = 1/2 h^3 sum (b~ + b) V_c + E_self^h -
 * E~_self^h }.  Errors: EINVAL, ESHAPE, ENAN, ENOMEM, EDEVICE. */
int sparc_pseudocharge(sparc_ctx* ctx, const sparc_grid* grid, const sparc_atoms* atoms, const int32_t* boxes,
                       double* b_dev, double* bref_dev, double* vc_dev, double* energies);

/* Local and overlap-correction components of the atomic forces with pseudocharges
 * (Sec. 3.6, discrete local force; Appendix A, discrete correction force), for every
 * atom J summed over its images J':
 *   f_J,loc = h^3 sum_J' sum_{box of J'} grad_h b_J' (phi - V_J'),
 *   f_J,c   = 1/2 h^3 sum_J' [ sum_{box~} (grad_h b~_J' (V_c - V~_J') - b~_J' grad_h V~_J')
 *             + sum_{box} (grad_h b_J' (V_c + V_J') + b_J' grad_h V_J')
 *             + sum_x grad_h (V~_J' - V_J') (b~ + b) ],
 * with grad_h the FD gradient of Sec. 3.1 and b_J' at the stencil neighbours of a box
 * node computed like inside the box.  phi_dev, b_dev, bref_dev, vc_dev: device FP64
 * [N_d] (phi for the density at hand; the rest from sparc_pseudocharge with the same
 * boxes).  Floc_dev, Fc_dev: device FP64 [n_atoms][3], ADDED to (either may be NULL).
 * Errors: EINVAL, ESHAPE, ENAN, ENOMEM, EDEVICE. */
int sparc_forces_psd(sparc_ctx* ctx, const sparc_grid* grid, const sparc_atoms* atoms, const int32_t* boxes,
                     const double* phi_dev, const double* b_dev, const double* bref_dev, const double* vc_dev,
                     double* Floc_dev, double* Fc_dev);

/* ---- learned initial density ------------------------------------------------------
 * Replaces the atomic-superposition start of the SCF (Sec. 4) by
 *   rho_0 = renorm( relu(x + d - mean(d)) * rho_bar ),  x = rho_SAD / rho_bar,
 *   d = f(x, u),  u = -V_loc (Ha),  rho_bar = n_elec / (N_d dV),
 * f = four 3x3x3 periodic convolutions with dilations 1, 2, 4, 8, channels
 * 2 -> 16 -> 32 -> 32 -> 1 and ReLU after the first three (43281 parameters, FP32).
 * Host parameter vector, layer by layer: W[c_out][c_in][kz][ky][kx] (with dilation
 * q, tap (kz, ky, kx) reads the input at offset q (kz-1, ky-1, kx-1)), then
 * b[c_out].  Network inputs are device FP32 arrays [batch][N_d][2] (x fastest,
 * channels (x, u) innermost); targets and outputs [batch][N_d].  The net owns its
 * parameters, Adam state and activations for up to max_batch cells (1..128);
 * calls on one net are not concurrent. */
typedef struct sparc_dnet sparc_dnet;
int64_t sparc_dnet_num_params(void);
/* n: grid points per direction (9..1024).  Parameters start at zero. */
int sparc_dnet_create(sparc_ctx* ctx, const int32_t* n, int32_t max_batch, sparc_dnet** out);
void sparc_dnet_destroy(sparc_dnet* net);
/* Host parameter vector in/out (sparc_dnet_num_params floats).  Setting the
 * parameters restarts Adam. */
int sparc_dnet_set_params(sparc_dnet* net, const float* theta);
/* Precision of the network's inference (sparc_dnet_forward, sparc_dnet_predict_density):
 * 0 FP32 (default); 1 bfloat16 activations and weights (round-to-nearest-even of the
 * FP32 values) with FP32 products and sums, the last layer's output and the head in
 * FP32.  Training (loss_grad, train_step) always runs in FP32.  Errors: EINVAL. */
int sparc_dnet_set_precision(sparc_dnet* net, int32_t bf16);
int sparc_dnet_get_params(const sparc_dnet* net, float* theta);
/* x_dev (FP32, N_d) = rho_dev / rho_bar: the scaling of the training targets. */
int sparc_dnet_scale_density(sparc_dnet* net, const double* rho_dev, double n_elec, double dV, float* x_dev);
/* in_dev (FP32, N_d x 2) = (rho_dev / rho_bar, -vloc_dev): one cell's network input
 * from its atomic superposition and local potential (device FP64). */
int sparc_dnet_prepare_input(sparc_dnet* net, const double* rho_dev, const double* vloc_dev, double n_elec, double dV,
                             float* in_dev);
/* Raw network output d = f(x, u) for `batch` cells (d_dev: batch * N_d floats). */
int sparc_dnet_forward(sparc_dnet* net, const float* in_dev, int32_t batch, float* d_dev);
/* Loss L = mean over cells and points of (x + d - mean(d) - y)^2 and its
 * gradient (kept on the device for sparc_dnet_adam_step; also copied to grad_host,
 * in the host parameter layout, when that is not NULL).  Synchronous.  ENAN for a
 * non-finite loss. */
int sparc_dnet_loss_grad(sparc_dnet* net, const float* in_dev, const float* y_dev, int32_t batch, double* loss,
                         float* grad_host);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the last
 * gradient. */
int sparc_dnet_adam_step(sparc_dnet* net, double lr);
/* loss_grad followed by adam_step. */
int sparc_dnet_train_step(sparc_dnet* net, const float* in_dev, const float* y_dev, int32_t batch, double lr,
                          double* loss);
/* Learned start density of one cell from its atomic superposition and local
 * potential (device FP64, N_d each); rho_dev receives rho_0 (FP64, h^3 sum =
 * n_elec).  Falls back to a copy of rho_sad_dev, with *used_net = 0, when any value
 * is not finite or the charge before renormalisation differs from n_elec by more
 * than charge_tol * n_elec.  Synchronous. */
int sparc_dnet_predict_density(sparc_dnet* net, const double* rho_sad_dev, const double* vloc_dev, double n_elec,
                               double dV, double charge_tol, double* rho_dev, int32_t* used_net);

#ifdef __cplusplus
}
#endif
#endif /* SPARC_HIP_H */
