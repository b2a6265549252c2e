// C-ABI entry points of the CheFSI hot path: H*X, Chebyshev filter,
// Rayleigh-Ritz, Lanczos bounds, density and Fermi level.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "devmath.hpp"

namespace sparc {

// ------------------------------------------------------------ workspace carving
struct Carver {
  char* p;
  size_t left;
  bool ok = true;
  void* take(size_t bytes) {
    size_t b = ((bytes + 255) / 256) * 256;
    if (b > left) { ok = false; return nullptr; }
    void* q = p;
    p += b;
    left -= b;
    return q;
  }
};
static size_t al(size_t b) { return ((b + 255) / 256) * 256; }

int check_ham(const sparc_ham* H, const char* who) {
  if (!H) return fail(SPARC_EINVAL, "%s: ham is NULL", who);
  return SPARC_OK;
}

int check_block(const sparc_ham* H, const void* X, int64_t ldx, int32_t n_s, const char* who) {
  if (!X) return fail(SPARC_EINVAL, "%s: block pointer is NULL", who);
  if (n_s < 1) return fail(SPARC_ESHAPE, "%s: n_s=%d < 1", who, n_s);
  if (ldx < H->n_d) return fail(SPARC_ESHAPE, "%s: ld=%lld < N_d=%lld", who, (long long)ldx, (long long)H->n_d);
  return SPARC_OK;
}

// ------------------------------------------------------------ small element-wise kernels
template <typename E>
__global__ void scale_by_rnorm_kernel(const E* __restrict__ x, E* __restrict__ y, int64_t n, const double* nrm2) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 1.0 / sqrt(nrm2[0]);
  y[i] = scale((typename elem<E>::real)s, x[i]);
}

template <typename E>
__global__ void sub_kernel(E* __restrict__ w, const E* __restrict__ t, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) w[i] = w[i] + scale((typename elem<E>::real)-1, t[i]);
}

__global__ void herm_sym_kernel(int n, double* A, int cplx) {
  int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  int i = (int)(idx % n), j = (int)(idx / n);
  if (i > j) return;
  if (!cplx) {
    double v = 0.5 * (A[i + (int64_t)j * n] + A[j + (int64_t)i * n]);
    A[i + (int64_t)j * n] = v;
    A[j + (int64_t)i * n] = v;
  } else {
    double* a = A + 2 * (i + (int64_t)j * n);
    double* b = A + 2 * (j + (int64_t)i * n);
    double re = 0.5 * (a[0] + b[0]), im = 0.5 * (a[1] - b[1]);
    if (i == j) im = 0;
    a[0] = re; a[1] = im;
    b[0] = re; b[1] = -im;
  }
}

// Lanczos: coefficients -> tridiagonal matrix (dense, n x n) and bookkeeping
__global__ void lanczos_record_kernel(const double* c, int j, int cplx, double* alph) {
  if (threadIdx.x == 0 && blockIdx.x == 0) alph[j] = c[cplx ? 2 * j : j];
}
__global__ void lanczos_beta_kernel(const double* nrm2, int j, double* beta) {
  if (threadIdx.x == 0 && blockIdx.x == 0) beta[j] = sqrt(nrm2[0]);
}
__global__ void tridiag_kernel(int m, const double* alph, const double* beta, double* T) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  int i = idx % m, j = idx / m;
  double v = 0;
  if (i == j) v = alph[i];
  else if (i == j + 1) v = beta[j];
  else if (j == i + 1) v = beta[i];
  T[idx] = v;
}

// ------------------------------------------------------------ density
constexpr int MAXK = 64;
template <typename E>
struct DensArgs {
  const E* x[MAXK];
  int64_t ld[MAXK];
};

template <typename E>
__global__ __launch_bounds__(256) void density_kernel(DensArgs<E> A, int nk, int n_s, int64_t n_d,
                                                      const double* __restrict__ occ, double scale_,
                                                      double* __restrict__ rho) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= n_d) return;
  double acc = 0;
  for (int b = 0; b < nk; ++b) {
    const E* __restrict__ x = A.x[b];
    const int64_t ld = A.ld[b];
    const double* oc = occ + (int64_t)b * n_s;
    int n = 0;
    for (; n + 4 <= n_s; n += 4) {
      E v0 = x[g + (int64_t)n * ld], v1 = x[g + (int64_t)(n + 1) * ld];
      E v2 = x[g + (int64_t)(n + 2) * ld], v3 = x[g + (int64_t)(n + 3) * ld];
      acc += oc[n] * abs2(v0) + oc[n + 1] * abs2(v1) + oc[n + 2] * abs2(v2) + oc[n + 3] * abs2(v3);
    }
    for (; n < n_s; ++n) acc += oc[n] * abs2(x[g + (int64_t)n * ld]);
  }
  rho[g] = scale_ * acc;
}

// ------------------------------------------------------------ Fermi level
struct FermiArgs {
  double wk[MAXK];
};
__global__ __launch_bounds__(256) void fermi_kernel(int nk, int ns, const double* __restrict__ lam, FermiArgs W,
                                                    double ne, double kT, double* __restrict__ occ_w,
                                                    double* __restrict__ mu_out) {
  __shared__ double red[4];
  __shared__ double s_lo, s_hi;
  const int tid = threadIdx.x;
  const int tot = nk * ns;
  double lmin = 1e300, lmax = -1e300;
  for (int i = tid; i < tot; i += blockDim.x) { lmin = fmin(lmin, lam[i]); lmax = fmax(lmax, lam[i]); }
  // block min / max
  for (int o = 32; o > 0; o >>= 1) {
    lmin = fmin(lmin, __shfl_xor(lmin, o, 64));
    lmax = fmax(lmax, __shfl_xor(lmax, o, 64));
  }
  __shared__ double mn[4], mx[4];
  if ((tid & 63) == 0) { mn[tid >> 6] = lmin; mx[tid >> 6] = lmax; }
  __syncthreads();
  if (tid == 0) {
    double a = mn[0], b = mx[0];
    for (int i = 1; i < (int)(blockDim.x >> 6); ++i) { a = fmin(a, mn[i]); b = fmax(b, mx[i]); }
    s_lo = a - 40.0 * kT - 1.0;
    s_hi = b + 40.0 * kT + 1.0;
  }
  __syncthreads();
  double lo = s_lo, hi = s_hi;
  auto count = [&](double mu) {
    double c = 0;
    for (int i = tid; i < tot; i += blockDim.x) {
      int b = i / ns;
      c += 2.0 * W.wk[b] * 0.5 * (1.0 - tanh((lam[i] - mu) / (2.0 * kT)));
    }
    c = wave_sum(c);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = c;
    __syncthreads();
    double s = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    return s;
  };
  // Brent's method (inverse quadratic interpolation or secant inside a bracket, with
  // bisection whenever the interpolated step is not safely inside it or shrinks too
  // slowly) on f(mu) = count(mu) - ne, which increases with mu; f(lo) < 0 < f(hi).
  // Every thread runs the same scalar iteration on the block-reduced counts.
  double a = lo, b = hi, fa = count(lo) - ne, fb = count(hi) - ne;
  if (fabs(fa) < fabs(fb)) { double t = a; a = b; b = t; t = fa; fa = fb; fb = t; }
  double c = a, fc = fa, d = a;
  bool bisected = true;
  for (int it = 0; it < 200; ++it) {
    if (fabs(fb) < 1e-13 * ne || fabs(b - a) < 1e-15 * fmax(1.0, fabs(b))) break;
    double s;
    if (fa != fc && fb != fc) {  // inverse quadratic interpolation through (a, fa), (b, fb), (c, fc)
      s = a * fb * fc / ((fa - fb) * (fa - fc)) + b * fa * fc / ((fb - fa) * (fb - fc)) +
          c * fa * fb / ((fc - fa) * (fc - fb));
    } else {  // secant through (a, fa), (b, fb)
      s = b - fb * (b - a) / (fb - fa);
    }
    const double q = 0.25 * (3.0 * a + b);
    const double tol = 1e-15 * fmax(1.0, fabs(b));
    const bool outside = !((s > fmin(q, b)) && (s < fmax(q, b)));
    const bool slow = bisected ? (fabs(s - b) >= 0.5 * fabs(b - c) || fabs(b - c) < tol)
                               : (fabs(s - b) >= 0.5 * fabs(c - d) || fabs(c - d) < tol);
    if (outside || slow || !isfinite(s)) {
      s = 0.5 * (a + b);
      bisected = true;
    } else {
      bisected = false;
    }
    const double fs = count(s) - ne;
    d = c;
    c = b;
    fc = fb;
    if ((fa < 0.0) != (fs < 0.0)) { b = s; fb = fs; }
    else { a = s; fa = fs; }
    if (fabs(fa) < fabs(fb)) { double t = a; a = b; b = t; t = fa; fa = fb; fb = t; }
  }
  double mu = b;
  if (tid == 0) *mu_out = mu;
  if (occ_w)
    for (int i = tid; i < tot; i += blockDim.x) {
      int b = i / ns;
      occ_w[i] = W.wk[b] * 0.5 * (1.0 - tanh((lam[i] - mu) / (2.0 * kT)));
    }
}

// ------------------------------------------------------------ Rayleigh-Ritz workspace
struct RRWork {
  void *W1, *W2, *alpha, *M, *T1, *T2, *A1, *tmp, *Z, *Qf, *qp, *gw, *cw, *hw;
  int* info;
  size_t gw_bytes;
};

static size_t rr_layout(const sparc_ham* H, int32_t n_s, void* base, size_t bytes, RRWork* w) {
  const bool cp = dtype_complex(H->dtype);
  const size_t blk = (size_t)H->n_d * n_s * elem_bytes(H->dtype);
  const size_t sm = (size_t)n_s * n_s * (cp ? 16 : 8);
  const size_t gwb = std::max(gram_work_bytes(H->n_d, n_s, n_s, H->dtype),
                              gram_work_bytes(n_s, n_s, n_s, cp ? SPARC_C128 : SPARC_R64));
  size_t need = al(blk) * 2 + al(alpha_bytes(H, n_s)) + al(sm) * 8 + al(gwb) +
                al(chol_orth_work_bytes(n_s, cp)) + al(heev_work_bytes(n_s, cp)) + 256;
  if (w && base) {
    Carver c{(char*)base, bytes};
    w->W1 = c.take(blk);
    w->W2 = c.take(blk);
    w->alpha = c.take(alpha_bytes(H, n_s));
    w->M = c.take(sm);
    w->T1 = c.take(sm);
    w->T2 = c.take(sm);
    w->A1 = c.take(sm);
    w->tmp = c.take(sm);
    w->Z = c.take(sm);
    w->Qf = c.take(sm);
    w->qp = c.take(sm);
    w->gw = c.take(gwb);
    w->gw_bytes = gwb;
    w->cw = c.take(chol_orth_work_bytes(n_s, cp));
    w->hw = c.take(heev_work_bytes(n_s, cp));
    w->info = (int*)c.take(256);
    if (!c.ok) return 0;
  }
  return need;
}

struct LzWork {
  void *V, *w, *t, *alpha, *c, *nrm, *alph, *beta, *T, *S, *theta, *gw, *hw;
  size_t gw_bytes;
};

static size_t lz_layout(const sparc_ham* H, int32_t m, void* base, size_t bytes, LzWork* w) {
  const size_t eb = elem_bytes(H->dtype);
  const size_t vb = (size_t)H->n_d * eb;
  const size_t gwb = gram_work_bytes(H->n_d, m + 1, 1, H->dtype);
  size_t need = al(vb * (m + 1)) + 2 * al(vb) + al(alpha_bytes(H, 1)) + al((m + 1) * 16) + al(64) + 2 * al(m * 8) +
                2 * al((size_t)m * m * 8) + al(m * 8) + al(gwb) + al(heev_work_bytes(m, false)) + 256;
  if (w && base) {
    Carver c{(char*)base, bytes};
    w->V = c.take(vb * (m + 1));
    w->w = c.take(vb);
    w->t = c.take(vb);
    w->alpha = c.take(alpha_bytes(H, 1));
    w->c = c.take((m + 1) * 16);
    w->nrm = c.take(64);
    w->alph = c.take(m * 8);
    w->beta = c.take(m * 8);
    w->T = c.take((size_t)m * m * 8);
    w->S = c.take((size_t)m * m * 8);
    w->theta = c.take(m * 8);
    w->gw = c.take(gwb);
    w->gw_bytes = gwb;
    w->hw = c.take(heev_work_bytes(m, false));
    if (!c.ok) return 0;
  }
  return need;
}

template <typename E>
static int launch_scale(hipStream_t s, const void* x, void* y, int64_t n, const double* nrm2) {
  scale_by_rnorm_kernel<E><<<(unsigned)((n + 255) / 256), 256, 0, s>>>((const E*)x, (E*)y, n, nrm2);
  return check_launch("scale_by_rnorm_kernel");
}
template <typename E>
static int launch_sub(hipStream_t s, void* w, const void* t, int64_t n) {
  sub_kernel<E><<<(unsigned)((n + 255) / 256), 256, 0, s>>>((E*)w, (const E*)t, n);
  return check_launch("sub_kernel");
}
static int scale_rnorm(sparc_dtype dt, hipStream_t s, const void* x, void* y, int64_t n, const double* nrm2) {
  switch (dt) {
    case SPARC_R64: return launch_scale<double>(s, x, y, n, nrm2);
    case SPARC_R32: return launch_scale<float>(s, x, y, n, nrm2);
    case SPARC_C128: return launch_scale<cd>(s, x, y, n, nrm2);
    case SPARC_C64: return launch_scale<cf>(s, x, y, n, nrm2);
  }
  return SPARC_EINVAL;
}
static int sub_vec(sparc_dtype dt, hipStream_t s, void* w, const void* t, int64_t n) {
  switch (dt) {
    case SPARC_R64: return launch_sub<double>(s, w, t, n);
    case SPARC_R32: return launch_sub<float>(s, w, t, n);
    case SPARC_C128: return launch_sub<cd>(s, w, t, n);
    case SPARC_C64: return launch_sub<cf>(s, w, t, n);
  }
  return SPARC_EINVAL;
}

// Chebyshev filter of degree m (three-term recurrence, one stencil step per degree):
// each step projects its input onto the projectors, then the stencil step applies the
// local and (inside the step, or with the scatter kernel after it) non-local terms.
int filter_impl(sparc_ham* H, void* X, int64_t ldx, int32_t n_s, int32_t degree, double lcut, double lmax,
                void* Wb, void* alpha) {
  const double c = 0.5 * (lmax + lcut), e = 0.5 * (lmax - lcut);
  const int64_t N = H->n_d;
  SPARC_TRY(nl_project(H, X, ldx, n_s, alpha));
  SPARC_TRY(ham_step(H, X, ldx, nullptr, 0, Wb, N, n_s, 1.0 / e, -c / e, 0.0, alpha));
  void* prev = X;
  int64_t ldp = ldx;
  void* cur = Wb;
  int64_t ldc = N;
  for (int j = 1; j < degree; ++j) {
    SPARC_TRY(nl_project(H, cur, ldc, n_s, alpha));
    SPARC_TRY(ham_step(H, cur, ldc, prev, ldp, prev, ldp, n_s, 2.0 / e, -2.0 * c / e, -1.0, alpha));
    std::swap(prev, cur);
    std::swap(ldp, ldc);
  }
  if (cur != X) {
    size_t eb = elem_bytes(H->dtype);
    SPARC_HIP(hipMemcpy2DAsync(X, ldx * eb, cur, ldc * eb, N * eb, n_s, hipMemcpyDeviceToDevice, H->ctx->stream));
  }
  return SPARC_OK;
}

// Out = A Q for the N_d-long rotations of Rayleigh-Ritz: split-BF16 (x3) products from
// pieces made in W2 (free at every rotation) when the mode asks for them and n is a
// multiple of 16, else the element type's MFMA
// dst(:, c) = src(:, c) for n columns of `bytes` bytes each: one 16-byte element per
// thread, all accesses non-temporal (the block is streamed once); falls back to a 2-D
// runtime copy when the columns or leading dimensions are not 16-byte multiples
typedef double v2d_t __attribute__((ext_vector_type(2)));
__global__ __launch_bounds__(256) void copy_cols_kernel(const v2d_t* __restrict__ src, int64_t lds,
                                                        v2d_t* __restrict__ dst, int64_t ldd, int64_t rows) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (i < rows) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[c * lds + i]), &dst[c * ldd + i]);
}

static int copy_cols(hipStream_t s, void* dst, int64_t ld_dst, const void* src, int64_t ld_src, int64_t bytes,
                     int32_t n) {
  const bool vec = bytes % 16 == 0 && ld_dst % 16 == 0 && ld_src % 16 == 0 && (uintptr_t)dst % 16 == 0 &&
                   (uintptr_t)src % 16 == 0 && n <= 65535 && (bytes / 16 + 255) / 256 <= (int64_t)UINT32_MAX;
  if (!vec) {
    SPARC_HIP(hipMemcpy2DAsync(dst, ld_dst, src, ld_src, bytes, n, hipMemcpyDeviceToDevice, s));
    return SPARC_OK;
  }
  const int64_t rows = bytes / 16;
  copy_cols_kernel<<<dim3((unsigned)((rows + 255) / 256), (unsigned)n), 256, 0, s>>>(
      (const v2d_t*)src, ld_src / 16, (v2d_t*)dst, ld_dst / 16, rows);
  return check_launch("copy_cols_kernel");
}

static int rr_rotate(sparc_ham* H, sparc_gemm_mode mode, int32_t n, const void* A, int64_t lda, const void* Q,
                     void* Out, int64_t ldo, int q_upper, RRWork& w) {
  hipStream_t s = H->ctx->stream;
  if (mode == SPARC_GEMM_BF16X3 && dtype_single(H->dtype) && n % 16 == 0)
    return rotate_split_x3(s, H->dtype, H->n_d, n, n, A, lda, Q, n, Out, ldo, q_upper, w.W2, w.qp);
  return rotate(s, H->dtype, H->n_d, n, n, A, lda, Q, n, Out, ldo, q_upper, H->ctx);
}

// Largest estimated condition number of the column-scaled Gram matrix for which one
// Cholesky-QR pass is taken (orthonormality defect about kappa * eps); above it, two.
constexpr double kSinglePassKappa = 50.0;

int rr_impl(sparc_ham* H, void* X, int64_t ldx, int32_t n, sparc_gemm_mode mode, double* ritz, RRWork& w,
            int32_t* info_out) {
  hipStream_t s = H->ctx->stream;
  const sparc_dtype dt = H->dtype;
  const bool cp = dtype_complex(dt);
  const sparc_dtype sdt = cp ? SPARC_C128 : SPARC_R64;
  const int64_t N = H->n_d;
  const int ncu = H->ctx->n_cu;
  g_timer_ctx = H->ctx;
  int info = 0;
  // pass 1: T1 from the Gram matrix of X (shifted if it is numerically singular), and the
  // condition estimate of the column-scaled Gram matrix
  SPARC_TRY(gram(s, dt, N, n, n, X, ldx, X, ldx, w.M, n, w.gw, w.gw_bytes, mode, ncu, false, H->ctx));
  bool shifted = false;
  SPARC_TRY(chol_orth(s, cp, n, w.M, w.T1, w.info, w.cw, 0.0));
  double* kappa_dev = (double*)((char*)w.info + 8);
  SPARC_TRY(chol_cond_est(s, cp, n, w.M, w.T1, w.info, w.cw, kappa_dev));
  struct { int32_t info; int32_t pad; double kappa; } st{};
  SPARC_HIP(hipMemcpyAsync(&st, w.info, sizeof(st), hipMemcpyDeviceToHost, s));
  SPARC_HIP(hipStreamSynchronize(s));
  info = st.info;
  if (info == 0 && st.kappa <= kSinglePassKappa) {
    // a nearly orthogonal block (the steady state of the iteration): one Cholesky-QR pass
    // leaves an orthonormality defect of about kappa * eps, so H X, the projected matrix
    // and the rotation to the Ritz vectors are taken on X itself, T = T1
    SPARC_TRY(nl_project(H, X, ldx, n, w.alpha));
    SPARC_TRY(ham_step(H, X, ldx, nullptr, 0, w.W2, N, n, 1.0, 0.0, 0.0, w.alpha));
    SPARC_TRY(gram(s, dt, N, n, n, X, ldx, w.W2, N, w.A1, n, w.gw, w.gw_bytes, mode, ncu, true, H->ctx));
    SPARC_TRY(rotate(s, sdt, n, n, n, w.A1, n, w.T1, n, w.tmp, n, 1));
    SPARC_TRY(gram(s, sdt, n, n, n, w.T1, n, w.tmp, n, w.A1, n, w.gw, w.gw_bytes, SPARC_GEMM_NATIVE, ncu, true));
    herm_sym_kernel<<<(unsigned)(((int64_t)n * n + 255) / 256), 256, 0, s>>>(n, (double*)w.A1, cp ? 1 : 0);
    SPARC_TRY(check_launch("herm_sym_kernel"));
    SPARC_TRY(heev(s, cp, n, w.A1, ritz, w.Z, w.hw));
    // U = X (T1 Z), formed out of place and copied back
    SPARC_TRY(rotate(s, sdt, n, n, n, w.T1, n, w.Z, n, w.Qf, n, 0));
    SPARC_TRY(rr_rotate(H, mode, n, X, ldx, w.Qf, w.W1, N, 0, w));
    SPARC_TRY(copy_cols(s, X, ldx * elem_bytes(dt), w.W1, N * elem_bytes(dt), N * elem_bytes(dt), n));
    if (info_out) *info_out = 0;
    return SPARC_OK;
  }
  if (info != 0) {
    const double shift = 11.0 * ((double)N * n + (double)n * (n + 1)) * 2.2e-16 * n;
    SPARC_TRY(chol_orth(s, cp, n, w.M, w.T1, w.info, w.cw, shift));
    SPARC_HIP(hipMemcpyAsync(&info, w.info, 4, hipMemcpyDeviceToHost, s));
    SPARC_HIP(hipStreamSynchronize(s));
    if (info != 0) {
      if (info_out) *info_out = info;
      return fail(SPARC_ENOTSPD, "rayleigh_ritz: Gram matrix not positive definite at column %d", info);
    }
    shifted = true;
  }
  SPARC_TRY(rr_rotate(H, mode, n, X, ldx, w.T1, w.W1, N, 1, w));
  if (shifted) {  // one more explicit pass after a shifted factorisation
    SPARC_TRY(gram(s, dt, N, n, n, w.W1, N, w.W1, N, w.M, n, w.gw, w.gw_bytes, mode, ncu, false, H->ctx));
    SPARC_TRY(chol_orth(s, cp, n, w.M, w.T1, w.info, w.cw, 0.0));
    SPARC_HIP(hipMemcpyAsync(&info, w.info, 4, hipMemcpyDeviceToHost, s));
    SPARC_HIP(hipStreamSynchronize(s));
    if (info != 0) {
      if (info_out) *info_out = info;
      return fail(SPARC_ENOTSPD, "rayleigh_ritz: Gram matrix not positive definite at column %d", info);
    }
    SPARC_TRY(rr_rotate(H, mode, n, w.W1, N, w.T1, X, ldx, 1, w));
    SPARC_HIP(hipMemcpy2DAsync(w.W1, N * elem_bytes(dt), X, ldx * elem_bytes(dt), N * elem_bytes(dt), n,
                               hipMemcpyDeviceToDevice, s));
  }
  // pass 2 (implicit): T2 from the Gram matrix of X1 = X T1
  SPARC_TRY(gram(s, dt, N, n, n, w.W1, N, w.W1, N, w.M, n, w.gw, w.gw_bytes, mode, ncu, false, H->ctx));
  SPARC_TRY(chol_orth(s, cp, n, w.M, w.T2, w.info, w.cw, 0.0));
  // H X1 and the projected matrix A1 = X1^H H X1 (Hermitian: its upper triangle, mirrored)
  SPARC_TRY(nl_project(H, w.W1, N, n, w.alpha));
  SPARC_TRY(ham_step(H, w.W1, N, nullptr, 0, w.W2, N, n, 1.0, 0.0, 0.0, w.alpha));
  SPARC_TRY(gram(s, dt, N, n, n, w.W1, N, w.W2, N, w.A1, n, w.gw, w.gw_bytes, mode, ncu, true, H->ctx));
  // H~ = T2^H A1 T2 (FP64, Hermitian by the same mirror), symmetrised
  SPARC_TRY(rotate(s, sdt, n, n, n, w.A1, n, w.T2, n, w.tmp, n, 1));
  SPARC_TRY(gram(s, sdt, n, n, n, w.T2, n, w.tmp, n, w.A1, n, w.gw, w.gw_bytes, SPARC_GEMM_NATIVE, ncu, true));
  herm_sym_kernel<<<(unsigned)(((int64_t)n * n + 255) / 256), 256, 0, s>>>(n, (double*)w.A1, cp ? 1 : 0);
  SPARC_TRY(check_launch("herm_sym_kernel"));
  SPARC_HIP(hipMemcpyAsync(&info, w.info, 4, hipMemcpyDeviceToHost, s));
  SPARC_HIP(hipStreamSynchronize(s));
  if (info != 0) {
    if (info_out) *info_out = info;
    return fail(SPARC_ENOTSPD, "rayleigh_ritz: second Gram matrix not positive definite at column %d", info);
  }
  SPARC_TRY(heev(s, cp, n, w.A1, ritz, w.Z, w.hw));
  // U = X1 (T2 Z)
  SPARC_TRY(rotate(s, sdt, n, n, n, w.T2, n, w.Z, n, w.Qf, n, 0));
  SPARC_TRY(rr_rotate(H, mode, n, w.W1, N, w.Qf, X, ldx, 0, w));
  if (info_out) *info_out = 0;
  return SPARC_OK;
}

}  // namespace sparc

using namespace sparc;

extern "C" {

size_t sparc_workspace_bytes(const sparc_ham* H, int32_t n_s, int32_t op) {
  if (!H || n_s < 1) return 0;
  const size_t blk = (size_t)H->n_d * n_s * elem_bytes(H->dtype);
  switch (op) {
    case SPARC_OP_APPLY: return al(alpha_bytes(H, n_s));
    case SPARC_OP_FILTER: return al(blk) + al(alpha_bytes(H, n_s));
    case SPARC_OP_RR: return rr_layout(H, n_s, nullptr, 0, nullptr);
    case SPARC_OP_LANCZOS: return lz_layout(H, n_s, nullptr, 0, nullptr);
    case SPARC_OP_FORCES: return al(alpha_bytes(H, n_s)) + al(force_nl_part_bytes(H, n_s));
  }
  return 0;
}

int fd_hamiltonian_apply(sparc_ham* H, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t n_s, void* work,
                         size_t work_bytes) {
  SPARC_TRY(check_ham(H, "fd_hamiltonian_apply"));
  SPARC_TRY(check_block(H, X, ldx, n_s, "fd_hamiltonian_apply"));
  SPARC_TRY(check_block(H, Y, ldy, n_s, "fd_hamiltonian_apply"));
  if (X == Y) return fail(SPARC_EINVAL, "fd_hamiltonian_apply: X and Y must not alias");
  size_t need = sparc_workspace_bytes(H, n_s, SPARC_OP_APPLY);
  if (H->n_proj > 0 && (!work || work_bytes < need))
    return fail(SPARC_ENOMEM, "fd_hamiltonian_apply: workspace %zu < %zu bytes", work_bytes, need);
  SPARC_TRY(nl_project(H, X, ldx, n_s, work));
  return ham_step(H, X, ldx, nullptr, 0, Y, ldy, n_s, 1.0, 0.0, 0.0, work);
}

int chebyshev_filter(sparc_ham* H, void* X, int64_t ldx, int32_t n_s, int32_t degree, double lambda_cut,
                     double lambda_max, void* work, size_t work_bytes) {
  SPARC_TRY(check_ham(H, "chebyshev_filter"));
  SPARC_TRY(check_block(H, X, ldx, n_s, "chebyshev_filter"));
  if (degree < 1) return fail(SPARC_EINVAL, "chebyshev_filter: degree=%d < 1", degree);
  if (!(lambda_max > lambda_cut) || !std::isfinite(lambda_max) || !std::isfinite(lambda_cut))
    return fail(SPARC_EINVAL, "chebyshev_filter: need finite lambda_max > lambda_cut");
  size_t need = sparc_workspace_bytes(H, n_s, SPARC_OP_FILTER);
  if (!work || work_bytes < need) return fail(SPARC_ENOMEM, "chebyshev_filter: workspace %zu < %zu bytes", work_bytes, need);
  const size_t blk = (size_t)H->n_d * n_s * elem_bytes(H->dtype);
  return filter_impl(H, X, ldx, n_s, degree, lambda_cut, lambda_max, work, (char*)work + al(blk));
}

int rayleigh_ritz(sparc_ham* H, void* X, int64_t ldx, int32_t n_s, sparc_gemm_mode mode, double* ritz_dev,
                  void* work, size_t work_bytes, int32_t* info) {
  if (info) *info = 0;
  SPARC_TRY(check_ham(H, "rayleigh_ritz"));
  SPARC_TRY(check_block(H, X, ldx, n_s, "rayleigh_ritz"));
  if (!ritz_dev) return fail(SPARC_EINVAL, "rayleigh_ritz: ritz_dev is NULL");
  if (mode != SPARC_GEMM_NATIVE && mode != SPARC_GEMM_BF16X3 && mode != SPARC_GEMM_BF16X6)
    return fail(SPARC_EINVAL, "rayleigh_ritz: unknown GEMM mode %d", (int)mode);
  if (mode != SPARC_GEMM_NATIVE && !dtype_single(H->dtype))
    return fail(SPARC_EINVAL, "rayleigh_ritz: split-BF16 modes take FP32 / complex64 blocks");
  if (n_s > 2048) return fail(SPARC_ESHAPE, "rayleigh_ritz: n_s=%d above 2048", n_s);
  if (n_s > H->n_d) return fail(SPARC_ESHAPE, "rayleigh_ritz: n_s=%d exceeds N_d", n_s);
  RRWork w;
  size_t need = rr_layout(H, n_s, nullptr, 0, nullptr);
  if (!work || work_bytes < need) return fail(SPARC_ENOMEM, "rayleigh_ritz: workspace %zu < %zu bytes", work_bytes, need);
  if (!rr_layout(H, n_s, work, work_bytes, &w)) return fail(SPARC_ENOMEM, "rayleigh_ritz: workspace layout failed");
  return rr_impl(H, X, ldx, n_s, mode, ritz_dev, w, info);
}

int lanczos_bounds(sparc_ham* H, const void* v0, int32_t steps, void* work, size_t work_bytes, double* lmin,
                   double* lmax) {
  SPARC_TRY(check_ham(H, "lanczos_bounds"));
  if (!v0 || !lmin || !lmax) return fail(SPARC_EINVAL, "lanczos_bounds: null argument");
  if (steps < 2 || steps > 512 || steps > H->n_d) return fail(SPARC_EINVAL, "lanczos_bounds: steps=%d outside 2..512", steps);
  LzWork w;
  size_t need = lz_layout(H, steps, nullptr, 0, nullptr);
  if (!work || work_bytes < need) return fail(SPARC_ENOMEM, "lanczos_bounds: workspace %zu < %zu bytes", work_bytes, need);
  if (!lz_layout(H, steps, work, work_bytes, &w)) return fail(SPARC_ENOMEM, "lanczos_bounds: workspace layout failed");
  hipStream_t s = H->ctx->stream;
  const sparc_dtype dt = H->dtype;
  const bool cp = dtype_complex(dt);
  const int64_t N = H->n_d;
  const size_t eb = elem_bytes(dt);
  const int ncu = H->ctx->n_cu;
  char* V = (char*)w.V;
  const int m = steps;
  SPARC_TRY(gram(s, dt, N, 1, 1, v0, N, v0, N, w.nrm, 1, w.gw, w.gw_bytes, SPARC_GEMM_NATIVE, ncu));
  SPARC_TRY(scale_rnorm(dt, s, v0, V, N, (const double*)w.nrm));
  for (int j = 0; j < m; ++j) {
    void* vj = V + (size_t)j * N * eb;
    SPARC_TRY(nl_project(H, vj, N, 1, w.alpha));
    SPARC_TRY(ham_step(H, vj, N, nullptr, 0, w.w, N, 1, 1.0, 0.0, 0.0, w.alpha));
    for (int pass = 0; pass < 2; ++pass) {
      SPARC_TRY(gram(s, dt, N, j + 1, 1, V, N, w.w, N, w.c, j + 1, w.gw, w.gw_bytes, SPARC_GEMM_NATIVE, ncu));
      if (pass == 0) {
        lanczos_record_kernel<<<1, 1, 0, s>>>((const double*)w.c, j, cp ? 1 : 0, (double*)w.alph);
        SPARC_TRY(check_launch("lanczos_record_kernel"));
      }
      SPARC_TRY(rotate(s, dt, N, j + 1, 1, V, N, w.c, j + 1, w.t, N, 0));
      SPARC_TRY(sub_vec(dt, s, w.w, w.t, N));
    }
    SPARC_TRY(gram(s, dt, N, 1, 1, w.w, N, w.w, N, w.nrm, 1, w.gw, w.gw_bytes, SPARC_GEMM_NATIVE, ncu));
    lanczos_beta_kernel<<<1, 1, 0, s>>>((const double*)w.nrm, j, (double*)w.beta);
    SPARC_TRY(check_launch("lanczos_beta_kernel"));
    if (j + 1 < m) SPARC_TRY(scale_rnorm(dt, s, w.w, V + (size_t)(j + 1) * N * eb, N, (const double*)w.nrm));
  }
  tridiag_kernel<<<(m * m + 255) / 256, 256, 0, s>>>(m, (const double*)w.alph, (const double*)w.beta, (double*)w.T);
  SPARC_TRY(check_launch("tridiag_kernel"));
  SPARC_TRY(heev(s, false, m, w.T, (double*)w.theta, w.S, w.hw));
  std::vector<double> theta(m), S(m * m), beta(m);
  SPARC_HIP(hipMemcpyAsync(theta.data(), w.theta, m * 8, hipMemcpyDeviceToHost, s));
  SPARC_HIP(hipMemcpyAsync(S.data(), w.S, m * m * 8, hipMemcpyDeviceToHost, s));
  SPARC_HIP(hipMemcpyAsync(beta.data(), w.beta, m * 8, hipMemcpyDeviceToHost, s));
  SPARC_HIP(hipStreamSynchronize(s));
  double up = theta[m - 1] + std::fabs(beta[m - 1] * S[(m - 1) + (size_t)(m - 1) * m]);
  up += 0.01 * std::fabs(up);
  *lmin = theta[0];
  *lmax = up;
  if (!std::isfinite(*lmin) || !std::isfinite(*lmax)) return fail(SPARC_ENAN, "lanczos_bounds: non-finite bounds");
  return SPARC_OK;
}

int density_from_orbitals(sparc_ctx* ctx, int32_t n_k, const void* const* X, const int64_t* ldx, int32_t n_s,
                          sparc_dtype dtype, const double* occ_w, int64_t n_d, double dV, double* rho_dev) {
  if (!ctx || !X || !ldx || !occ_w || !rho_dev) return fail(SPARC_EINVAL, "density_from_orbitals: null argument");
  if (n_k < 1 || n_k > MAXK) return fail(SPARC_EINVAL, "density_from_orbitals: n_k=%d outside 1..%d", n_k, MAXK);
  if (n_s < 1 || n_d < 1) return fail(SPARC_ESHAPE, "density_from_orbitals: empty block");
  if (!(dV > 0)) return fail(SPARC_EINVAL, "density_from_orbitals: dV must be > 0");
  for (int b = 0; b < n_k; ++b) {
    if (!X[b]) return fail(SPARC_EINVAL, "density_from_orbitals: X[%d] is NULL", b);
    if (ldx[b] < n_d) return fail(SPARC_ESHAPE, "density_from_orbitals: ldx[%d] < n_d", b);
  }
  hipStream_t s = ctx->stream;
  unsigned nb = (unsigned)((n_d + 255) / 256);
  const double sc = 2.0 / dV;
#define DENS(E)                                                                                     \
  {                                                                                                 \
    DensArgs<E> A;                                                                                  \
    for (int b = 0; b < n_k; ++b) { A.x[b] = (const E*)X[b]; A.ld[b] = ldx[b]; }                     \
    density_kernel<E><<<nb, 256, 0, s>>>(A, n_k, n_s, n_d, occ_w, sc, rho_dev);                      \
    return check_launch("density_kernel");                                                          \
  }
  switch (dtype) {
    case SPARC_R64: DENS(double)
    case SPARC_R32: DENS(float)
    case SPARC_C128: DENS(cd)
    case SPARC_C64: DENS(cf)
  }
#undef DENS
  return fail(SPARC_EINVAL, "density_from_orbitals: bad dtype");
}

int sparc_fermi(sparc_ctx* ctx, int32_t n_k, int32_t n_s, const double* lambda_dev, const double* wk, double n_elec,
                double kT, double* occ_w_dev, double* mu) {
  if (!ctx || !lambda_dev || !wk || !mu) return fail(SPARC_EINVAL, "sparc_fermi: null argument");
  if (n_k < 1 || n_k > MAXK || n_s < 1) return fail(SPARC_EINVAL, "sparc_fermi: bad sizes");
  if (!(kT > 0) || !(n_elec > 0)) return fail(SPARC_EINVAL, "sparc_fermi: kT and n_elec must be > 0");
  double wsum = 0;
  for (int b = 0; b < n_k; ++b) wsum += wk[b];
  if (n_elec > 2.0 * n_s * wsum * (1.0 - 1e-12))
    return fail(SPARC_EINVAL, "sparc_fermi: %g electrons do not fit in %d states", n_elec, n_s);
  FermiArgs W;
  for (int b = 0; b < n_k; ++b) W.wk[b] = wk[b];
  double* dmu = ctx->scalars;
  fermi_kernel<<<1, 256, 0, ctx->stream>>>(n_k, n_s, lambda_dev, W, n_elec, kT, occ_w_dev, dmu);
  int rc = check_launch("fermi_kernel");
  double h = 0;
  if (rc == SPARC_OK) {
    hipError_t e = hipMemcpyAsync(&h, dmu, 8, hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) rc = fail(SPARC_EDEVICE, "sparc_fermi: %s", hipGetErrorString(e));
  }
  *mu = h;
  return rc;
}

}  // extern "C"
