// Minimal self-consistent field driver (Gamma point, reduced model):
//   V_eff = V_loc + V_H[rho_in] + V_x[rho_in]   (Slater exchange; jellium Hartree)
//   -Lap_h V_H = 4 pi (rho - mean rho)          (conjugate gradients, FD Laplacian)
//   CheFSI: n_first_passes filter + Rayleigh-Ritz passes on the first step, then one
//   Fermi level, occupations, density; Harris-Foulkes free energy at rho_in
//   rho_in <- rho_in + mix P(rho_out - rho_in), Anderson-extrapolated over the last
//   mix_history iterates, P the Kerker filter (or the identity), until
//   ||rho_out - rho_in|| < tol ||rho_in||
// Every step runs in device kernels; the host only sequences calls and reads
// back scalars (Fermi level, residuals, energy).  With an FP32 filter the passes
// run on an FP32 copy of the orbitals until the density residual stalls near
// FP32 resolution, then switch to FP64 passes (the final FP64 correction).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "devmath.hpp"

namespace sparc {

// ------------------------------------------------------------ reductions
// partial sums of f(i) per block (deterministic two-pass reduction)
enum RedOp { RED_SUM = 0, RED_DOT = 1, RED_DIFF2 = 2 };

constexpr int RED_BLOCKS = 1024;

// One launch per reduction (finish_sums: block partials, then the last block adds them
// in block order)
__device__ __forceinline__ void finish_reduction(double s, double* part, double* __restrict__ out) {
  double v[1] = {s};
  finish_sums<1>(v, part, RED_BLOCKS, out);
}

__global__ __launch_bounds__(256) void reduce_kernel(int64_t n, const double* __restrict__ a,
                                                     const double* __restrict__ b, int op, double* part,
                                                     double* __restrict__ out) {
  double s = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double v;
    if (op == RED_SUM) v = a[i];
    else if (op == RED_DOT) v = a[i] * b[i];
    else { double d = a[i] - b[i]; v = d * d; }
    s += v;
  }
  finish_reduction(s, part, out);
}

// conjugate-gradient update x += a p, r -= a Ap (a = rr / pAp) and the new r.r, one launch
__global__ __launch_bounds__(256) void cg_xr_rr_kernel(int64_t n, double* __restrict__ x, double* __restrict__ r,
                                                       const double* __restrict__ p, const double* __restrict__ Ap,
                                                       const double* rr, const double* pAp, double* part,
                                                       double* __restrict__ rr_new) {
  const double a = (*rr) / (*pAp);
  double s = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    x[i] += a * p[i];
    const double ri = r[i] - a * Ap[i];
    r[i] = ri;
    s += ri * ri;
  }
  finish_reduction(s, part, rr_new);
}

static int red_blocks(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(RED_BLOCKS, (n + 1023) / 1024));
}

// part: RED_BLOCKS doubles and the ticket word (zeroed once after allocation)
static int reduce(hipStream_t s, int64_t n, const double* a, const double* b, int op, double* part, double* out) {
  reduce_kernel<<<red_blocks(n), 256, 0, s>>>(n, a, b, op, part, out);
  return check_launch("reduce");
}

// ------------------------------------------------------------ element-wise kernels
#define GRID1(n) dim3((unsigned)(((n) + 255) / 256)), dim3(256), 0, s

// atomic superposition: Z_J (2 pi w^2)^{-3/2} exp(-r^2/(2 w^2)), images within 10 w
__global__ void sad_kernel(int n1, int n2, int n3, double h1, double h2, double h3, double L1, double L2, double L3,
                           int dmask, int n_atoms, const double* __restrict__ R, const double* __restrict__ W,
                           const double* __restrict__ Z, double* __restrict__ rho) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (g >= (int64_t)n1 * n2 * n3) return;
  int i = (int)(g % n1), j = (int)((g / n1) % n2), k = (int)(g / ((int64_t)n1 * n2));
  double x = i * h1, y = j * h2, z = k * h3, acc = 0;
  for (int a = 0; a < n_atoms; ++a) {
    double w = W[a], rc = 10.0 * w, amp = Z[a] * pow(2.0 * M_PI * w * w, -1.5);
    double dx0 = x - R[3 * a], dy0 = y - R[3 * a + 1], dz0 = z - R[3 * a + 2];
    // images only along periodic directions
    const int az0 = (dmask & 4) ? 0 : (int)ceil((dz0 - rc) / L3), az1 = (dmask & 4) ? 0 : (int)floor((dz0 + rc) / L3);
    const int ay0 = (dmask & 2) ? 0 : (int)ceil((dy0 - rc) / L2), ay1 = (dmask & 2) ? 0 : (int)floor((dy0 + rc) / L2);
    const int ax0 = (dmask & 1) ? 0 : (int)ceil((dx0 - rc) / L1), ax1 = (dmask & 1) ? 0 : (int)floor((dx0 + rc) / L1);
    for (int az = az0; az <= az1; ++az)
      for (int ay = ay0; ay <= ay1; ++ay)
        for (int ax = ax0; ax <= ax1; ++ax) {
          double dx = dx0 - ax * L1, dy = dy0 - ay * L2, dz = dz0 - az * L3;
          double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 <= rc * rc) acc += amp * exp(-r2 / (2.0 * w * w));
        }
  }
  rho[g] = acc;
}

// y = alpha * x (alpha from a device scalar expression: num / den)
__global__ void scale_ratio_kernel(int64_t n, double* __restrict__ y, const double* num, const double* den, double c) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] *= c * (*num) / (*den);
}

// b = 4 pi (rho - sum/n)
__global__ void poisson_rhs_kernel(int64_t n, const double* __restrict__ rho, const double* sum, double* __restrict__ b) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = 4.0 * M_PI * (rho[i] - (*sum) / (double)n);
}

// CG updates with device scalars: alpha = rr / pAp
__global__ void cg_update_p_kernel(int64_t n, double* __restrict__ p, const double* __restrict__ r, const double* rr_new,
                                   const double* rr_old) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) p[i] = r[i] + ((*rr_new) / (*rr_old)) * p[i];
}
__global__ void sub_mean_kernel(int64_t n, double* __restrict__ x, const double* sum) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] -= (*sum) / (double)n;
}
__global__ void copy_kernel(int64_t n, const double* __restrict__ a, double* __restrict__ b) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i];
}
// r = b - A x  with Ax in r on entry
__global__ void residual_kernel(int64_t n, const double* __restrict__ b, double* __restrict__ r) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) r[i] = b[i] - r[i];
}

// Slater exchange and the effective potential; e_dc = eps*rho - vx*rho + 1/2 (b - rho) vh
// (b = 0 for jellium: bpsd == nullptr)
__global__ void xc_veff_kernel(int64_t n, const double* __restrict__ rho, const double* __restrict__ vloc,
                               const double* __restrict__ vh, const double* __restrict__ bpsd,
                               double* __restrict__ veff, double* __restrict__ edc) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double r = fmax(rho[i], 0.0);
  const double r13 = cbrt(r);
  const double eps = -0.75 * cbrt(3.0 / M_PI) * r13;
  const double vx = -cbrt(3.0 / M_PI) * r13;
  veff[i] = vloc[i] + vh[i] + vx;
  const double hb = bpsd ? 0.5 * bpsd[i] : 0.0;
  edc[i] = eps * r - vx * r + (hb - 0.5 * r) * vh[i];
}

__global__ void add_kernel(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                           double* __restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] + b[i];
}

__global__ void mix_kernel(int64_t n, double* __restrict__ rin, const double* __restrict__ rout, double beta) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) rin[i] += beta * (rout[i] - rin[i]);
}

// band and entropy terms from occupations (occ = g for one k-point of weight 1)
__global__ void band_entropy_kernel(int ns, const double* __restrict__ lam, const double* __restrict__ g, double kT,
                                    double* out) {
  double band = 0, ent = 0;
  for (int i = threadIdx.x; i < ns; i += blockDim.x) {
    double gi = g[i];
    band += 2.0 * gi * lam[i];
    double t = 0;
    if (gi > 0) t += gi * log(gi);
    if (gi < 1) t += (1 - gi) * log(1 - gi);
    ent += 2.0 * kT * t;
  }
  __shared__ double rb[4], re[4];
  band = wave_sum(band);
  ent = wave_sum(ent);
  if ((threadIdx.x & 63) == 0) { rb[threadIdx.x >> 6] = band; re[threadIdx.x >> 6] = ent; }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = rb[0] + rb[1] + rb[2] + rb[3];
    out[1] = re[0] + re[1] + re[2] + re[3];
  }
}

// Anderson extrapolation: normal equations of min ||f - dF gamma|| from all pairwise dot
// products (one block per chunk of the grid), a single-thread solve, and the update
constexpr int AMAX = 8;
struct VecSet {
  const double* v[AMAX + 1];
};
template <int NV>
__global__ __launch_bounds__(256) void multi_dot_partial_kernel(int64_t n, VecSet S, double* __restrict__ part) {
  // all pairs (a <= b) of the NV vectors (the last one is f); NP = NV (NV + 1) / 2
  constexpr int NP = NV * (NV + 1) / 2;
  __shared__ double red[4][NP];
  double acc[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) acc[q] = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double x[NV];
#pragma unroll
    for (int a = 0; a < NV; ++a) x[a] = S.v[a][i];
    int q = 0;
#pragma unroll
    for (int a = 0; a < NV; ++a)
#pragma unroll
      for (int b = a; b < NV; ++b) acc[q++] += x[a] * x[b];
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    double v = wave_sum(acc[q]);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][q] = v;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < NP; q += blockDim.x)
    part[(int64_t)blockIdx.x * NP + q] = red[0][q] + red[1][q] + red[2][q] + red[3][q];
}

static void launch_multi_dot(hipStream_t s, int nblk, int64_t n, int m, const VecSet& vs, double* part) {
  switch (m + 1) {
    case 2: multi_dot_partial_kernel<2><<<nblk, 256, 0, s>>>(n, vs, part); break;
    case 3: multi_dot_partial_kernel<3><<<nblk, 256, 0, s>>>(n, vs, part); break;
    case 4: multi_dot_partial_kernel<4><<<nblk, 256, 0, s>>>(n, vs, part); break;
    case 5: multi_dot_partial_kernel<5><<<nblk, 256, 0, s>>>(n, vs, part); break;
    case 6: multi_dot_partial_kernel<6><<<nblk, 256, 0, s>>>(n, vs, part); break;
    case 7: multi_dot_partial_kernel<7><<<nblk, 256, 0, s>>>(n, vs, part); break;
    case 8: multi_dot_partial_kernel<8><<<nblk, 256, 0, s>>>(n, vs, part); break;
    default: multi_dot_partial_kernel<9><<<nblk, 256, 0, s>>>(n, vs, part); break;
  }
}
// gamma from (dF^T dF) gamma = dF^T f by Gaussian elimination with partial pivoting; a
// pivot below 1e-14 of the largest diagonal drops that direction (gamma_k = 0).  One
// work-group of 256 threads: the pair sums over the multi-dot blocks (one wave per pair,
// lanes over blocks), then the elimination in LDS (one matrix element per thread).
__global__ __launch_bounds__(256) void anderson_gamma_kernel(int nblocks, int m, const double* __restrict__ part,
                                                             double* __restrict__ pairs, double* __restrict__ gamma) {
  __shared__ double pr[(AMAX + 1) * (AMAX + 2) / 2];
  __shared__ double A[AMAX][AMAX + 1];
  __shared__ double f[AMAX];
  __shared__ double dmax;
  __shared__ int piv;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int nv = m + 1, np = nv * (nv + 1) / 2;
  for (int q = wv; q < np; q += 4) {
    double v = 0;
    for (int b = lane; b < nblocks; b += 64) v += part[(int64_t)b * np + q];
    v = wave_sum(v);
    if (lane == 0) {
      pr[q] = v;
      pairs[q] = v;
    }
  }
  __syncthreads();
  auto pidx = [&](int a, int b) {  // index of pair (a <= b)
    return a * nv - a * (a - 1) / 2 + (b - a);
  };
  for (int e = tid; e < m * (m + 1); e += 256) {
    const int i = e / (m + 1), j = e % (m + 1);
    A[i][j] = (j < m) ? pr[pidx(min(i, j), max(i, j))] : pr[pidx(i, m)];
  }
  __syncthreads();
  if (tid == 0) {
    double d = 0;
    for (int i = 0; i < m; ++i) d = fmax(d, A[i][i]);
    dmax = d;
  }
  bool dead[AMAX];
  for (int k = 0; k < m; ++k) {
    if (tid == 0) {
      int p = k;
      for (int i = k + 1; i < m; ++i)
        if (fabs(A[i][k]) > fabs(A[p][k])) p = i;
      piv = p;
    }
    __syncthreads();
    const int p = piv;
    if (p != k && tid <= m) {
      const double t = A[k][tid];
      A[k][tid] = A[p][tid];
      A[p][tid] = t;
    }
    __syncthreads();
    dead[k] = fabs(A[k][k]) <= 1e-14 * dmax;
    if (dead[k]) continue;
    if (tid > k && tid < m) f[tid] = A[tid][k] / A[k][k];
    __syncthreads();
    for (int e = tid; e < (m - k - 1) * (m + 1 - k); e += 256) {
      const int i = k + 1 + e / (m + 1 - k), j = k + e % (m + 1 - k);
      A[i][j] -= f[i] * A[k][j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    double x[AMAX];
    for (int k = m - 1; k >= 0; --k) {
      if (dead[k]) {
        x[k] = 0;
        continue;
      }
      double s = A[k][m];
      for (int j = k + 1; j < m; ++j) s -= A[k][j] * x[j];
      x[k] = s / A[k][k];
    }
    for (int i = 0; i < m; ++i) gamma[i] = x[i];
  }
}
struct GammaSet {
  const double* dx[AMAX];
  const double* df[AMAX];
};
// x <- xbar + beta fbar (fbar_out == nullptr), or x <- xbar and fbar_out <- fbar (the
// preconditioned form adds beta P(fbar) afterwards); xbar = x - dX gamma, fbar = f - dF gamma
__global__ void anderson_update_kernel(int64_t n, int m, GammaSet S, const double* __restrict__ gamma,
                                       const double* __restrict__ f, double beta, double* __restrict__ x,
                                       double* __restrict__ fbar_out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double xb = x[i], fb = f[i];
  for (int k = 0; k < m; ++k) {
    const double g = gamma[k];
    xb -= g * S.dx[k][i];
    fb -= g * S.df[k][i];
  }
  if (fbar_out) {
    x[i] = xb;
    fbar_out[i] = fb;
  } else {
    x[i] = xb + beta * fb;
  }
}
// Kerker step: x += beta (f - k2 g), g the Helmholtz solution of f
__global__ void kerker_mix_kernel(int64_t n, double* __restrict__ x, const double* __restrict__ f,
                                  const double* __restrict__ g, double k2, double beta) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] += beta * (f[i] - k2 * g[i]);
}
__global__ void diff_kernel(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ out) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) out[i] = a[i] - b[i];
}

__global__ void d2f_block_kernel(int64_t n, const double* __restrict__ a, float* __restrict__ b) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}
__global__ void f2d_block_kernel(int64_t n, const float* __restrict__ a, double* __restrict__ b) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

// ------------------------------------------------------------ device buffers owned by one SCF run
struct Buffers {
  std::vector<void*> ptrs;
  ~Buffers() {
    for (void* p : ptrs) hipFree(p);
  }
  template <typename T>
  int alloc(T** p, size_t count) {
    *p = nullptr;
    void* q = nullptr;
    if (hipMalloc(&q, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess)
      return fail(SPARC_ENOMEM, "sparc_scf_run: device allocation of %zu bytes failed", count * sizeof(T));
    ptrs.push_back(q);
    *p = (T*)q;
    return SPARC_OK;
  }
};

// -Lap_h V = b by conjugate gradients (V warm-started, zero mean on exit)
struct Poisson {
  sparc_ham* H;
  int64_t n;
  double *b, *r, *p, *Ap, *part, *sc;  // sc: [0] rr, [1] pAp, [2] rr_new, [3] sum, [4] bb
  int iters_total = 0;
  int last_iters = 0;  // iterations of the previous solve: the next one is checked from 3/4 of it

  double shift = 0.0;  // k^2 of the Helmholtz form (-Lap_h + k^2); 0: Poisson
  // two-launch iterations (cg_iterate) on grids whose stencil step runs in point form:
  // w = A r and s = A p, the scalar ring and its partial sums
  bool fused = false;
  double *w = nullptr, *sv = nullptr, *cs = nullptr, *cpart = nullptr;

  int apply(const double* x, double* y) {
    // -Lap_h x + shift x = 2 * (-1/2 Lap_h x) + shift x: stencil only
    return ham_step(H, x, n, nullptr, 0, y, n, 1, 2.0, shift, 0.0, nullptr, STEP_NO_VEFF | STEP_NO_NONLOCAL);
  }

  // (-Lap_h + k2) g = f by conjugate gradients from g = 0 (the operator is positive
  // definite for k2 > 0)
  int solve_helmholtz(hipStream_t s, const double* f, double* g, double k2, double tol, int max_it) {
    SPARC_HIP(hipMemsetAsync(g, 0, n * 8, s));
    copy_kernel<<<GRID1(n)>>>(n, f, b);
    shift = k2;
    const int rc = cg(s, g, tol, max_it, false);
    shift = 0.0;
    return rc;
  }

  int solve(hipStream_t s, const double* rho, double* v, double tol, int max_it) {
    SPARC_TRY(reduce(s, n, rho, nullptr, RED_SUM, part, sc + 3));
    poisson_rhs_kernel<<<GRID1(n)>>>(n, rho, sc + 3, b);
    return cg(s, v, tol, max_it, true);
  }

  // conjugate gradients on apply(v) = b from the current v; zero_mean: remove the mean
  // of v on exit (the Poisson form)
  int cg(hipStream_t s, double* v, double tol, int max_it, bool zero_mean) {
    if (fused) return cg_fused(s, v, tol, max_it, zero_mean);
    SPARC_TRY(reduce(s, n, b, b, RED_DOT, part, sc + 4));
    SPARC_TRY(apply(v, r));
    residual_kernel<<<GRID1(n)>>>(n, b, r);
    copy_kernel<<<GRID1(n)>>>(n, r, p);
    SPARC_TRY(reduce(s, n, r, r, RED_DOT, part, sc + 0));
    double bb = 0, rr = 0;
    SPARC_HIP(hipMemcpyAsync(&bb, sc + 4, 8, hipMemcpyDeviceToHost, s));
    SPARC_HIP(hipStreamSynchronize(s));
    if (bb == 0.0) return SPARC_OK;
    int it = 0;
    for (; it < max_it; ++it) {
      // r.r of the current and of the updated residual alternate between sc[0] and sc[2]
      double* rr0 = sc + ((it & 1) ? 2 : 0);
      double* rr1 = sc + ((it & 1) ? 0 : 2);
      SPARC_TRY(apply(p, Ap));
      SPARC_TRY(reduce(s, n, p, Ap, RED_DOT, part, sc + 1));
      cg_xr_rr_kernel<<<red_blocks(n), 256, 0, s>>>(n, v, r, p, Ap, rr0, sc + 1, part, rr1);
      cg_update_p_kernel<<<GRID1(n)>>>(n, p, r, rr1, rr0);
      // the residual is read back (a host synchronisation) every 8 iterations, from 3/4
      // of the previous solve's count on (warm-started solves take similar counts)
      if (it % 8 == 7 && it >= (3 * last_iters) / 4 - 8) {
        SPARC_HIP(hipMemcpyAsync(&rr, rr1, 8, hipMemcpyDeviceToHost, s));
        SPARC_HIP(hipStreamSynchronize(s));
        if (!std::isfinite(rr)) return fail(SPARC_ENAN, "poisson: non-finite residual");
        if (rr <= tol * tol * bb) break;
      }
    }
    return finish(s, v, it, max_it, zero_mean);
  }

  int finish(hipStream_t s, double* v, int it, int max_it, bool zero_mean) {
    iters_total += it + 1;
    last_iters = it + 1;
    if (it >= max_it) return fail(SPARC_ENOCONV, "poisson: CG did not converge in %d iterations", max_it);
    if (!zero_mean) return check_launch("helmholtz");
    SPARC_TRY(reduce(s, n, v, nullptr, RED_SUM, part, sc + 3));
    sub_mean_kernel<<<GRID1(n)>>>(n, v, sc + 3);
    return check_launch("poisson");
  }

  // The same iteration in two launches per step (cg_iterate): r = b - A v, w = A r and
  // their dot products start it; p and s start at zero.
  int cg_fused(hipStream_t s, double* v, double tol, int max_it, bool zero_mean) {
    CgIter C{r, w, sv, p, v, cs, cpart, cg_blocks(H), 0};
    SPARC_TRY(reduce(s, n, b, b, RED_DOT, part, sc + 4));
    SPARC_TRY(apply(v, r));
    residual_kernel<<<GRID1(n)>>>(n, b, r);
    SPARC_TRY(cg_apply(H, 2.0, shift, C));
    SPARC_TRY(cg_residual_norm(H, C));
    SPARC_HIP(hipMemsetAsync(p, 0, n * 8, s));
    SPARC_HIP(hipMemsetAsync(sv, 0, n * 8, s));
    double bb = 0, rr = 0;
    SPARC_HIP(hipMemcpyAsync(&bb, sc + 4, 8, hipMemcpyDeviceToHost, s));
    SPARC_HIP(hipMemcpyAsync(&rr, cs + 8, 8, hipMemcpyDeviceToHost, s));
    SPARC_HIP(hipStreamSynchronize(s));
    if (bb == 0.0) return SPARC_OK;
    if (!std::isfinite(rr)) return fail(SPARC_ENAN, "poisson: non-finite residual");
    if (rr <= tol * tol * bb) return finish(s, v, -1, max_it, zero_mean);
    int it = 0;
    for (; it < max_it; ++it) {
      C.it = it;
      SPARC_TRY(cg_iterate(H, 2.0, shift, C));
      if (it % 8 == 7 && it >= (3 * last_iters) / 4 - 8) {
        SPARC_TRY(cg_residual_norm(H, C));
        SPARC_HIP(hipMemcpyAsync(&rr, cs + 8, 8, hipMemcpyDeviceToHost, s));
        SPARC_HIP(hipStreamSynchronize(s));
        if (!std::isfinite(rr)) return fail(SPARC_ENAN, "poisson: non-finite residual");
        if (rr <= tol * tol * bb) break;
      }
    }
    return finish(s, v, it, max_it, zero_mean);
  }
};

static double host_scalar(hipStream_t s, const double* d) {
  double h = NAN;
  if (hipMemcpyAsync(&h, d, 8, hipMemcpyDeviceToHost, s) != hipSuccess) return NAN;
  if (hipStreamSynchronize(s) != hipSuccess) return NAN;
  return h;
}

// Superposition of atomic densities (the SCF start of Sec. 4), renormalised so that
// h^3 sum rho = n_elec; part: RED_BLOCKS doubles and a zeroed ticket word, sc: 8 doubles of scratch.
// Synchronous (the renormalisation factor is read back to the host).
static int sad_fill(hipStream_t s, Buffers& B, const sparc_grid* grid, const sparc_atoms* atoms, double n_elec,
                    double* rho_in, double* part, double* sc) {
  const int64_t n = (int64_t)grid->n[0] * grid->n[1] * grid->n[2];
  const double h1 = grid->L[0] / grid->n[0], h2 = grid->L[1] / grid->n[1], h3 = grid->L[2] / grid->n[2];
  const double dV = h1 * h2 * h3;
  std::vector<double> R(3 * atoms->n_atoms), W(atoms->n_atoms), Z(atoms->n_atoms);
  for (int a = 0; a < atoms->n_atoms; ++a) {
    for (int c = 0; c < 3; ++c) R[3 * a + c] = atoms->R[3 * a + c];
    W[a] = atoms->vloc_width[a];
    Z[a] = atoms->Z ? atoms->Z[a] : 2.0;
  }
  double *dR, *dW, *dZ;
  SPARC_TRY(B.alloc(&dR, R.size()));
  SPARC_TRY(B.alloc(&dW, W.size()));
  SPARC_TRY(B.alloc(&dZ, Z.size()));
  SPARC_HIP(hipMemcpyAsync(dR, R.data(), R.size() * 8, hipMemcpyHostToDevice, s));
  SPARC_HIP(hipMemcpyAsync(dW, W.data(), W.size() * 8, hipMemcpyHostToDevice, s));
  SPARC_HIP(hipMemcpyAsync(dZ, Z.data(), Z.size() * 8, hipMemcpyHostToDevice, s));
  sad_kernel<<<GRID1(n)>>>(grid->n[0], grid->n[1], grid->n[2], h1, h2, h3, grid->L[0], grid->L[1], grid->L[2],
                           dirichlet_mask(*grid), atoms->n_atoms, dR, dW, dZ, rho_in);
  SPARC_TRY(check_launch("sad_kernel"));
  SPARC_TRY(reduce(s, n, rho_in, nullptr, RED_SUM, part, sc + 5));
  // rho *= N_e / (dV * sum rho)
  double tot = host_scalar(s, sc + 5);   // synchronises the stream (the host vectors stay valid)
  if (!(tot > 0)) return fail(SPARC_ENAN, "atomic superposition has no charge");
  double f = n_elec / (dV * tot);
  std::vector<double> one{f, 1.0};
  SPARC_HIP(hipMemcpyAsync(sc + 6, one.data(), 16, hipMemcpyHostToDevice, s));
  scale_ratio_kernel<<<GRID1(n)>>>(n, rho_in, sc + 6, sc + 7, 1.0);
  SPARC_HIP(hipStreamSynchronize(s));
  return check_launch("scale_ratio_kernel");
}

}  // namespace sparc

using namespace sparc;

extern "C" int sparc_sad_density(sparc_ctx* ctx, const sparc_grid* grid, const sparc_atoms* atoms, double n_elec,
                                 double* rho_dev) {
  if (!ctx || !grid || !atoms || !rho_dev) return fail(SPARC_EINVAL, "sparc_sad_density: null argument");
  if (atoms->n_atoms < 1 || !atoms->R || !atoms->vloc_width)
    return fail(SPARC_EINVAL, "sparc_sad_density: needs at least one atom with positions and widths");
  for (int s3 = 0; s3 < 3; ++s3)
    if (grid->n[s3] < 1 || !(grid->L[s3] > 0)) return fail(SPARC_ESHAPE, "sparc_sad_density: bad grid");
  if (!(n_elec > 0)) return fail(SPARC_EINVAL, "sparc_sad_density: n_elec must be positive");
  Buffers B;
  double *part, *sc;
  SPARC_TRY(B.alloc(&part, RED_BLOCKS + 2));
  SPARC_TRY(B.alloc(&sc, 16));
  hipStream_t s = ctx->stream;
  SPARC_HIP(hipMemsetAsync(part + RED_BLOCKS, 0, 16, s));
  return sad_fill(s, B, grid, atoms, n_elec, rho_dev, part, sc);
}

extern "C" int sparc_scf_run(sparc_ctx* ctx, const sparc_grid* grid, const sparc_atoms* atoms,
                             const sparc_scf_params* P, sparc_scf_result* res) {
  if (!ctx || !grid || !atoms || !P || !res) return fail(SPARC_EINVAL, "sparc_scf_run: null argument");
  if (dirichlet_mask(*grid) != 0)
    return fail(SPARC_EINVAL, "sparc_scf_run: periodic cells only (its Poisson solve is periodic)");
  if (P->electrostatics != SPARC_ELEC_JELLIUM && P->electrostatics != SPARC_ELEC_PSEUDOCHARGE)
    return fail(SPARC_EINVAL, "sparc_scf_run: electrostatics must be SPARC_ELEC_JELLIUM or SPARC_ELEC_PSEUDOCHARGE");
  const bool psd = P->electrostatics == SPARC_ELEC_PSEUDOCHARGE;
  if (psd && (P->eps_b < 0.0 || P->eps_b >= 1.0)) return fail(SPARC_EINVAL, "sparc_scf_run: eps_b outside [0, 1)");
  if (grid->kpt[0] != 0 || grid->kpt[1] != 0 || grid->kpt[2] != 0)
    return fail(SPARC_EINVAL, "sparc_scf_run: the SCF driver runs at the Gamma point");
  if (P->n_s < 1 || P->degree < 1 || P->max_iter < 1 || P->n_first_passes < 1 || P->lanczos_steps < 2)
    return fail(SPARC_EINVAL, "sparc_scf_run: bad schedule parameters");
  if (!(P->kT > 0) || !(P->mix > 0 && P->mix <= 1) || !(P->tol > 0) || !(P->n_elec > 0))
    return fail(SPARC_EINVAL, "sparc_scf_run: bad kT, mix, tol or n_elec");
  if (P->n_elec > 2.0 * P->n_s) return fail(SPARC_EINVAL, "sparc_scf_run: n_s too small for n_elec");
  if (!P->x0_dev || !P->lanczos_v0_dev) return fail(SPARC_EINVAL, "sparc_scf_run: x0_dev and lanczos_v0_dev needed");
  if (P->filt != SPARC_R64 && P->filt != SPARC_R32) return fail(SPARC_EINVAL, "sparc_scf_run: filt must be R64 or R32");
  if (P->mix_history < 0 || P->mix_history > AMAX) return fail(SPARC_EINVAL, "sparc_scf_run: mix_history outside 0..%d", AMAX);
  if (!(P->kerker_k0 >= 0) || !std::isfinite(P->kerker_k0)) return fail(SPARC_EINVAL, "sparc_scf_run: kerker_k0 must be >= 0");
  if (!res->rho_dev || !res->ritz_dev) return fail(SPARC_EINVAL, "sparc_scf_run: result buffers missing");
  const auto t_start = std::chrono::steady_clock::now();
  hipStream_t s = ctx->stream;
  SPARC_HIP(hipSetDevice(ctx->device));

  sparc_ham* H64 = nullptr;
  sparc_ham* H32 = nullptr;
  SPARC_TRY(sparc_ham_create(ctx, grid, atoms, SPARC_R64, &H64));
  struct HamGuard { sparc_ham* a; sparc_ham** b; ~HamGuard() { sparc_ham_destroy(a); if (*b) sparc_ham_destroy(*b); } } hg{H64, &H32};
  const bool mixed = P->filt == SPARC_R32;
  if (mixed) SPARC_TRY(sparc_ham_create(ctx, grid, atoms, SPARC_R32, &H32));
  const int64_t n = H64->n_d;
  const int ns = P->n_s;
  const double dV = H64->dV;

  Buffers B;
  double *rho_in, *rho_out, *vh, *veff, *edc, *X, *ritz, *occ, *part, *sc;
  double *pb, *pr, *pp, *pAp;
  float* X32 = nullptr;
  SPARC_TRY(B.alloc(&rho_in, n));
  SPARC_TRY(B.alloc(&rho_out, n));
  SPARC_TRY(B.alloc(&vh, n));
  SPARC_TRY(B.alloc(&veff, n));
  SPARC_TRY(B.alloc(&edc, n));
  SPARC_TRY(B.alloc(&X, (size_t)n * ns));
  SPARC_TRY(B.alloc(&ritz, ns));
  SPARC_TRY(B.alloc(&occ, ns));
  SPARC_TRY(B.alloc(&part, RED_BLOCKS + 2));
  SPARC_TRY(B.alloc(&sc, 16));
  SPARC_HIP(hipMemsetAsync(part + RED_BLOCKS, 0, 16, ctx->stream));
  SPARC_TRY(B.alloc(&pb, n));
  SPARC_TRY(B.alloc(&pr, n));
  SPARC_TRY(B.alloc(&pp, n));
  SPARC_TRY(B.alloc(&pAp, n));
  if (mixed) SPARC_TRY(B.alloc(&X32, (size_t)n * ns));
  // Anderson history: previous iterate and residual, ring of m differences
  const int am = P->mix_history;
  double *xprev = nullptr, *fprev = nullptr, *fcur = nullptr, *apairs = nullptr, *agamma = nullptr, *apart = nullptr;
  std::vector<double*> dXh(am, nullptr), dFh(am, nullptr);
  constexpr int ABLK = 256;
  if (am > 0) {
    SPARC_TRY(B.alloc(&xprev, n));
    SPARC_TRY(B.alloc(&fprev, n));
    SPARC_TRY(B.alloc(&fcur, n));
    for (int k = 0; k < am; ++k) {
      SPARC_TRY(B.alloc(&dXh[k], n));
      SPARC_TRY(B.alloc(&dFh[k], n));
    }
    SPARC_TRY(B.alloc(&apairs, (AMAX + 1) * (AMAX + 2) / 2));
    SPARC_TRY(B.alloc(&agamma, AMAX));
    SPARC_TRY(B.alloc(&apart, (size_t)ABLK * (AMAX + 1) * (AMAX + 2) / 2));
  }
  int a_count = 0, a_head = 0;
  // Kerker preconditioning of the mixed residual: f - k0^2 g, (-Lap_h + k0^2) g = f
  const double kk2 = P->kerker_k0 > 0 ? P->kerker_k0 * P->kerker_k0 : 0.0;
  double *kf = nullptr, *kg = nullptr;
  if (kk2 > 0) {
    SPARC_TRY(B.alloc(&kf, n));
    SPARC_TRY(B.alloc(&kg, n));
  }
  size_t wf64 = sparc_workspace_bytes(H64, ns, SPARC_OP_FILTER), wr64 = sparc_workspace_bytes(H64, ns, SPARC_OP_RR);
  size_t wl = sparc_workspace_bytes(H64, P->lanczos_steps, SPARC_OP_LANCZOS);
  size_t wbytes = std::max({wf64, wr64, wl});
  if (mixed)
    wbytes = std::max({wbytes, sparc_workspace_bytes(H32, ns, SPARC_OP_FILTER), sparc_workspace_bytes(H32, ns, SPARC_OP_RR)});
  char* work = nullptr;
  SPARC_TRY(B.alloc(&work, wbytes));

  // start density and orbitals
  if (P->rho_init_dev) {
    SPARC_HIP(hipMemcpyAsync(rho_in, P->rho_init_dev, n * 8, hipMemcpyDeviceToDevice, s));
  } else {
    SPARC_TRY(sad_fill(s, B, grid, atoms, P->n_elec, rho_in, part, sc));
  }
  SPARC_HIP(hipMemcpyAsync(X, P->x0_dev, (size_t)n * ns * 8, hipMemcpyDeviceToDevice, s));
  SPARC_HIP(hipMemsetAsync(vh, 0, n * 8, s));
  double* vloc;
  SPARC_TRY(B.alloc(&vloc, n));
  SPARC_TRY(sparc_ham_get_vloc(H64, vloc));

  // pseudocharge electrostatics: b, E_self^h and E_c^h once; the electrons see phi, not V_loc
  double *bpsd = nullptr, *rhob = nullptr;
  double e_psd = 0.0;
  if (psd) {
    std::vector<int32_t> boxes(6 * (size_t)atoms->n_atoms);
    SPARC_TRY(sparc_psd_boxes(ctx, grid, atoms, P->eps_b > 0 ? P->eps_b : 1e-8, boxes.data()));
    double *bref, *vc;
    SPARC_TRY(B.alloc(&bpsd, n));
    SPARC_TRY(B.alloc(&bref, n));
    SPARC_TRY(B.alloc(&vc, n));
    SPARC_TRY(B.alloc(&rhob, n));
    double en[3];
    SPARC_TRY(sparc_pseudocharge(ctx, grid, atoms, boxes.data(), bpsd, bref, vc, en));
    e_psd = en[2] - en[0];
    SPARC_HIP(hipMemsetAsync(vloc, 0, n * 8, s));
  }

  Poisson PS{H64, n, pb, pr, pp, pAp, part, sc};
  if (cg_point_form(H64)) {
    PS.fused = true;
    SPARC_TRY(B.alloc(&PS.w, n));
    SPARC_TRY(B.alloc(&PS.sv, n));
    SPARC_TRY(B.alloc(&PS.cs, 12));
    SPARC_TRY(B.alloc(&PS.cpart, 2 * kCgBlocks));
  }
  const double ptol = P->poisson_tol > 0 ? P->poisson_tol : 1e-10;
  // phi (or V_H) of the current input density, warm-started from the previous one; the
  // CG tolerance follows the SCF: a thousandth of the last density residual, at most
  // 1e-4 and at least poisson_tol, which the final iterations reach
  auto solve_potential = [&](double res) -> int {
    const double tol_now = std::max(ptol, std::min(1e-4, 1e-3 * res));
    if (!psd) return PS.solve(s, rho_in, vh, tol_now, 20000);
    add_kernel<<<GRID1(n)>>>(n, rho_in, bpsd, rhob);
    SPARC_TRY(check_launch("add_kernel"));
    return PS.solve(s, rhob, vh, tol_now, 20000);
  };
  SPARC_TRY(solve_potential(1.0));

  double lmin = 0, lmax = 0, lcut = 0;
  bool have_ritz = false;
  bool use32 = mixed;
  if (mixed) {
    d2f_block_kernel<<<GRID1((int64_t)n * ns)>>>((int64_t)n * ns, X, X32);
    SPARC_TRY(check_launch("d2f_block_kernel"));
  }
  double F = 0, mu = 0, err = 1, prev_err = 1e300, lcut_next = 0;
  int it = 1;
  int converged = 0;
  for (; it <= P->max_iter; ++it) {
    xc_veff_kernel<<<GRID1(n)>>>(n, rho_in, vloc, vh, bpsd, veff, edc);
    SPARC_TRY(check_launch("xc_veff_kernel"));
    SPARC_TRY(sparc_ham_set_veff(H64, veff));
    if (mixed) SPARC_TRY(sparc_ham_set_veff(H32, veff));
    if (it == 1) SPARC_TRY(lanczos_bounds(H64, P->lanczos_v0_dev, P->lanczos_steps, work, wbytes, &lmin, &lmax));
    const int passes = (it == 1) ? P->n_first_passes : 1;
    for (int ps = 0; ps < passes; ++ps) {
      // the largest Ritz value of the previous pass (read with the last iteration's
      // energy after the first iteration's passes)
      lcut = !have_ritz ? 0.5 * (lmin + lmax) : (it > 1 && ps == 0) ? lcut_next : host_scalar(s, ritz + ns - 1);
      if (use32) {
        SPARC_TRY(chebyshev_filter(H32, X32, n, ns, P->degree, lcut, lmax, work, wbytes));
        SPARC_TRY(rayleigh_ritz(H32, X32, n, ns, P->rr, ritz, work, wbytes, nullptr));
      } else {
        SPARC_TRY(chebyshev_filter(H64, X, n, ns, P->degree, lcut, lmax, work, wbytes));
        SPARC_TRY(rayleigh_ritz(H64, X, n, ns, SPARC_GEMM_NATIVE, ritz, work, wbytes, nullptr));
      }
      have_ritz = true;
    }
    const double wk = 1.0;
    SPARC_TRY(sparc_fermi(ctx, 1, ns, ritz, &wk, P->n_elec, P->kT, occ, &mu));
    // Harris-Foulkes free energy at rho_in, the output density and its residual; the
    // energy terms, the residual norms and the next filter cut come back in one
    // synchronisation
    band_entropy_kernel<<<1, 256, 0, s>>>(ns, ritz, occ, P->kT, sc + 8);
    SPARC_TRY(reduce(s, n, edc, nullptr, RED_SUM, part, sc + 10));
    const void* xs[1] = {use32 ? (const void*)X32 : (const void*)X};
    const int64_t lds[1] = {n};
    SPARC_TRY(density_from_orbitals(ctx, 1, xs, lds, ns, use32 ? SPARC_R32 : SPARC_R64, occ, n, dV, rho_out));
    SPARC_TRY(reduce(s, n, rho_out, rho_in, RED_DIFF2, part, sc + 11));
    SPARC_TRY(reduce(s, n, rho_in, rho_in, RED_DOT, part, sc + 12));
    double hv[5];
    SPARC_HIP(hipMemcpyAsync(hv, sc + 8, 5 * 8, hipMemcpyDeviceToHost, s));
    SPARC_HIP(hipMemcpyAsync(&lcut_next, ritz + ns - 1, 8, hipMemcpyDeviceToHost, s));
    SPARC_HIP(hipStreamSynchronize(s));
    F = hv[0] + dV * hv[2] + hv[1] + e_psd;
    if (!std::isfinite(F)) return fail(SPARC_ENAN, "sparc_scf_run: non-finite energy at iteration %d", it);
    err = std::sqrt(hv[3] / hv[4]);
    if (res->history) {
      res->history[3 * (it - 1)] = F;
      res->history[3 * (it - 1) + 1] = err;
      res->history[3 * (it - 1) + 2] =
          std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    }
    if (!std::isfinite(err)) return fail(SPARC_ENAN, "sparc_scf_run: non-finite density residual");
    if (use32 && P->final_fp64_pass && (err < 1e-4 || (it > 2 && err > 0.8 * prev_err))) {
      // hand the FP32 orbitals over to FP64 passes; this iterate is not accepted as converged
      f2d_block_kernel<<<GRID1((int64_t)n * ns)>>>((int64_t)n * ns, X32, X);
      SPARC_TRY(check_launch("f2d_block_kernel"));
      use32 = false;
    } else if (err < P->tol) {
      converged = 1;
      break;
    }
    prev_err = err;
    // rho_in += mix P(f) with the Helmholtz solve of the Kerker form (f in kf)
    auto kerker_mix = [&]() -> int {
      SPARC_TRY(PS.solve_helmholtz(s, kf, kg, kk2, 1e-10, 20000));
      kerker_mix_kernel<<<GRID1(n)>>>(n, rho_in, kf, kg, kk2, P->mix);
      return check_launch("kerker_mix_kernel");
    };
    if (am == 0) {
      if (kk2 > 0) {
        diff_kernel<<<GRID1(n)>>>(n, rho_out, rho_in, kf);
        SPARC_TRY(kerker_mix());
      } else {
        mix_kernel<<<GRID1(n)>>>(n, rho_in, rho_out, P->mix);
      }
    } else {
      diff_kernel<<<GRID1(n)>>>(n, rho_out, rho_in, fcur);
      if (it > 1) {  // new differences into the ring
        diff_kernel<<<GRID1(n)>>>(n, rho_in, xprev, dXh[a_head]);
        diff_kernel<<<GRID1(n)>>>(n, fcur, fprev, dFh[a_head]);
        a_head = (a_head + 1) % am;
        a_count = std::min(a_count + 1, am);
      }
      SPARC_HIP(hipMemcpyAsync(xprev, rho_in, n * 8, hipMemcpyDeviceToDevice, s));
      SPARC_HIP(hipMemcpyAsync(fprev, fcur, n * 8, hipMemcpyDeviceToDevice, s));
      if (a_count == 0) {
        if (kk2 > 0) {
          SPARC_HIP(hipMemcpyAsync(kf, fcur, n * 8, hipMemcpyDeviceToDevice, s));
          SPARC_TRY(kerker_mix());
        } else {
          mix_kernel<<<GRID1(n)>>>(n, rho_in, rho_out, P->mix);
        }
      } else {
        VecSet vs;
        GammaSet gs;
        for (int k = 0; k < a_count; ++k) {
          vs.v[k] = dFh[k];
          gs.dx[k] = dXh[k];
          gs.df[k] = dFh[k];
        }
        vs.v[a_count] = fcur;
        launch_multi_dot(s, ABLK, n, a_count, vs, apart);
        anderson_gamma_kernel<<<1, 256, 0, s>>>(ABLK, a_count, apart, apairs, agamma);
        anderson_update_kernel<<<GRID1(n)>>>(n, a_count, gs, agamma, fcur, P->mix, rho_in, kk2 > 0 ? kf : nullptr);
        if (kk2 > 0) SPARC_TRY(kerker_mix());
      }
    }
    SPARC_TRY(check_launch("density mixing"));
    SPARC_TRY(solve_potential(err));
  }
  res->energy = F;
  res->mu = mu;
  res->iterations = std::min(it, P->max_iter);
  res->converged = converged;
  SPARC_HIP(hipMemcpyAsync(res->rho_dev, rho_in, n * 8, hipMemcpyDeviceToDevice, s));
  SPARC_HIP(hipMemcpyAsync(res->ritz_dev, ritz, ns * 8, hipMemcpyDeviceToDevice, s));
  if (res->phi_dev) SPARC_HIP(hipMemcpyAsync(res->phi_dev, vh, n * 8, hipMemcpyDeviceToDevice, s));
  if (res->x_dev) {
    if (use32) f2d_block_kernel<<<GRID1((int64_t)n * ns)>>>((int64_t)n * ns, X32, X);
    SPARC_HIP(hipMemcpyAsync(res->x_dev, X, (size_t)n * ns * 8, hipMemcpyDeviceToDevice, s));
  }
  SPARC_HIP(hipStreamSynchronize(s));
  if (!converged) return fail(SPARC_ENOCONV, "sparc_scf_run: not converged in %d iterations (residual %.3e)", P->max_iter, err);
  return SPARC_OK;
}
