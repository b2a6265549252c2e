// Atomic forces f_J = -dF/dR_J (Sec. 2, atomic forces; Sec. 3.6, discrete local and
// non-local components, Algorithms 2 and 3) for the synthetic cell, whose Gaussian
// wells are an external local potential under jellium electrostatics.
//
//  local:     f_J,loc = h1h2h3 sum_g rho_g sum_L D_J e^{-r^2/(2 w_J^2)} (x_g - R_J - L) / w_J^2
//             over the images L with r = |x_g - R_J - L| <= 10 w_J (the exact derivative of
//             the trapezoidal local energy h1h2h3 sum_g rho_g V_loc(x_g)).  One work-group per
//             (atom, z-chunk of the atom's box of unwrapped nodes); partial sums reduced in a
//             fixed order.
//  non-local: f_J,nloc = -4 sum_n occ_n sum_p gamma_p Re[ conj(alpha_pn) beta_pn ] / h1h2h3
//             with alpha = h1h2h3 sum_t conj(chi~_p(t)) u_n(t) (the projections of H X) and
//             beta = h1h2h3 sum_t conj(chi~_p(t)) (grad_h u_n)(t): the paper's Y W with the
//             derivative on the orbitals, for Euclidean-orthonormal orbitals.  Regrouped per
//             support node t as -4 sum_t sum_n occ_n Re[c_n(t) (grad_h u_n)(t)] with
//             c_n(t) = sum_p gamma_p conj(alpha_pn chi~_p(t)), so a thread keeps three sums.
//             One work-group per (atom, block of orbitals); the FD gradient (Sec. 3.1) is
//             evaluated on the fly at the support nodes with the Bloch-periodic index map
//             (zero past a Dirichlet face).
//             Orbitals with zero occupation are skipped.
#include <algorithm>
#include <cmath>

#include "devmath.hpp"

namespace sparc {

// ---------------------------------------------------------------- block reduction
// sum of three per-thread values over a 256-thread work-group (fixed order)
__device__ __forceinline__ void block_sum3(double v[3], double* out) {
  __shared__ double red[3][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double s = wave_sum(v[d]);
    if (lane == 0) red[d][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int d = threadIdx.x;
    out[d] = ((red[d][0] + red[d][1]) + red[d][2]) + red[d][3];
  }
}

__device__ __forceinline__ int64_t floordiv_l(int64_t a, int64_t b) {
  int64_t q = a / b;
  return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}

// ---------------------------------------------------------------- local component
__global__ __launch_bounds__(256) void force_local_kernel(int n1, int n2, int n3, double h1, double h2, double h3,
                                                          int dmask, const double* __restrict__ R,
                                                          const double* __restrict__ D,
                                                          const double* __restrict__ W,
                                                          const double* __restrict__ rho, double* __restrict__ part) {
  const int J = blockIdx.x, chunk = blockIdx.y;
  const double Rx = R[3 * J], Ry = R[3 * J + 1], Rz = R[3 * J + 2];
  const double w = W[J], rc = 10.0 * w, inv2w2 = 1.0 / (2.0 * w * w), amp = D[J] / (w * w);
  // box of unwrapped nodes within rc of the centre (each is one image point)
  int64_t i0 = (int64_t)ceil((Rx - rc) / h1), i1 = (int64_t)floor((Rx + rc) / h1);
  int64_t j0 = (int64_t)ceil((Ry - rc) / h2), j1 = (int64_t)floor((Ry + rc) / h2);
  int64_t k0 = (int64_t)ceil((Rz - rc) / h3), k1 = (int64_t)floor((Rz + rc) / h3);
  // no images across a Dirichlet direction: keep the nodes inside the grid
  if (dmask & 1) { i0 = max(i0, (int64_t)0); i1 = min(i1, (int64_t)n1 - 1); }
  if (dmask & 2) { j0 = max(j0, (int64_t)0); j1 = min(j1, (int64_t)n2 - 1); }
  if (dmask & 4) { k0 = max(k0, (int64_t)0); k1 = min(k1, (int64_t)n3 - 1); }
  const int64_t nx = max(i1 - i0 + 1, (int64_t)0), ny = max(j1 - j0 + 1, (int64_t)0),
                nz = max(k1 - k0 + 1, (int64_t)0);
  // this chunk's z planes
  const int64_t zc = (nz + gridDim.y - 1) / gridDim.y;
  const int64_t kb = k0 + chunk * zc, ke = std::min(k1 + 1, kb + zc);
  const int64_t total = (ke > kb) ? nx * ny * (ke - kb) : 0;
  double f[3] = {0.0, 0.0, 0.0};
  for (int64_t q = threadIdx.x; q < total; q += blockDim.x) {
    const int64_t i = i0 + q % nx, j = j0 + (q / nx) % ny, k = kb + q / (nx * ny);
    const double dx = i * h1 - Rx, dy = j * h2 - Ry, dz = k * h3 - Rz;
    const double r2 = dx * dx + dy * dy + dz * dz;
    if (r2 > rc * rc) continue;
    const int64_t gi = i - floordiv_l(i, n1) * n1, gj = j - floordiv_l(j, n2) * n2, gk = k - floordiv_l(k, n3) * n3;
    const double s = rho[gi + n1 * (gj + (int64_t)n2 * gk)] * amp * exp(-r2 * inv2w2);
    f[0] = fma(s, dx, f[0]);
    f[1] = fma(s, dy, f[1]);
    f[2] = fma(s, dz, f[2]);
  }
  block_sum3(f, part + ((int64_t)J * gridDim.y + chunk) * 3);
}

__global__ void force_local_reduce(int n_atoms, int n_chunks, double dV, const double* __restrict__ part,
                                   double* __restrict__ F) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 3 * n_atoms) return;
  const int J = q / 3, d = q % 3;
  double s = 0.0;
  for (int c = 0; c < n_chunks; ++c) s += part[((int64_t)J * n_chunks + c) * 3 + d];
  F[q] += dV * s;
}

// ---------------------------------------------------------------- non-local component
struct GradArgs {
  int n1, n2, n3, no, dmask;
  double w[3][8];    // w~_p / h_s
  double kl[3];      // k_s L_s
};

template <typename E>
__device__ __forceinline__ E bloch_load(const E* __restrict__ xn, int64_t idx, int wraps, double kl) {
  E v = xn[idx];
  if constexpr (elem<E>::is_cplx) {
    if (wraps != 0 && kl != 0.0) {
      double s, c;
      sincos(kl * wraps, &s, &c);
      v = rot(v, (typename elem<E>::real)c, (typename elem<E>::real)s);
    }
  }
  return v;
}

__device__ __forceinline__ double re_mul(double a, double b) { return a * b; }
__device__ __forceinline__ double re_mul(float a, float b) { return (double)a * b; }
__device__ __forceinline__ double re_mul(cd a, cd b) { return a.re * b.re - a.im * b.im; }
__device__ __forceinline__ double re_mul(cf a, cf b) { return (double)a.re * b.re - (double)a.im * b.im; }
__device__ __forceinline__ double cj(double a) { return a; }
__device__ __forceinline__ float cj(float a) { return a; }
__device__ __forceinline__ cd cj(cd a) { return {a.re, -a.im}; }
__device__ __forceinline__ cf cj(cf a) { return {a.re, -a.im}; }

template <typename E, int MAXP, int NB>
__global__ __launch_bounds__(256) void force_nl_kernel(const E* __restrict__ x, int64_t ldx, int n_s,
                                                       const int32_t* __restrict__ sup_ptr,
                                                       const int32_t* __restrict__ sup_idx,
                                                       const int32_t* __restrict__ atom_pbeg,
                                                       const int64_t* __restrict__ proj_voff,
                                                       const E* __restrict__ pval,
                                                       const typename elem<E>::real* __restrict__ gamma,
                                                       const E* __restrict__ alpha, int lda,
                                                       const double* __restrict__ occ, GradArgs G,
                                                       double* __restrict__ part) {
  typedef typename elem<E>::real R;
  const int a = blockIdx.x;
  const int nb0 = blockIdx.y * NB;
  const int t0 = sup_ptr[a], t1 = sup_ptr[a + 1];
  const int pb = atom_pbeg[a], np = atom_pbeg[a + 1] - pb;
  const int n1 = G.n1, n2 = G.n2, n3 = G.n3;
  const int64_t plane = (int64_t)n1 * n2;
  double f[3] = {0.0, 0.0, 0.0};
  // occupations and projections of this block (uniform over the work-group)
  double on[NB];
  bool any = false;
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    on[j] = (nb0 + j < n_s) ? occ[nb0 + j] : 0.0;
    any |= (on[j] != 0.0);
  }
  if (any) {
    int64_t voff[MAXP];
    R gam[MAXP];
#pragma unroll
    for (int p = 0; p < MAXP; ++p) {
      voff[p] = (p < np) ? proj_voff[pb + p] : 0;
      gam[p] = (p < np) ? gamma[pb + p] : (R)0;
    }
    for (int t = t0 + (int)threadIdx.x; t < t1; t += blockDim.x) {
      const int g = sup_idx[t];
      const int i = g % n1, jy = (g / n1) % n2, k = g / (int)plane;
      // c_n(t) = sum_p gamma_p conj(alpha_pn chi~_p(t))
      E c[NB];
#pragma unroll
      for (int j = 0; j < NB; ++j) c[j] = zero<E>();
#pragma unroll
      for (int p = 0; p < MAXP; ++p) {
        if (p < np) {
          const E chi = pval[voff[p] + (t - t0)];
          const E* ap = alpha + (int64_t)(pb + p) * lda + nb0;
#pragma unroll
          for (int j = 0; j < NB; ++j)
            if (on[j] != 0.0) c[j] = fmar(c[j], gam[p], cj(ap[j] * chi));
        }
      }
      // gradient components, one direction at a time
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        E gs[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) gs[j] = zero<E>();
        const int pos = (d == 0) ? i : (d == 1) ? jy : k;
        const int nn = (d == 0) ? n1 : (d == 1) ? n2 : n3;
        const int64_t stride = (d == 0) ? 1 : (d == 1) ? n1 : plane;
        const int64_t base = g - (int64_t)pos * stride;
        for (int p = 1; p <= G.no; ++p) {
          const int ip = pos + p, im = pos - p;
          const int wp = floordiv_i(ip, nn), wm = floordiv_i(im, nn);
          const int64_t op = base + (int64_t)(ip - wp * nn) * stride, om = base + (int64_t)(im - wm * nn) * stride;
          const R wt = (R)G.w[d][p - 1];
          // zero Dirichlet conditions: values past the face are zero
          const bool zp = ((G.dmask >> d) & 1) && wp != 0, zm = ((G.dmask >> d) & 1) && wm != 0;
#pragma unroll
          for (int j = 0; j < NB; ++j) {
            if (on[j] != 0.0) {
              const E* xn = x + (int64_t)(nb0 + j) * ldx;
              E vp = bloch_load(xn, op, wp, G.kl[d]);
              E vm = bloch_load(xn, om, wm, G.kl[d]);
              if (zp) vp = zero<E>();
              if (zm) vm = zero<E>();
              gs[j] = fmar(gs[j], wt, vp - vm);
            }
          }
        }
#pragma unroll
        for (int j = 0; j < NB; ++j)
          if (on[j] != 0.0) f[d] = fma(on[j], re_mul(c[j], gs[j]), f[d]);
      }
    }
  }
  block_sum3(f, part + ((int64_t)a * gridDim.y + blockIdx.y) * 3);
}

__global__ void force_nl_reduce(int n_atoms_nl, int n_blk, const double* __restrict__ part,
                                const int32_t* __restrict__ nl_atom, double* __restrict__ F) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= 3 * n_atoms_nl) return;
  const int a = q / 3, d = q % 3;
  double s = 0.0;
  for (int b = 0; b < n_blk; ++b) s += part[((int64_t)a * n_blk + b) * 3 + d];
  F[3 * nl_atom[a] + d] += -4.0 * s;
}

constexpr int kForceNB = 8;   // orbitals per work-group of the non-local force

size_t force_nl_part_bytes(const sparc_ham* H, int32_t n_s) {
  const int nblk = (n_s + kForceNB - 1) / kForceNB;
  return (size_t)std::max(H->n_atoms_nl, 1) * nblk * 3 * sizeof(double);
}

template <typename E>
static int force_nl_t(sparc_ham* H, const void* X, int64_t ldx, int32_t n_s, const double* occ, double* F,
                      void* alpha, double* part) {
  hipStream_t st = H->ctx->stream;
  SPARC_TRY(nl_project(H, X, ldx, n_s, alpha));
  GradArgs G;
  G.n1 = H->grid.n[0];
  G.n2 = H->grid.n[1];
  G.n3 = H->grid.n[2];
  G.no = H->grid.n_o;
  G.dmask = dirichlet_mask(H->grid);
  for (int s = 0; s < 3; ++s) {
    for (int p = 0; p < 8; ++p) G.w[s][p] = H->gtap[s][p];
    G.kl[s] = H->grid.kpt[s] * H->grid.L[s];
  }
  const int nblk = (n_s + kForceNB - 1) / kForceNB;
  if (nblk > 65535) return fail(SPARC_ESHAPE, "sparc_forces_nonlocal: n_s=%d too large", n_s);
  dim3 grid(H->n_atoms_nl, nblk);
  typedef typename elem<E>::real R;
  if (H->max_proj_per_atom <= 1)
    force_nl_kernel<E, 1, kForceNB><<<grid, 256, 0, st>>>((const E*)X, ldx, n_s, H->sup_ptr, H->sup_idx,
                                                          H->atom_pbeg, H->proj_voff, (const E*)H->pval,
                                                          (const R*)H->gamma_d, (const E*)alpha, alpha_ld(n_s), occ,
                                                          G, part);
  else if (H->max_proj_per_atom <= 4)
    force_nl_kernel<E, 4, kForceNB><<<grid, 256, 0, st>>>((const E*)X, ldx, n_s, H->sup_ptr, H->sup_idx,
                                                          H->atom_pbeg, H->proj_voff, (const E*)H->pval,
                                                          (const R*)H->gamma_d, (const E*)alpha, alpha_ld(n_s), occ,
                                                          G, part);
  else
    return fail(SPARC_EINVAL, "sparc_forces_nonlocal: more than 4 projector functions on one atom");
  SPARC_TRY(check_launch("force_nl_kernel"));
  const int nq = 3 * H->n_atoms_nl;
  force_nl_reduce<<<(nq + 255) / 256, 256, 0, st>>>(H->n_atoms_nl, nblk, part, H->nl_atom, F);
  return check_launch("force_nl_reduce");
}

}  // namespace sparc

using namespace sparc;

extern "C" {

int sparc_forces_local(sparc_ham* H, const double* rho_dev, double* F_dev) {
  if (!H || !rho_dev || !F_dev) return fail(SPARC_EINVAL, "sparc_forces_local: null argument");
  if (H->n_atoms == 0) return SPARC_OK;
  hipStream_t st = H->ctx->stream;
  const int t = timer_begin(H->ctx, "force_local");
  force_local_kernel<<<dim3(H->n_atoms, kForceChunks), 256, 0, st>>>(
      H->grid.n[0], H->grid.n[1], H->grid.n[2], H->h[0], H->h[1], H->h[2], dirichlet_mask(H->grid), H->atom_R,
      H->atom_D, H->atom_W, rho_dev, H->force_part);
  timer_end(H->ctx, t);
  SPARC_TRY(check_launch("force_local_kernel"));
  const int nq = 3 * H->n_atoms;
  force_local_reduce<<<(nq + 255) / 256, 256, 0, st>>>(H->n_atoms, kForceChunks, H->dV, H->force_part, F_dev);
  return check_launch("force_local_reduce");
}

int sparc_forces_nonlocal(sparc_ham* H, const void* X, int64_t ldx, int32_t n_s, const double* occ_dev,
                          double* F_dev, void* work, size_t work_bytes) {
  if (!H || !X || !occ_dev || !F_dev) return fail(SPARC_EINVAL, "sparc_forces_nonlocal: null argument");
  if (n_s < 1) return fail(SPARC_ESHAPE, "sparc_forces_nonlocal: n_s=%d < 1", n_s);
  if (ldx < H->n_d) return fail(SPARC_ESHAPE, "sparc_forces_nonlocal: ld=%lld < N_d=%lld", (long long)ldx,
                                (long long)H->n_d);
  if (H->n_proj == 0) return SPARC_OK;
  const size_t need = sparc_workspace_bytes(H, n_s, SPARC_OP_FORCES);
  if (!work || work_bytes < need)
    return fail(SPARC_ENOMEM, "sparc_forces_nonlocal: workspace %zu < %zu bytes", work_bytes, need);
  const size_t ab = ((alpha_bytes(H, n_s) + 255) / 256) * 256;
  void* alpha = work;
  double* part = (double*)((char*)work + ab);
  const int t = timer_begin(H->ctx, "force_nl");
  int rc = SPARC_EINVAL;
  switch (H->dtype) {
    case SPARC_R64: rc = force_nl_t<double>(H, X, ldx, n_s, occ_dev, F_dev, alpha, part); break;
    case SPARC_R32: rc = force_nl_t<float>(H, X, ldx, n_s, occ_dev, F_dev, alpha, part); break;
    case SPARC_C128: rc = force_nl_t<cd>(H, X, ldx, n_s, occ_dev, F_dev, alpha, part); break;
    case SPARC_C64: rc = force_nl_t<cf>(H, X, ldx, n_s, occ_dev, F_dev, alpha, part); break;
  }
  timer_end(H->ctx, t);
  return rc;
}

}  // extern "C"
