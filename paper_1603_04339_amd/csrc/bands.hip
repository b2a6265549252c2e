// Band structure at the electronic ground state (Sec. 4: at every k-point of a path the
// CheFSI steps of Sec. 3.4 are repeated until convergence with the ground-state
// potential fixed), and the density of states D(E) = 2 sum_n fint_BZ delta(lambda_n(k) - E) dk
// with a Gaussian-broadened delta.
//
// All k-points advance together: one batched filter plan (one stencil launch per
// recurrence step over every k, captured in a HIP graph) and one batched Rayleigh-Ritz
// per pass.  Filter bounds per k as in the SCF: lambda_max from Lanczos, lambda_cut the
// midpoint of the Lanczos interval for the first pass and the largest Ritz value of the
// previous pass afterwards.  A k-point is converged once the lowest n_bands Ritz values
// move by less than tol between two passes.
#include <algorithm>
#include <cmath>
#include <vector>

#include "devmath.hpp"

using namespace sparc;

namespace {

struct DevBufs {
  std::vector<void*> p;
  ~DevBufs() {
    for (void* q : p) hipFree(q);
  }
  int alloc(void** q, size_t bytes) {
    *q = nullptr;
    if (hipMalloc(q, std::max<size_t>(bytes, 1)) != hipSuccess)
      return fail(SPARC_ENOMEM, "sparc_band_structure: device allocation of %zu bytes failed", bytes);
    p.push_back(*q);
    return SPARC_OK;
  }
};

struct Hams {
  std::vector<sparc_ham*> h;
  ~Hams() {
    for (sparc_ham* q : h) sparc_ham_destroy(q);
  }
};

struct PlanGuard {
  sparc_filter_plan* p = nullptr;
  ~PlanGuard() { sparc_filter_plan_destroy(p); }
};

}  // namespace

extern "C" {

int sparc_band_structure(sparc_ctx* ctx, const sparc_grid* grid, const sparc_atoms* atoms, const double* veff_dev,
                         int32_t n_k, const double* kpts, void* const* X, int32_t n_s, int32_t n_bands,
                         int32_t degree, int32_t max_passes, double tol, int32_t use_graph, double* eig_out,
                         int32_t* passes_out) {
  if (!ctx || !grid || !atoms || !veff_dev || !kpts || !X || !eig_out || !passes_out)
    return fail(SPARC_EINVAL, "sparc_band_structure: null argument");
  if (n_k < 1) return fail(SPARC_EINVAL, "sparc_band_structure: n_k=%d < 1", n_k);
  if (n_s < 1 || n_bands < 1 || n_bands > n_s)
    return fail(SPARC_ESHAPE, "sparc_band_structure: need 1 <= n_bands (%d) <= n_s (%d)", n_bands, n_s);
  if (degree < 1 || max_passes < 1 || !(tol > 0.0))
    return fail(SPARC_EINVAL, "sparc_band_structure: need degree >= 1, max_passes >= 1, tol > 0");
  for (int b = 0; b < n_k; ++b)
    if (!X[b]) return fail(SPARC_EINVAL, "sparc_band_structure: X[%d] is NULL", b);

  // one complex Hamiltonian per k, all with the given potential
  Hams hs;
  for (int b = 0; b < n_k; ++b) {
    sparc_grid g = *grid;
    for (int s = 0; s < 3; ++s) g.kpt[s] = kpts[3 * b + s];
    sparc_ham* h = nullptr;
    SPARC_TRY(sparc_ham_create(ctx, &g, atoms, SPARC_C128, &h));
    hs.h.push_back(h);
    SPARC_TRY(sparc_ham_set_veff(h, veff_dev));
  }
  const int64_t nd = hs.h[0]->n_d;
  std::vector<int64_t> ld(n_k, nd);
  std::vector<int32_t> ns(n_k, n_s), deg(n_k, degree);

  DevBufs bufs;
  // filter bounds per k: Lanczos from the first column of the start block
  const int lz_steps = 20;
  void* lzw = nullptr;
  const size_t lz_bytes = sparc_workspace_bytes(hs.h[0], lz_steps, SPARC_OP_LANCZOS);
  SPARC_TRY(bufs.alloc(&lzw, lz_bytes));
  std::vector<double> lmin(n_k), lmax(n_k), lcut(n_k);
  for (int b = 0; b < n_k; ++b) {
    SPARC_TRY(lanczos_bounds(hs.h[b], X[b], lz_steps, lzw, lz_bytes, &lmin[b], &lmax[b]));
    lcut[b] = 0.5 * (lmin[b] + lmax[b]);
  }

  // batched filter plan and Rayleigh-Ritz workspace
  const size_t pw_bytes = sparc_filter_plan_workspace_bytes(n_k, hs.h.data(), ns.data(), deg.data());
  void* pw = nullptr;
  SPARC_TRY(bufs.alloc(&pw, pw_bytes));
  PlanGuard plan;
  SPARC_TRY(sparc_filter_plan_create(ctx, n_k, hs.h.data(), X, ld.data(), ns.data(), deg.data(), use_graph ? 1 : 0,
                                     pw, pw_bytes, &plan.p));
  const size_t rw_bytes = sparc_rr_batched_workspace_bytes(n_k, hs.h.data(), ns.data());
  void* rw = nullptr;
  SPARC_TRY(bufs.alloc(&rw, rw_bytes));
  void* ritz_all = nullptr;
  SPARC_TRY(bufs.alloc(&ritz_all, (size_t)n_k * n_s * sizeof(double)));
  std::vector<double*> ritz(n_k);
  for (int b = 0; b < n_k; ++b) ritz[b] = (double*)ritz_all + (size_t)b * n_s;

  std::vector<double> cur((size_t)n_k * n_s), prev((size_t)n_k * n_s, 0.0);
  std::vector<int> done(n_k, 0);
  int n_done = 0;
  for (int pass = 1; pass <= max_passes && n_done < n_k; ++pass) {
    SPARC_TRY(sparc_filter_plan_run(plan.p, lcut.data(), lmax.data()));
    SPARC_TRY(rayleigh_ritz_batched(ctx, n_k, hs.h.data(), X, ld.data(), ns.data(), SPARC_GEMM_NATIVE, ritz.data(),
                                    rw, rw_bytes));
    SPARC_HIP(hipMemcpyAsync(cur.data(), ritz_all, cur.size() * sizeof(double), hipMemcpyDeviceToHost,
                             ctx->stream));
    SPARC_HIP(hipStreamSynchronize(ctx->stream));
    for (int b = 0; b < n_k; ++b) {
      const double* c = &cur[(size_t)b * n_s];
      const double* p = &prev[(size_t)b * n_s];
      for (int i = 0; i < n_s; ++i)
        if (!std::isfinite(c[i])) return fail(SPARC_ENAN, "sparc_band_structure: non-finite Ritz value at k %d", b);
      if (!done[b] && pass > 1) {
        double d = 0.0;
        for (int i = 0; i < n_bands; ++i) d = std::max(d, std::fabs(c[i] - p[i]));
        if (d < tol) {
          done[b] = 1;
          passes_out[b] = pass;
          ++n_done;
        }
      }
      lcut[b] = c[n_s - 1];
    }
    std::swap(cur, prev);
  }
  // prev holds the last pass
  for (int b = 0; b < n_k; ++b) {
    for (int i = 0; i < n_bands; ++i) eig_out[(size_t)b * n_bands + i] = prev[(size_t)b * n_s + i];
    if (!done[b]) passes_out[b] = max_passes;
  }
  if (n_done < n_k)
    return fail(SPARC_ENOCONV, "sparc_band_structure: %d of %d k-points not converged in %d passes", n_k - n_done,
                n_k, max_passes);
  return SPARC_OK;
}

int sparc_dos(int32_t n_k, int32_t n_bands, const double* eig, const double* wk, int32_t n_e, const double* energies,
              double sigma, double* dos_out) {
  if (!eig || !wk || !energies || !dos_out) return fail(SPARC_EINVAL, "sparc_dos: null argument");
  if (n_k < 1 || n_bands < 1 || n_e < 0) return fail(SPARC_ESHAPE, "sparc_dos: bad sizes");
  if (!(sigma > 0.0)) return fail(SPARC_EINVAL, "sparc_dos: sigma must be positive");
  const double norm = 1.0 / (sigma * std::sqrt(2.0 * M_PI));
  for (int e = 0; e < n_e; ++e) {
    double acc = 0.0;
    for (int b = 0; b < n_k; ++b) {
      double s = 0.0;
      for (int i = 0; i < n_bands; ++i) {
        const double t = (energies[e] - eig[(size_t)b * n_bands + i]) / sigma;
        s += std::exp(-0.5 * t * t);
      }
      acc += wk[b] * s;
    }
    dos_out[e] = 2.0 * norm * acc;
  }
  return SPARC_OK;
}

}  // extern "C"
