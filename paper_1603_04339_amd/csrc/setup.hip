// Context, error reporting and Hamiltonian set-up (FD weights, local potential,
// Bloch-phased projector table).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <numeric>

#include "internal.hpp"

namespace sparc {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

int fail(int status, const char* fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

// Local potential: one thread per node, summing every atom image whose well
// reaches the node (cut at 10 widths); images only along periodic directions.
__global__ void vloc_kernel(int n1, int n2, int n3, double h1, double h2, double h3, double L1, double L2,
                            double L3, int dmask, int n_atoms, const double* __restrict__ R,
                            const double* __restrict__ D, const double* __restrict__ W, double* __restrict__ v) {
  int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  int64_t nd = (int64_t)n1 * n2 * n3;
  if (g >= nd) return;
  int i = (int)(g % n1);
  int j = (int)((g / n1) % n2);
  int k = (int)(g / ((int64_t)n1 * n2));
  double x = i * h1, y = j * h2, z = k * h3;
  double acc = 0.0;
  for (int a = 0; a < n_atoms; ++a) {
    double w = W[a], rc = 10.0 * w, inv2w2 = 1.0 / (2.0 * w * w), dep = D[a];
    double dx0 = x - R[3 * a], dy0 = y - R[3 * a + 1], dz0 = z - R[3 * a + 2];
    int ax0 = (int)ceil((dx0 - rc) / L1), ax1 = (int)floor((dx0 + rc) / L1);
    int ay0 = (int)ceil((dy0 - rc) / L2), ay1 = (int)floor((dy0 + rc) / L2);
    int az0 = (int)ceil((dz0 - rc) / L3), az1 = (int)floor((dz0 + rc) / L3);
    // no images across a Dirichlet direction
    if (dmask & 1) ax0 = ax1 = 0;
    if (dmask & 2) ay0 = ay1 = 0;
    if (dmask & 4) az0 = az1 = 0;
    for (int az = az0; az <= az1; ++az) {
      double dz = dz0 - az * L3;
      for (int ay = ay0; ay <= ay1; ++ay) {
        double dy = dy0 - ay * L2;
        for (int ax = ax0; ax <= ax1; ++ax) {
          double dx = dx0 - ax * L1;
          double r2 = dx * dx + dy * dy + dz * dz;
          if (r2 <= rc * rc) acc -= dep * exp(-r2 * inv2w2);
        }
      }
    }
  }
  v[g] = acc;
}

__global__ void d2f_kernel(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

static hipEvent_t pooled_event(sparc_ctx* c) {
  if (!c->pool.empty()) {
    hipEvent_t e = c->pool.back();
    c->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

int timer_begin(sparc_ctx* c, const char* name) {
  if (!c || !c->timing) return -1;
  sparc_ctx::TimeRec r;
  r.name = name;
  r.a = pooled_event(c);
  r.b = pooled_event(c);
  if (!r.a || !r.b) return -1;
  hipEventRecord(r.a, c->stream);
  c->recs.push_back(r);
  return (int)c->recs.size() - 1;
}

void timer_end(sparc_ctx* c, int idx) {
  if (!c || idx < 0 || idx >= (int)c->recs.size()) return;
  hipEventRecord(c->recs[idx].b, c->stream);
}

static int64_t floordiv(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b != 0) && ((a < 0) != (b < 0))) --q;
  return q;
}

// Host construction of the projector table for one cell.
struct ProjTable {
  std::vector<int32_t> sup_ptr, sup_idx, atom_pbeg, atom_id;
  std::vector<int64_t> proj_voff;
  std::vector<double> gamma;
  std::vector<double> vre, vim;  // values of chi~ (re, im)
};

static int build_projectors(const sparc_grid& G, const double h[3], double dV, const sparc_atoms& A,
                            ProjTable& T) {
  const int n1 = G.n[0], n2 = G.n[1], n3 = G.n[2];
  T.sup_ptr.push_back(0);
  T.atom_pbeg.push_back(0);
  for (int J = 0; J < A.n_atoms; ++J) {
    std::vector<int> chans;
    double rmax = 0.0;
    for (int c = 0; c < A.n_chan; ++c)
      if (A.chan_atom[c] == J) {
        chans.push_back(c);
        rmax = std::max(rmax, A.chan_rc[c]);
      }
    if (chans.empty()) continue;
    // projector functions of this atom: (channel, angular index m; -1 for s)
    std::vector<std::pair<int, int>> funcs;
    for (int c : chans) {
      if (A.chan_l[c] == 0) funcs.push_back({c, -1});
      else for (int m = 0; m < 3; ++m) funcs.push_back({c, m});
    }
    const int nf = (int)funcs.size();
    const double Rx = A.R[3 * J], Ry = A.R[3 * J + 1], Rz = A.R[3 * J + 2];
    // unwrapped nodes within the largest cutoff
    struct Pt { int64_t g; double ph_re, ph_im; std::vector<double> val; };
    std::vector<Pt> pts;
    std::vector<double> norm2(nf, 0.0);
    int64_t i0 = (int64_t)std::ceil((Rx - rmax) / h[0]), i1 = (int64_t)std::floor((Rx + rmax) / h[0]);
    int64_t j0 = (int64_t)std::ceil((Ry - rmax) / h[1]), j1 = (int64_t)std::floor((Ry + rmax) / h[1]);
    int64_t k0 = (int64_t)std::ceil((Rz - rmax) / h[2]), k1 = (int64_t)std::floor((Rz + rmax) / h[2]);
    // a Dirichlet direction keeps the nodes inside the grid (no images, no wrap)
    if (G.bc[0] == 1) { i0 = std::max<int64_t>(i0, 0); i1 = std::min<int64_t>(i1, n1 - 1); }
    if (G.bc[1] == 1) { j0 = std::max<int64_t>(j0, 0); j1 = std::min<int64_t>(j1, n2 - 1); }
    if (G.bc[2] == 1) { k0 = std::max<int64_t>(k0, 0); k1 = std::min<int64_t>(k1, n3 - 1); }
    for (int64_t k = k0; k <= k1; ++k)
      for (int64_t j = j0; j <= j1; ++j)
        for (int64_t i = i0; i <= i1; ++i) {
          double d[3] = {i * h[0] - Rx, j * h[1] - Ry, k * h[2] - Rz};
          double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          if (r2 > rmax * rmax) continue;
          Pt p;
          int64_t wi = floordiv(i, n1), wj = floordiv(j, n2), wk = floordiv(k, n3);
          p.g = (i - wi * n1) + (int64_t)n1 * ((j - wj * n2) + (int64_t)n2 * (k - wk * n3));
          // node x_u = x_g - L with L = -(wraps) * cell; the ket carries e^{i k.L}
          double arg = -(G.kpt[0] * G.L[0] * wi + G.kpt[1] * G.L[1] * wj + G.kpt[2] * G.L[2] * wk);
          p.ph_re = std::cos(arg);
          p.ph_im = std::sin(arg);
          p.val.resize(nf);
          for (int f = 0; f < nf; ++f) {
            int c = funcs[f].first, m = funcs[f].second;
            double rc = A.chan_rc[c], s = rc / 4.0;
            double v = 0.0;
            if (r2 <= rc * rc) {
              v = std::exp(-r2 / (2.0 * s * s));
              if (m >= 0) v *= d[m] / s;
            }
            p.val[f] = v;
            norm2[f] += v * v;
          }
          pts.push_back(std::move(p));
        }
    // merge nodes reached by several images (cutoffs beyond half a cell)
    std::sort(pts.begin(), pts.end(), [](const Pt& a, const Pt& b) { return a.g < b.g; });
    std::vector<int64_t> uniq;
    std::vector<std::vector<double>> re(nf), im(nf);
    for (size_t q = 0; q < pts.size(); ++q) {
      if (uniq.empty() || uniq.back() != pts[q].g) {
        uniq.push_back(pts[q].g);
        for (int f = 0; f < nf; ++f) { re[f].push_back(0.0); im[f].push_back(0.0); }
      }
      for (int f = 0; f < nf; ++f) {
        re[f].back() += pts[q].ph_re * pts[q].val[f];
        im[f].back() += pts[q].ph_im * pts[q].val[f];
      }
    }
    for (int64_t g : uniq) T.sup_idx.push_back((int32_t)g);
    T.sup_ptr.push_back((int32_t)T.sup_idx.size());
    for (int f = 0; f < nf; ++f) {
      double cn = norm2[f] > 0 ? 1.0 / std::sqrt(dV * norm2[f]) : 0.0;
      T.proj_voff.push_back((int64_t)T.vre.size());
      T.gamma.push_back(A.chan_gamma[funcs[f].first]);
      for (size_t t = 0; t < uniq.size(); ++t) {
        T.vre.push_back(cn * re[f][t]);
        T.vim.push_back(cn * im[f][t]);
      }
    }
    T.atom_pbeg.push_back(T.atom_pbeg.back() + nf);
    T.atom_id.push_back(J);
  }
  return SPARC_OK;
}

template <typename E>
static void pack_values(const std::vector<double>& re, const std::vector<double>& im, std::vector<char>& out) {
  out.resize(re.size() * sizeof(E));
  E* p = (E*)out.data();
  for (size_t i = 0; i < re.size(); ++i) {
    if constexpr (elem<E>::is_cplx) {
      p[i].re = (typename elem<E>::real)re[i];
      p[i].im = (typename elem<E>::real)im[i];
    } else {
      p[i] = (E)re[i];
    }
  }
}

static void pack(sparc_dtype dt, const std::vector<double>& re, const std::vector<double>& im,
                 std::vector<char>& out) {
  switch (dt) {
    case SPARC_R64: pack_values<double>(re, im, out); break;
    case SPARC_R32: pack_values<float>(re, im, out); break;
    case SPARC_C128: pack_values<cd>(re, im, out); break;
    case SPARC_C64: pack_values<cf>(re, im, out); break;
  }
}

template <typename T>
static int upload(const std::vector<T>& h, T** d) {
  *d = nullptr;
  size_t bytes = std::max<size_t>(h.size(), 1) * sizeof(T);
  SPARC_HIP(hipMalloc((void**)d, bytes));
  if (!h.empty()) SPARC_HIP(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return SPARC_OK;
}

}  // namespace sparc

using namespace sparc;

extern "C" {

const char* sparc_last_error(void) { return g_last_error.c_str(); }

const char* sparc_status_string(int s) {
  switch (s) {
    case SPARC_OK: return "ok";
    case SPARC_EINVAL: return "invalid argument";
    case SPARC_ESHAPE: return "inconsistent shape";
    case SPARC_ENOMEM: return "workspace too small or allocation failed";
    case SPARC_ENOTSPD: return "Gram matrix not positive definite";
    case SPARC_ENOCONV: return "not converged";
    case SPARC_EDEVICE: return "HIP device error";
    case SPARC_ENAN: return "NaN or Inf in result";
  }
  return "unknown status";
}

int sparc_ctx_create(int device, void* hip_stream, sparc_ctx** out) {
  if (!out) return fail(SPARC_EINVAL, "sparc_ctx_create: out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= device || device < 0)
    return fail(SPARC_EDEVICE, "sparc_ctx_create: device %d not available (%d devices, %s)", device, n,
                hipGetErrorString(e));
  SPARC_HIP(hipSetDevice(device));
  SPARC_TRY(noalloc_scratch_init(device));
  hipDeviceProp_t prop;
  SPARC_HIP(hipGetDeviceProperties(&prop, device));
  sparc_ctx* c = new sparc_ctx;
  c->device = device;
  c->stream = (hipStream_t)hip_stream;
  c->n_cu = prop.multiProcessorCount;
  c->scalars = nullptr;
  if (hipMalloc((void**)&c->scalars, 64 * sizeof(double)) != hipSuccess) {
    delete c;
    return fail(SPARC_ENOMEM, "sparc_ctx_create: scalar scratch allocation failed");
  }
  *out = c;
  return SPARC_OK;
}

static void drop_records(sparc_ctx* ctx) {
  for (auto& r : ctx->recs) {
    ctx->pool.push_back(r.a);
    ctx->pool.push_back(r.b);
  }
  ctx->recs.clear();
}

int sparc_ctx_set_timing(sparc_ctx* ctx, int enable) {
  if (!ctx) return fail(SPARC_EINVAL, "sparc_ctx_set_timing: ctx is NULL");
  SPARC_HIP(hipStreamSynchronize(ctx->stream));
  drop_records(ctx);
  ctx->timing = enable != 0;
  return SPARC_OK;
}

int sparc_ctx_kernel_time(sparc_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches) {
  if (!ctx || !kernel || !total_ms || !launches) return fail(SPARC_EINVAL, "sparc_ctx_kernel_time: null argument");
  SPARC_HIP(hipStreamSynchronize(ctx->stream));
  double t = 0;
  int64_t n = 0;
  for (auto& r : ctx->recs) {
    if (r.name != kernel) continue;
    float ms = 0;
    SPARC_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    t += ms;
    ++n;
  }
  *total_ms = t;
  *launches = n;
  return SPARC_OK;
}

void sparc_ctx_destroy(sparc_ctx* ctx) {
  if (!ctx) return;
  hipStreamSynchronize(ctx->stream);
  drop_records(ctx);
  for (hipEvent_t e : ctx->pool) hipEventDestroy(e);
  if (ctx->scalars) hipFree(ctx->scalars);
  delete ctx;
}

int sparc_ctx_sync(sparc_ctx* ctx) {
  if (!ctx) return fail(SPARC_EINVAL, "sparc_ctx_sync: ctx is NULL");
  SPARC_HIP(hipStreamSynchronize(ctx->stream));
  SPARC_HIP(hipGetLastError());
  return SPARC_OK;
}

int sparc_ham_create(sparc_ctx* ctx, const sparc_grid* grid, const sparc_atoms* atoms, sparc_dtype dtype,
                     sparc_ham** out) {
  if (!ctx || !grid || !atoms || !out) return fail(SPARC_EINVAL, "sparc_ham_create: null argument");
  *out = nullptr;
  if (dtype < SPARC_R64 || dtype > SPARC_C64) return fail(SPARC_EINVAL, "sparc_ham_create: bad dtype %d", dtype);
  if (grid->n_o < 1 || grid->n_o > 8) return fail(SPARC_EINVAL, "sparc_ham_create: n_o=%d outside 1..8", grid->n_o);
  int64_t nd = 1;
  for (int s = 0; s < 3; ++s) {
    if (grid->n[s] < 1 || grid->n[s] > 4096) return fail(SPARC_ESHAPE, "sparc_ham_create: n[%d]=%d", s, grid->n[s]);
    if (!(grid->L[s] > 0)) return fail(SPARC_EINVAL, "sparc_ham_create: L[%d] must be > 0", s);
    nd *= grid->n[s];
  }
  if (nd >= (int64_t(1) << 31)) return fail(SPARC_ESHAPE, "sparc_ham_create: N_d=%lld too large", (long long)nd);
  for (int s = 0; s < 3; ++s) {
    if (grid->bc[s] != 0 && grid->bc[s] != 1)
      return fail(SPARC_EINVAL, "sparc_ham_create: bc[%d]=%d (0 periodic, 1 Dirichlet)", s, grid->bc[s]);
    if (grid->bc[s] == 1 && grid->kpt[s] != 0.0)
      return fail(SPARC_EINVAL, "sparc_ham_create: k[%d] must be 0 in a Dirichlet direction", s);
  }
  bool gamma = grid->kpt[0] == 0.0 && grid->kpt[1] == 0.0 && grid->kpt[2] == 0.0;
  if (!dtype_complex(dtype) && !gamma)
    return fail(SPARC_EINVAL, "sparc_ham_create: real dtype needs the Gamma point");
  if (atoms->n_atoms < 0 || atoms->n_chan < 0) return fail(SPARC_EINVAL, "sparc_ham_create: negative counts");
  if (atoms->n_atoms > 0 && (!atoms->R || !atoms->vloc_depth || !atoms->vloc_width))
    return fail(SPARC_EINVAL, "sparc_ham_create: atom arrays missing");
  if (atoms->n_chan > 0 && (!atoms->chan_atom || !atoms->chan_l || !atoms->chan_gamma || !atoms->chan_rc))
    return fail(SPARC_EINVAL, "sparc_ham_create: channel arrays missing");
  for (int c = 0; c < atoms->n_chan; ++c) {
    if (atoms->chan_atom[c] < 0 || atoms->chan_atom[c] >= atoms->n_atoms)
      return fail(SPARC_EINVAL, "sparc_ham_create: channel %d atom %d out of range", c, atoms->chan_atom[c]);
    if (atoms->chan_l[c] != 0 && atoms->chan_l[c] != 1)
      return fail(SPARC_EINVAL, "sparc_ham_create: channel %d has l=%d (0 or 1 supported)", c, atoms->chan_l[c]);
    if (!(atoms->chan_rc[c] > 0)) return fail(SPARC_EINVAL, "sparc_ham_create: channel %d rc <= 0", c);
  }
  SPARC_HIP(hipSetDevice(ctx->device));

  sparc_ham* H = new sparc_ham();
  H->ctx = ctx;
  H->grid = *grid;
  H->dtype = dtype;
  H->n_d = nd;
  H->gamma = gamma;
  for (int s = 0; s < 3; ++s) H->h[s] = grid->L[s] / grid->n[s];
  H->dV = H->h[0] * H->h[1] * H->h[2];
  // FD weights of the Laplacian (Sec. 3.1): w0 = -(1/h^2) sum 1/q^2,
  // w_p = 2(-1)^{p+1}(n_o!)^2 / (h^2 p^2 (n_o-p)!(n_o+p)!); the operator is -1/2 of the sum.
  const int no = grid->n_o;
  double fact[20];
  fact[0] = 1.0;
  for (int i = 1; i < 20; ++i) fact[i] = fact[i - 1] * i;
  H->centre = 0.0;
  for (int s = 0; s < 3; ++s) {
    double inv_h2 = 1.0 / (H->h[s] * H->h[s]);
    double w0 = 0.0;
    for (int q = 1; q <= no; ++q) w0 -= 1.0 / (double(q) * q);
    H->centre += -0.5 * 2.0 * w0 * inv_h2;
    for (int p = 1; p <= 8; ++p) {
      double wp = 0.0;
      if (p <= no) wp = 2.0 * ((p & 1) ? 1.0 : -1.0) * fact[no] * fact[no] / (double(p) * p * fact[no - p] * fact[no + p]) * inv_h2;
      H->tap[s][p - 1] = -0.5 * wp;
    }
    double kl = grid->kpt[s] * grid->L[s];
    H->ph_re[s] = std::cos(kl);
    H->ph_im[s] = std::sin(kl);
    // FD gradient weights (Sec. 3.1): w~_p = (-1)^{p+1} (n_o!)^2 / (h p (n_o-p)! (n_o+p)!)
    for (int p = 1; p <= 8; ++p)
      H->gtap[s][p - 1] = (p <= no) ? ((p & 1) ? 1.0 : -1.0) * fact[no] * fact[no] /
                                          (H->h[s] * p * fact[no - p] * fact[no + p])
                                    : 0.0;
  }

  // local potential on the device
  hipStream_t st = ctx->stream;
  int rc = SPARC_OK;
  double *dR = nullptr, *dD = nullptr, *dW = nullptr;
  {
    std::vector<double> R(atoms->R ? atoms->R : (const double*)nullptr,
                          atoms->R ? atoms->R + 3 * atoms->n_atoms : (const double*)nullptr);
    std::vector<double> Dp(atoms->vloc_depth ? atoms->vloc_depth : (const double*)nullptr,
                           atoms->vloc_depth ? atoms->vloc_depth + atoms->n_atoms : (const double*)nullptr);
    std::vector<double> Wp(atoms->vloc_width ? atoms->vloc_width : (const double*)nullptr,
                           atoms->vloc_width ? atoms->vloc_width + atoms->n_atoms : (const double*)nullptr);
    rc = upload(R, &dR);
    if (!rc) rc = upload(Dp, &dD);
    if (!rc) rc = upload(Wp, &dW);
    H->n_atoms = atoms->n_atoms;
    H->atom_R = dR;   // owned by the Hamiltonian from here on (atomic forces)
    H->atom_D = dD;
    H->atom_W = dW;
    if (!rc && atoms->n_atoms > 0 &&
        hipMalloc(&H->force_part, (size_t)atoms->n_atoms * kForceChunks * 3 * sizeof(double)) != hipSuccess)
      rc = fail(SPARC_ENOMEM, "sparc_ham_create: force buffer allocation failed");
    if (!rc && grid->bc[2] == 1) {   // plane of zeros (16 bytes per node covers every element type)
      const size_t zb = (size_t)grid->n[0] * grid->n[1] * 16;
      if (hipMalloc(&H->zplane, zb) != hipSuccess || hipMemsetAsync(H->zplane, 0, zb, ctx->stream) != hipSuccess)
        rc = fail(SPARC_ENOMEM, "sparc_ham_create: zero-plane allocation failed");
    }
    if (rc) {
      sparc_ham_destroy(H);
      return rc;
    }
  }
  if (hipMalloc(&H->vloc, nd * 8) != hipSuccess || hipMalloc(&H->veff, nd * 8) != hipSuccess ||
      hipMalloc(&H->veff32, nd * 4) != hipSuccess) {
    sparc_ham_destroy(H);
    return fail(SPARC_ENOMEM, "sparc_ham_create: potential allocation failed");
  }
  {
    int blk = 256;
    int64_t nb = (nd + blk - 1) / blk;
    vloc_kernel<<<dim3((unsigned)nb), dim3(blk), 0, st>>>(grid->n[0], grid->n[1], grid->n[2], H->h[0], H->h[1],
                                                           H->h[2], grid->L[0], grid->L[1], grid->L[2],
                                                           dirichlet_mask(*grid), atoms->n_atoms, dR, dD, dW,
                                                           H->vloc);
    if ((rc = check_launch("vloc_kernel"))) { sparc_ham_destroy(H); return rc; }
    hipMemcpyAsync(H->veff, H->vloc, nd * 8, hipMemcpyDeviceToDevice, st);
    d2f_kernel<<<dim3((unsigned)nb), dim3(blk), 0, st>>>(H->vloc, H->veff32, nd);
  }

  // projector table (host construction, then upload)
  ProjTable T;
  build_projectors(*grid, H->h, H->dV, *atoms, T);
  H->n_atoms_nl = (int32_t)T.sup_ptr.size() - 1;
  H->n_proj = (int32_t)T.gamma.size();
  H->n_sup = (int64_t)T.sup_idx.size();
  H->max_proj_per_atom = 0;
  for (int a = 0; a < H->n_atoms_nl; ++a)
    H->max_proj_per_atom = std::max(H->max_proj_per_atom, T.atom_pbeg[a + 1] - T.atom_pbeg[a]);
  // per-node entry lists (CSR over grid nodes)
  std::vector<int32_t> cnt(nd + 1, 0);
  for (int a = 0; a < H->n_atoms_nl; ++a) {
    int np = T.atom_pbeg[a + 1] - T.atom_pbeg[a];
    for (int t = T.sup_ptr[a]; t < T.sup_ptr[a + 1]; ++t) cnt[T.sup_idx[t] + 1] += np;
  }
  std::vector<int64_t> pt_ptr(nd + 1, 0);
  for (int64_t g = 0; g < nd; ++g) pt_ptr[g + 1] = pt_ptr[g] + cnt[g + 1];
  H->n_ent = pt_ptr[nd];
  if (H->n_ent >= (int64_t(1) << 31)) {
    sparc_ham_destroy(H);
    return fail(SPARC_ESHAPE, "sparc_ham_create: %lld projector entries exceed int32", (long long)H->n_ent);
  }
  // compressed to the nodes that carry support
  std::vector<int32_t> nl_pts, nl_ptr;
  for (int64_t g = 0; g < nd; ++g)
    if (cnt[g + 1] > 0) {
      nl_pts.push_back((int32_t)g);
      nl_ptr.push_back((int32_t)pt_ptr[g]);
    }
  nl_ptr.push_back((int32_t)H->n_ent);
  H->n_nlpts = (int64_t)nl_pts.size();
  std::vector<int32_t> ent_proj(H->n_ent), ent_key(H->n_ent);
  std::vector<double> ere(H->n_ent), eim(H->n_ent), cre(H->n_ent), cim(H->n_ent);
  {
    std::vector<int64_t> fill(pt_ptr.begin(), pt_ptr.end() - 1);
    for (int a = 0; a < H->n_atoms_nl; ++a)
      for (int p = T.atom_pbeg[a]; p < T.atom_pbeg[a + 1]; ++p)
        for (int t = T.sup_ptr[a]; t < T.sup_ptr[a + 1]; ++t) {
          int64_t g = T.sup_idx[t];
          int64_t e = fill[g]++;
          int64_t vi = T.proj_voff[p] + (t - T.sup_ptr[a]);
          ent_proj[e] = p;
          ent_key[e] = 4 * a + (p - T.atom_pbeg[a]);
          ere[e] = T.gamma[p] * T.vre[vi];
          eim[e] = T.gamma[p] * T.vim[vi];
          cre[e] = T.vre[vi];
          cim[e] = T.vim[vi];
        }
  }
  // the projector scatter inside the stencil step, on request (SPARC_NL_FUSED=1): the
  // separate projection and scatter kernels are the default, as fast or faster on the
  // measured cells (FP64 within 2 %, FP32 and complex slower fused)
  const char* fenv = getenv("SPARC_NL_FUSED");
  const bool fuse = fenv && fenv[0] == '1';
  H->nl_fused = H->n_proj > 0 && H->max_proj_per_atom <= 4 && fuse;
  std::vector<char> pv, ec, gm;
  pack(dtype, T.vre, T.vim, pv);
  pack(dtype, ere, eim, ec);
  std::vector<double> zeros(T.gamma.size(), 0.0);
  pack(dtype_single(dtype) ? SPARC_R32 : SPARC_R64, T.gamma, zeros, gm);
  if ((rc = upload(T.sup_ptr, &H->sup_ptr)) || (rc = upload(T.sup_idx, &H->sup_idx)) ||
      (rc = upload(T.atom_id, &H->nl_atom)) ||
      (rc = upload(T.atom_pbeg, &H->atom_pbeg)) || (rc = upload(T.proj_voff, &H->proj_voff)) ||
      (rc = upload(pv, (char**)&H->pval)) || (rc = upload(gm, (char**)&H->gamma_d)) ||
      (rc = upload(nl_pts, &H->nl_pts)) || (rc = upload(nl_ptr, &H->nl_ptr)) || (rc = upload(ent_proj, &H->ent_proj)) ||
      (rc = upload(ec, (char**)&H->ent_coef))) {
    sparc_ham_destroy(H);
    return rc;
  }
  if (H->nl_fused && (rc = nl_tables_build(H, T.sup_ptr, T.sup_idx, nl_pts, nl_ptr, ent_key, cre, cim))) {
    sparc_ham_destroy(H);
    return rc;
  }
  hipError_t e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    sparc_ham_destroy(H);
    return fail(SPARC_EDEVICE, "sparc_ham_create: %s", hipGetErrorString(e));
  }
  *out = H;
  return SPARC_OK;
}

void sparc_ham_destroy(sparc_ham* H) {
  if (!H) return;
  void* ptrs[] = {H->vloc, H->veff, H->veff32, H->sup_ptr, H->sup_idx, H->atom_pbeg, H->proj_voff,
                  H->pval, H->gamma_d, H->nl_pts, H->nl_ptr, H->ent_proj, H->ent_coef,
                  H->atom_R, H->atom_D, H->atom_W, H->force_part, H->nl_atom, H->zplane};
  for (void* p : ptrs)
    if (p) hipFree(p);
  nl_tables_free(H);
  delete H;
}

int sparc_ham_set_veff(sparc_ham* H, const double* veff_dev) {
  if (!H || !veff_dev) return fail(SPARC_EINVAL, "sparc_ham_set_veff: null argument");
  hipStream_t st = H->ctx->stream;
  SPARC_HIP(hipMemcpyAsync(H->veff, veff_dev, H->n_d * 8, hipMemcpyDeviceToDevice, st));
  int64_t nb = (H->n_d + 255) / 256;
  d2f_kernel<<<dim3((unsigned)nb), dim3(256), 0, st>>>(H->veff, H->veff32, H->n_d);
  return check_launch("d2f_kernel");
}

int sparc_ham_get_vloc(const sparc_ham* H, double* vloc_dev) {
  if (!H || !vloc_dev) return fail(SPARC_EINVAL, "sparc_ham_get_vloc: null argument");
  SPARC_HIP(hipMemcpyAsync(vloc_dev, H->vloc, H->n_d * 8, hipMemcpyDeviceToDevice, H->ctx->stream));
  return SPARC_OK;
}

int sparc_ham_info(const sparc_ham* H, int64_t* n_d, int32_t* n_proj, int64_t* n_entries) {
  if (!H) return fail(SPARC_EINVAL, "sparc_ham_info: null ham");
  if (n_d) *n_d = H->n_d;
  if (n_proj) *n_proj = H->n_proj;
  if (n_entries) *n_entries = H->n_ent;
  return SPARC_OK;
}

}  // extern "C"
