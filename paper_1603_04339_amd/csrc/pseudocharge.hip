// Pseudocharge electrostatics (Sec. 2, electrostatic reformulation with the pseudocharge
// b = -Lap V / (4 pi), the self energy and the overlap correction E_c; Sec. 3.2, the
// discrete pseudocharge and self energy of Algorithm 1 with the truncation radius r^b
// chosen from the charge error eps_b; Appendix A, discrete E_c and correction force;
// Sec. 3.6, discrete local force with pseudocharges).
//
// Local pseudopotential of atom J (valence charge Z_J, cutoff rc_J): the potential of
// the compactly supported charge -Z_J 315/(64 pi rc^3) (1 - r^2/rc^2)^3, i.e.
//   V(r) = -Z/r (r >= rc),   V(r) = -(Z/rc) (315 - 420 s^2 + 378 s^4 - 180 s^6 + 35 s^8)/128,
//   s = r/rc (r < rc);
// the reference potential of the overlap correction is the same form with cutoff
// rc~_J.  Potentials are evaluated in closed form at every node they are needed at (the
// paper interpolates radial tables with cubic splines there).
//
// Kernels:
//  * psd_shell_kernel: per (atom, kind) and z-plane of the largest candidate box, the
//    discrete pseudocharge of every node binned by the smallest candidate box holding it;
//    the host accumulates the shells and picks the first box whose charge is within
//    eps_b Z of -Z.
//  * psd_grid_kernel: node-major; a work-group owns a 16x4x4 tile of nodes, collects (in
//    image order) the atom images whose boxes meet the tile, and every thread sums over
//    them b, b~, V_c and the self-energy and E_c integrands of its node.  No atomics:
//    each node is written by one thread, the energy partials are reduced in a fixed order.
//  * psd_force_kernel: image-major; a work-group owns 256 nodes of one image's box and
//    evaluates the local-force and correction-force integrands there, with the FD
//    gradient of the node's pseudocharges taken from the closed-form potential; partials
//    per (image, chunk) are summed per atom in a fixed order on the host.
#include <algorithm>
#include <cmath>
#include <vector>

#include "devmath.hpp"

using namespace sparc;

namespace {

constexpr int kTruncSteps = 16;  // candidate boxes beyond ceil(rc/h): one node per direction each
constexpr int kMaxNo = 8;
constexpr int kMaxHalf = 1024;   // largest box half-width in nodes

// FD weights in device memory: [0,3) Laplacian centre per direction (2 w_0 / h^2),
// [3,27) Laplacian taps w_p / h^2, [27,51) gradient taps w~_p / h, [51,54) h
enum { W_LAP0 = 0, W_LAP = 3, W_GRD = 27, W_H = 51, W_COUNT = 54 };

void fd_weights(const sparc_grid& g, double* w) {
  const int no = g.n_o;
  double fact[20];
  fact[0] = 1.0;
  for (int i = 1; i < 20; ++i) fact[i] = fact[i - 1] * i;
  for (int s = 0; s < 3; ++s) {
    const double h = g.L[s] / g.n[s];
    double w0 = 0.0;
    for (int q = 1; q <= no; ++q) w0 -= 1.0 / (double(q) * q);
    w[W_LAP0 + s] = 2.0 * w0 / (h * h);
    for (int p = 1; p <= kMaxNo; ++p) {
      const double sg = (p & 1) ? 1.0 : -1.0;
      w[W_LAP + 8 * s + p - 1] =
          p <= no ? 2.0 * sg * fact[no] * fact[no] / (double(p) * p * fact[no - p] * fact[no + p]) / (h * h) : 0.0;
      w[W_GRD + 8 * s + p - 1] = p <= no ? sg * fact[no] * fact[no] / (h * p * fact[no - p] * fact[no + p]) : 0.0;
    }
    w[W_H + s] = h;
  }
}

// ---------------------------------------------------------------- potentials
__device__ __forceinline__ double vpsd(double r2, double Z, double rc) {
  const double r = sqrt(r2);
  if (r < rc) {
    const double t = r / rc, s2 = t * t;
    return -(Z / rc) * ((315.0 / 128.0) +
                        s2 * ((-420.0 / 128.0) + s2 * ((378.0 / 128.0) + s2 * ((-180.0 / 128.0) + s2 * (35.0 / 128.0)))));
  }
  return -Z / r;
}

// b = -(1/4pi) Lap_h V at offset (x, y, z) from the atom
__device__ double lap_b(const double* __restrict__ w, int no, double x, double y, double z, double Z, double rc) {
  const double x2 = x * x, y2 = y * y, z2 = z * z;
  double acc = (w[W_LAP0] + w[W_LAP0 + 1] + w[W_LAP0 + 2]) * vpsd(x2 + y2 + z2, Z, rc);
#pragma unroll 1
  for (int p = 1; p <= no; ++p) {
    const double ex = p * w[W_H], ey = p * w[W_H + 1], ez = p * w[W_H + 2];
    const double xp = x + ex, xm = x - ex, yp = y + ey, ym = y - ey, zp = z + ez, zm = z - ez;
    acc += w[W_LAP + p - 1] * (vpsd(xp * xp + y2 + z2, Z, rc) + vpsd(xm * xm + y2 + z2, Z, rc));
    acc += w[W_LAP + 8 + p - 1] * (vpsd(x2 + yp * yp + z2, Z, rc) + vpsd(x2 + ym * ym + z2, Z, rc));
    acc += w[W_LAP + 16 + p - 1] * (vpsd(x2 + y2 + zp * zp, Z, rc) + vpsd(x2 + y2 + zm * zm, Z, rc));
  }
  return acc * (-0.25 / M_PI);
}

// FD gradient (Sec. 3.1) of b_J' (KIND 0), of V (KIND 1) or of V(rc2) - V(rc) (KIND 2)
template <int KIND>
__device__ void fd_grad(const double* __restrict__ w, int no, double x, double y, double z, double Z, double rc,
                        double rc2, double g[3]) {
  auto f = [&](double a, double b, double c) -> double {
    if (KIND == 0) return lap_b(w, no, a, b, c, Z, rc);
    const double r2 = a * a + b * b + c * c;
    if (KIND == 1) return vpsd(r2, Z, rc);
    return vpsd(r2, Z, rc2) - vpsd(r2, Z, rc);
  };
  g[0] = g[1] = g[2] = 0.0;
#pragma unroll 1
  for (int p = 1; p <= no; ++p) {
    const double ex = p * w[W_H], ey = p * w[W_H + 1], ez = p * w[W_H + 2];
    g[0] += w[W_GRD + p - 1] * (f(x + ex, y, z) - f(x - ex, y, z));
    g[1] += w[W_GRD + 8 + p - 1] * (f(x, y + ey, z) - f(x, y - ey, z));
    g[2] += w[W_GRD + 16 + p - 1] * (f(x, y, z + ez) - f(x, y, z - ez));
  }
}

// ---------------------------------------------------------------- truncation boxes
struct ShellJob {
  double R[3];
  double Z, rc;
  int cu[3], fu[3];  // ceil and floor of R_s / h_s
  int m0[3];         // ceil(rc / h_s)
};

__global__ __launch_bounds__(256) void psd_shell_kernel(const double* __restrict__ w, int no,
                                                        const ShellJob* __restrict__ jobs, int max_planes,
                                                        double* __restrict__ part) {
  const ShellJob& jb = jobs[blockIdx.y];
  const int plane = blockIdx.x;
  const int M0 = jb.m0[0] + kTruncSteps, M1 = jb.m0[1] + kTruncSteps, M2 = jb.m0[2] + kTruncSteps;
  const int nx = jb.fu[0] - jb.cu[0] + 2 * M0 + 1, ny = jb.fu[1] - jb.cu[1] + 2 * M1 + 1;
  const int nz = jb.fu[2] - jb.cu[2] + 2 * M2 + 1;
  double sh[kTruncSteps + 1];
#pragma unroll
  for (int t = 0; t <= kTruncSteps; ++t) sh[t] = 0.0;
  if (plane < nz) {
    const int k = jb.cu[2] - M2 + plane;
    const int mk = max(jb.cu[2] - k, k - jb.fu[2]) - jb.m0[2];
    const double z = k * w[W_H + 2] - jb.R[2];
    for (int q = threadIdx.x; q < nx * ny; q += blockDim.x) {
      const int i = jb.cu[0] - M0 + q % nx, j = jb.cu[1] - M1 + q / nx;
      const int mi = max(jb.cu[0] - i, i - jb.fu[0]) - jb.m0[0];
      const int mj = max(jb.cu[1] - j, j - jb.fu[1]) - jb.m0[1];
      const int shell = max(0, max(mk, max(mi, mj)));
      const double b = lap_b(w, no, i * w[W_H] - jb.R[0], j * w[W_H + 1] - jb.R[1], z, jb.Z, jb.rc);
#pragma unroll
      for (int t = 0; t <= kTruncSteps; ++t) sh[t] += (shell == t) ? b : 0.0;
    }
  }
  __shared__ double red[kTruncSteps + 1][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int t = 0; t <= kTruncSteps; ++t) {
    const double s = wave_sum(sh[t]);
    if (lane == 0) red[t][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x <= kTruncSteps) {
    const int t = threadIdx.x;
    part[((size_t)blockIdx.y * max_planes + plane) * (kTruncSteps + 1) + t] =
        ((red[t][0] + red[t][1]) + red[t][2]) + red[t][3];
  }
}

// ---------------------------------------------------------------- images
struct PsdImage {
  double c[3];
  double Z, rc, rcr;
  int atom;
  int lo[3][3], hi[3][3];  // [kind][direction] node ranges (unclipped): 0 pseudocharge box,
                           // 1 reference box, 2 union with the support of grad (V~ - V)
};

__device__ __forceinline__ bool in_box(const PsdImage& im, int kind, int i, int j, int k) {
  return i >= im.lo[kind][0] && i <= im.hi[kind][0] && j >= im.lo[kind][1] && j <= im.hi[kind][1] &&
         k >= im.lo[kind][2] && k <= im.hi[kind][2];
}

// sum of three per-thread values over a 256-thread work-group (fixed order)
__device__ __forceinline__ void block_sum_n3(const double v[3], double* out) {
  __shared__ double red[3][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double s = wave_sum(v[d]);
    if (lane == 0) red[d][wv] = s;
  }
  __syncthreads();
  if (threadIdx.x < 3) out[threadIdx.x] = ((red[threadIdx.x][0] + red[threadIdx.x][1]) + red[threadIdx.x][2]) + red[threadIdx.x][3];
  __syncthreads();
}

constexpr int TX = 16, TY = 4, TZ = 4;

__global__ __launch_bounds__(256) void psd_grid_kernel(const double* __restrict__ w, int no, int n1, int n2, int n3,
                                                       const PsdImage* __restrict__ imgs, int n_img,
                                                       double* __restrict__ b, double* __restrict__ bref,
                                                       double* __restrict__ vc, double* __restrict__ part) {
  const int tx = (n1 + TX - 1) / TX, ty = (n2 + TY - 1) / TY;
  const int t = blockIdx.x;
  const int i0 = (t % tx) * TX, j0 = ((t / tx) % ty) * TY, k0 = (t / (tx * ty)) * TZ;
  const int i = i0 + (threadIdx.x & (TX - 1)), j = j0 + ((threadIdx.x >> 4) & (TY - 1)), k = k0 + (threadIdx.x >> 6);
  const bool valid = i < n1 && j < n2 && k < n3;
  const double x = i * w[W_H], y = j * w[W_H + 1], z = k * w[W_H + 2];
  __shared__ int list[256];
  __shared__ int wcount[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double sb = 0.0, sr = 0.0, sv = 0.0, es = 0.0, er = 0.0;
  for (int base = 0; base < n_img; base += 256) {
    const int q = base + threadIdx.x;
    bool hit = false;
    if (q < n_img) {
      const PsdImage& im = imgs[q];
      hit = im.lo[2][0] <= i0 + TX - 1 && im.hi[2][0] >= i0 && im.lo[2][1] <= j0 + TY - 1 && im.hi[2][1] >= j0 &&
            im.lo[2][2] <= k0 + TZ - 1 && im.hi[2][2] >= k0;
    }
    const uint64_t m = __ballot(hit);
    if (lane == 0) wcount[wv] = __popcll(m);
    __syncthreads();
    int off = 0;
    for (int v = 0; v < wv; ++v) off += wcount[v];
    const int total = wcount[0] + wcount[1] + wcount[2] + wcount[3];
    if (hit) list[off + __popcll(m & ((1ull << lane) - 1ull))] = q;
    __syncthreads();
    if (valid) {
      for (int e = 0; e < total; ++e) {
        const PsdImage& im = imgs[list[e]];
        const double dx = x - im.c[0], dy = y - im.c[1], dz = z - im.c[2];
        const double r2 = dx * dx + dy * dy + dz * dz;
        const double v = vpsd(r2, im.Z, im.rc), vr = vpsd(r2, im.Z, im.rcr);
        if (in_box(im, 0, i, j, k)) {
          const double bj = lap_b(w, no, dx, dy, dz, im.Z, im.rc);
          sb += bj;
          es += bj * v;
        }
        if (in_box(im, 1, i, j, k)) {
          const double bj = lap_b(w, no, dx, dy, dz, im.Z, im.rcr);
          sr += bj;
          er += bj * vr;
        }
        sv += vr - v;
      }
    }
    __syncthreads();
  }
  double e3[3] = {0.0, 0.0, 0.0};
  if (valid) {
    const int64_t g = i + (int64_t)n1 * (j + (int64_t)n2 * k);
    b[g] = sb;
    bref[g] = sr;
    vc[g] = sv;
    e3[0] = es;
    e3[1] = er;
    e3[2] = (sb + sr) * sv;
  }
  block_sum_n3(e3, part + 3 * (size_t)blockIdx.x);
}

// ---------------------------------------------------------------- forces
struct ForceJob {
  int img;
  int chunk;
  int lo[3];  // clipped union box
  int nx, ny, nz;
};

__global__ __launch_bounds__(256) void psd_force_kernel(const double* __restrict__ w, int no, int n1, int n2,
                                                        const PsdImage* __restrict__ imgs,
                                                        const ForceJob* __restrict__ jobs,
                                                        const double* __restrict__ phi, const double* __restrict__ b,
                                                        const double* __restrict__ bref,
                                                        const double* __restrict__ vc, double* __restrict__ part) {
  const ForceJob& jb = jobs[blockIdx.x];
  const PsdImage& im = imgs[jb.img];
  const int64_t nbox = (int64_t)jb.nx * jb.ny * jb.nz;
  const int64_t q = (int64_t)jb.chunk * 256 + threadIdx.x;
  double fl[3] = {0.0, 0.0, 0.0}, fc[3] = {0.0, 0.0, 0.0};
  if (q < nbox) {
    const int i = jb.lo[0] + (int)(q % jb.nx), j = jb.lo[1] + (int)((q / jb.nx) % jb.ny),
              k = jb.lo[2] + (int)(q / ((int64_t)jb.nx * jb.ny));
    const int64_t g = i + (int64_t)n1 * (j + (int64_t)n2 * k);
    const double dx = i * w[W_H] - im.c[0], dy = j * w[W_H + 1] - im.c[1], dz = k * w[W_H + 2] - im.c[2];
    const double r2 = dx * dx + dy * dy + dz * dz;
    const double vcg = vc[g];
    double gb[3], gv[3];
    if (in_box(im, 0, i, j, k)) {
      fd_grad<0>(w, no, dx, dy, dz, im.Z, im.rc, 0.0, gb);
      fd_grad<1>(w, no, dx, dy, dz, im.Z, im.rc, 0.0, gv);
      const double v = vpsd(r2, im.Z, im.rc), bj = lap_b(w, no, dx, dy, dz, im.Z, im.rc);
      const double pv = phi[g] - v;
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        fl[d] = gb[d] * pv;
        fc[d] += 0.5 * (gb[d] * (vcg + v) + bj * gv[d]);
      }
    }
    if (in_box(im, 1, i, j, k)) {
      fd_grad<0>(w, no, dx, dy, dz, im.Z, im.rcr, 0.0, gb);
      fd_grad<1>(w, no, dx, dy, dz, im.Z, im.rcr, 0.0, gv);
      const double v = vpsd(r2, im.Z, im.rcr), bj = lap_b(w, no, dx, dy, dz, im.Z, im.rcr);
#pragma unroll
      for (int d = 0; d < 3; ++d) fc[d] += 0.5 * (gb[d] * (vcg - v) - bj * gv[d]);
    }
    fd_grad<2>(w, no, dx, dy, dz, im.Z, im.rc, im.rcr, gv);
    const double bs = b[g] + bref[g];
#pragma unroll
    for (int d = 0; d < 3; ++d) fc[d] += 0.5 * gv[d] * bs;
  }
  block_sum_n3(fl, part + 6 * (size_t)blockIdx.x);
  block_sum_n3(fc, part + 6 * (size_t)blockIdx.x + 3);
}

__global__ void add_forces_kernel(int n, const double* __restrict__ a, double* __restrict__ F) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) F[t] += a[t];
}

// ---------------------------------------------------------------- host helpers
struct DevMem {
  std::vector<void*> p;
  ~DevMem() {
    for (void* q : p) hipFree(q);
  }
  template <typename T>
  int alloc(T** q, size_t count, const char* who) {
    *q = nullptr;
    void* r = nullptr;
    if (hipMalloc(&r, std::max<size_t>(count, 1) * sizeof(T)) != hipSuccess)
      return fail(SPARC_ENOMEM, "%s: device allocation of %zu bytes failed", who, count * sizeof(T));
    p.push_back(r);
    *q = (T*)r;
    return SPARC_OK;
  }
};

int check_common(const sparc_grid* g, const sparc_atoms* a, const char* who) {
  if (!g || !a) return fail(SPARC_EINVAL, "%s: null argument", who);
  if (g->n_o < 1 || g->n_o > kMaxNo) return fail(SPARC_EINVAL, "%s: n_o=%d outside 1..8", who, g->n_o);
  for (int s = 0; s < 3; ++s) {
    if (g->n[s] < 1 || g->n[s] > 4096) return fail(SPARC_ESHAPE, "%s: n[%d]=%d outside 1..4096", who, s, g->n[s]);
    if (!(g->L[s] > 0.0)) return fail(SPARC_EINVAL, "%s: L[%d] must be positive", who, s);
    if (g->bc[s] != 0 && g->bc[s] != 1) return fail(SPARC_EINVAL, "%s: bc[%d]=%d outside {0,1}", who, s, g->bc[s]);
  }
  if ((int64_t)g->n[0] * g->n[1] * g->n[2] >= (int64_t)1 << 31) return fail(SPARC_ESHAPE, "%s: N_d >= 2^31", who);
  if (a->n_atoms < 1 || !a->R || !a->Z || !a->psd_rc || !a->psd_rc_ref)
    return fail(SPARC_EINVAL, "%s: need n_atoms >= 1 and R, Z, psd_rc, psd_rc_ref", who);
  for (int J = 0; J < a->n_atoms; ++J) {
    if (!(a->Z[J] > 0.0) || !(a->psd_rc[J] > 0.0) || !(a->psd_rc_ref[J] > 0.0))
      return fail(SPARC_EINVAL, "%s: atom %d needs Z, psd_rc, psd_rc_ref > 0", who, J);
    for (int s = 0; s < 3; ++s)
      if (!std::isfinite(a->R[3 * J + s])) return fail(SPARC_EINVAL, "%s: atom %d position not finite", who, J);
  }
  return SPARC_OK;
}

int check_boxes(const sparc_atoms* a, const int32_t* boxes, const char* who) {
  if (!boxes) return fail(SPARC_EINVAL, "%s: null boxes", who);
  for (int q = 0; q < 6 * a->n_atoms; ++q)
    if (boxes[q] < 0 || boxes[q] > kMaxHalf)
      return fail(SPARC_EINVAL, "%s: box half-width %d outside 0..%d", who, boxes[q], kMaxHalf);
  return SPARC_OK;
}

// every image whose union box meets the cell (none across Dirichlet directions)
void build_images(const sparc_grid& g, const sparc_atoms* a, const int32_t* boxes, std::vector<PsdImage>& out) {
  out.clear();
  for (int J = 0; J < a->n_atoms; ++J) {
    const double rc = a->psd_rc[J], rcr = a->psd_rc_ref[J];
    int cu[3], fu[3], m[3][3];
    std::vector<int> shifts[3];
    for (int s = 0; s < 3; ++s) {
      const double h = g.L[s] / g.n[s];
      const double u = a->R[3 * J + s] / h;
      cu[s] = (int)std::ceil(u);
      fu[s] = (int)std::floor(u);
      m[0][s] = boxes[6 * J + s];
      m[1][s] = boxes[6 * J + 3 + s];
      m[2][s] = std::max({m[0][s], m[1][s], (int)std::ceil(std::max(rc, rcr) / h) + g.n_o + 1});
      const int lo = cu[s] - m[2][s], hi = fu[s] + m[2][s];
      if (g.bc[s] == 1) {
        if (lo <= g.n[s] - 1 && hi >= 0) shifts[s].push_back(0);
      } else {
        const int A = (std::abs(lo) + std::abs(hi)) / g.n[s] + 2;
        for (int sh = -A; sh <= A; ++sh)
          if (lo + sh * g.n[s] <= g.n[s] - 1 && hi + sh * g.n[s] >= 0) shifts[s].push_back(sh);
      }
    }
    for (int az : shifts[2])
      for (int ay : shifts[1])
        for (int ax : shifts[0]) {
          PsdImage im;
          const int sh[3] = {ax, ay, az};
          for (int s = 0; s < 3; ++s) {
            im.c[s] = a->R[3 * J + s] + sh[s] * g.L[s];
            for (int kind = 0; kind < 3; ++kind) {
              im.lo[kind][s] = cu[s] - m[kind][s] + sh[s] * g.n[s];
              im.hi[kind][s] = fu[s] + m[kind][s] + sh[s] * g.n[s];
            }
          }
          im.Z = a->Z[J];
          im.rc = rc;
          im.rcr = rcr;
          im.atom = J;
          out.push_back(im);
        }
  }
}

}  // namespace

extern "C" {

int sparc_psd_boxes(sparc_ctx* ctx, const sparc_grid* grid, const sparc_atoms* atoms, double eps_b, int32_t* boxes) {
  const char* who = "sparc_psd_boxes";
  if (!ctx || !boxes) return fail(SPARC_EINVAL, "%s: null argument", who);
  SPARC_TRY(check_common(grid, atoms, who));
  if (!(eps_b > 0.0) || !(eps_b < 1.0)) return fail(SPARC_EINVAL, "%s: eps_b must lie in (0, 1)", who);
  hipStream_t s = ctx->stream;
  const int na = atoms->n_atoms;
  double w[W_COUNT];
  fd_weights(*grid, w);
  std::vector<ShellJob> jobs(2 * na);
  int max_planes = 0;
  for (int J = 0; J < na; ++J)
    for (int kind = 0; kind < 2; ++kind) {
      ShellJob& jb = jobs[2 * J + kind];
      jb.Z = atoms->Z[J];
      jb.rc = kind == 0 ? atoms->psd_rc[J] : atoms->psd_rc_ref[J];
      for (int d = 0; d < 3; ++d) {
        const double h = w[W_H + d];
        jb.R[d] = atoms->R[3 * J + d];
        jb.cu[d] = (int)std::ceil(jb.R[d] / h);
        jb.fu[d] = (int)std::floor(jb.R[d] / h);
        jb.m0[d] = (int)std::ceil(jb.rc / h);
        if (jb.m0[d] + kTruncSteps > kMaxHalf)
          return fail(SPARC_EINVAL, "%s: atom %d cutoff spans more than %d nodes", who, J, kMaxHalf - kTruncSteps);
      }
      max_planes = std::max(max_planes, jb.fu[2] - jb.cu[2] + 2 * (jb.m0[2] + kTruncSteps) + 1);
    }
  DevMem M;
  double *dw, *part;
  ShellJob* dj;
  const size_t np = (size_t)2 * na * max_planes * (kTruncSteps + 1);
  SPARC_TRY(M.alloc(&dw, W_COUNT, who));
  SPARC_TRY(M.alloc(&dj, jobs.size(), who));
  SPARC_TRY(M.alloc(&part, np, who));
  SPARC_HIP(hipMemcpyAsync(dw, w, sizeof(w), hipMemcpyHostToDevice, s));
  SPARC_HIP(hipMemcpyAsync(dj, jobs.data(), jobs.size() * sizeof(ShellJob), hipMemcpyHostToDevice, s));
  psd_shell_kernel<<<dim3(max_planes, 2 * na), 256, 0, s>>>(dw, grid->n_o, dj, max_planes, part);
  SPARC_TRY(check_launch("psd_shell_kernel"));
  std::vector<double> hp(np);
  SPARC_HIP(hipMemcpyAsync(hp.data(), part, np * sizeof(double), hipMemcpyDeviceToHost, s));
  SPARC_HIP(hipStreamSynchronize(s));
  const double dV = w[W_H] * w[W_H + 1] * w[W_H + 2];
  for (int q = 0; q < 2 * na; ++q) {
    double shell[kTruncSteps + 1] = {};
    for (int pl = 0; pl < max_planes; ++pl)
      for (int t = 0; t <= kTruncSteps; ++t) shell[t] += hp[((size_t)q * max_planes + pl) * (kTruncSteps + 1) + t];
    const double Z = jobs[q].Z;
    double cum = 0.0;
    int found = -1;
    for (int t = 0; t <= kTruncSteps && found < 0; ++t) {
      cum += dV * shell[t];
      if (!std::isfinite(cum)) return fail(SPARC_ENAN, "%s: non-finite pseudocharge", who);
      if (std::fabs(cum + Z) < eps_b * Z) found = t;
    }
    if (found < 0)
      return fail(SPARC_ENOCONV, "%s: atom %d (%s): no box within %d steps meets eps_b=%.3e", who, q / 2,
                  q % 2 ? "reference" : "pseudocharge", kTruncSteps, eps_b);
    for (int d = 0; d < 3; ++d) boxes[6 * (q / 2) + 3 * (q % 2) + d] = jobs[q].m0[d] + found;
  }
  return SPARC_OK;
}

int sparc_pseudocharge(sparc_ctx* ctx, const sparc_grid* grid, const sparc_atoms* atoms, const int32_t* boxes,
                       double* b_dev, double* bref_dev, double* vc_dev, double* energies) {
  const char* who = "sparc_pseudocharge";
  if (!ctx || !b_dev || !bref_dev || !vc_dev || !energies) return fail(SPARC_EINVAL, "%s: null argument", who);
  SPARC_TRY(check_common(grid, atoms, who));
  SPARC_TRY(check_boxes(atoms, boxes, who));
  hipStream_t s = ctx->stream;
  double w[W_COUNT];
  fd_weights(*grid, w);
  std::vector<PsdImage> imgs;
  build_images(*grid, atoms, boxes, imgs);
  const int n1 = grid->n[0], n2 = grid->n[1], n3 = grid->n[2];
  const int nblk = ((n1 + TX - 1) / TX) * ((n2 + TY - 1) / TY) * ((n3 + TZ - 1) / TZ);
  DevMem M;
  double *dw, *part;
  PsdImage* di;
  SPARC_TRY(M.alloc(&dw, W_COUNT, who));
  SPARC_TRY(M.alloc(&di, imgs.size(), who));
  SPARC_TRY(M.alloc(&part, (size_t)3 * nblk, who));
  SPARC_HIP(hipMemcpyAsync(dw, w, sizeof(w), hipMemcpyHostToDevice, s));
  if (!imgs.empty())
    SPARC_HIP(hipMemcpyAsync(di, imgs.data(), imgs.size() * sizeof(PsdImage), hipMemcpyHostToDevice, s));
  const int t = timer_begin(ctx, "psd_grid");
  psd_grid_kernel<<<nblk, 256, 0, s>>>(dw, grid->n_o, n1, n2, n3, di, (int)imgs.size(), b_dev, bref_dev, vc_dev,
                                       part);
  timer_end(ctx, t);
  SPARC_TRY(check_launch("psd_grid_kernel"));
  std::vector<double> hp((size_t)3 * nblk);
  SPARC_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  SPARC_HIP(hipStreamSynchronize(s));
  double S[3] = {0.0, 0.0, 0.0};
  for (int q = 0; q < nblk; ++q)
    for (int d = 0; d < 3; ++d) S[d] += hp[3 * (size_t)q + d];
  const double dV = w[W_H] * w[W_H + 1] * w[W_H + 2];
  const double eself = 0.5 * dV * S[0], eref = 0.5 * dV * S[1];
  energies[0] = eself;
  energies[1] = eref;
  energies[2] = 0.5 * dV * S[2] + eself - eref;
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(energies[d])) return fail(SPARC_ENAN, "%s: non-finite energy", who);
  return SPARC_OK;
}

int sparc_forces_psd(sparc_ctx* ctx, const sparc_grid* grid, const sparc_atoms* atoms, const int32_t* boxes,
                     const double* phi_dev, const double* b_dev, const double* bref_dev, const double* vc_dev,
                     double* Floc_dev, double* Fc_dev) {
  const char* who = "sparc_forces_psd";
  if (!ctx || !phi_dev || !b_dev || !bref_dev || !vc_dev) return fail(SPARC_EINVAL, "%s: null argument", who);
  if (!Floc_dev && !Fc_dev) return SPARC_OK;
  SPARC_TRY(check_common(grid, atoms, who));
  SPARC_TRY(check_boxes(atoms, boxes, who));
  hipStream_t s = ctx->stream;
  double w[W_COUNT];
  fd_weights(*grid, w);
  std::vector<PsdImage> imgs;
  build_images(*grid, atoms, boxes, imgs);
  const int n[3] = {grid->n[0], grid->n[1], grid->n[2]};
  std::vector<ForceJob> jobs;
  for (int q = 0; q < (int)imgs.size(); ++q) {
    ForceJob jb;
    jb.img = q;
    int len[3];
    for (int d = 0; d < 3; ++d) {
      jb.lo[d] = std::max(imgs[q].lo[2][d], 0);
      len[d] = std::min(imgs[q].hi[2][d], n[d] - 1) - jb.lo[d] + 1;
    }
    if (len[0] <= 0 || len[1] <= 0 || len[2] <= 0) continue;
    jb.nx = len[0];
    jb.ny = len[1];
    jb.nz = len[2];
    const int64_t nodes = (int64_t)len[0] * len[1] * len[2];
    for (int64_t c = 0; c * 256 < nodes; ++c) {
      jb.chunk = (int)c;
      jobs.push_back(jb);
    }
  }
  const int na = atoms->n_atoms;
  std::vector<double> F((size_t)6 * na, 0.0);
  DevMem M;
  double *dw, *part, *dF;
  PsdImage* di;
  ForceJob* dj;
  SPARC_TRY(M.alloc(&dw, W_COUNT, who));
  SPARC_TRY(M.alloc(&di, imgs.size(), who));
  SPARC_TRY(M.alloc(&dj, jobs.size(), who));
  SPARC_TRY(M.alloc(&part, (size_t)6 * jobs.size(), who));
  SPARC_TRY(M.alloc(&dF, (size_t)6 * na, who));
  if (!jobs.empty()) {
    SPARC_HIP(hipMemcpyAsync(dw, w, sizeof(w), hipMemcpyHostToDevice, s));
    SPARC_HIP(hipMemcpyAsync(di, imgs.data(), imgs.size() * sizeof(PsdImage), hipMemcpyHostToDevice, s));
    SPARC_HIP(hipMemcpyAsync(dj, jobs.data(), jobs.size() * sizeof(ForceJob), hipMemcpyHostToDevice, s));
    const int t = timer_begin(ctx, "psd_force");
    psd_force_kernel<<<(unsigned)jobs.size(), 256, 0, s>>>(dw, grid->n_o, n[0], n[1], di, dj, phi_dev, b_dev,
                                                           bref_dev, vc_dev, part);
    timer_end(ctx, t);
    SPARC_TRY(check_launch("psd_force_kernel"));
    std::vector<double> hp((size_t)6 * jobs.size());
    SPARC_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    SPARC_HIP(hipStreamSynchronize(s));
    const double dV = w[W_H] * w[W_H + 1] * w[W_H + 2];
    for (size_t q = 0; q < jobs.size(); ++q) {
      const int J = imgs[jobs[q].img].atom;
      for (int d = 0; d < 6; ++d) F[6 * (size_t)J + d] += dV * hp[6 * q + d];
    }
  }
  // F = [atom][loc xyz, c xyz] -> the two outputs
  std::vector<double> out((size_t)6 * na);
  for (int J = 0; J < na; ++J)
    for (int d = 0; d < 3; ++d) {
      out[3 * (size_t)J + d] = F[6 * (size_t)J + d];
      out[3 * (size_t)na + 3 * J + d] = F[6 * (size_t)J + 3 + d];
    }
  for (int d = 0; d < 6 * na; ++d)
    if (!std::isfinite(out[d])) return fail(SPARC_ENAN, "%s: non-finite force", who);
  SPARC_HIP(hipMemcpyAsync(dF, out.data(), out.size() * sizeof(double), hipMemcpyHostToDevice, s));
  if (Floc_dev) add_forces_kernel<<<(3 * na + 255) / 256, 256, 0, s>>>(3 * na, dF, Floc_dev);
  if (Fc_dev) add_forces_kernel<<<(3 * na + 255) / 256, 256, 0, s>>>(3 * na, dF + 3 * na, Fc_dev);
  SPARC_TRY(check_launch("add_forces_kernel"));
  SPARC_HIP(hipStreamSynchronize(s));
  return SPARC_OK;
}

}  // extern "C"
