// H X without any device allocation: the projections of X (the only scratch the
// product needs beyond its input and output) live in a fixed device array of this
// library instead of a caller workspace.  Each device holds its own copy of the array;
// its address on a device is looked up once, when the first context on that device is
// created, and every later call on that device reuses it.
#include <mutex>

#include "internal.hpp"

namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;  // projections of at most 16 MiB
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

namespace sparc {

// with `device` current: the device address of its copy of the scratch array
int noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices)
    return fail(SPARC_EDEVICE, "static scratch: device %d beyond the %d supported", device, kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return SPARC_OK;
  void* p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(SPARC_EDEVICE, "static scratch: hipGetSymbolAddress failed on device %d (%s)", device,
                hipGetErrorString(e));
  g_scratch_ptr[device] = p;
  return SPARC_OK;
}

}  // namespace sparc

using namespace sparc;

extern "C" {

size_t fd_hamiltonian_apply_noalloc_max_bytes(void) { return kScratchBytes; }

int fd_hamiltonian_apply_noalloc(sparc_ham* H, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t n_s) {
  SPARC_TRY(check_ham(H, "fd_hamiltonian_apply_noalloc"));
  SPARC_TRY(check_block(H, X, ldx, n_s, "fd_hamiltonian_apply_noalloc"));
  SPARC_TRY(check_block(H, Y, ldy, n_s, "fd_hamiltonian_apply_noalloc"));
  if (X == Y) return fail(SPARC_EINVAL, "fd_hamiltonian_apply_noalloc: X and Y must not alias");
  const int dev = H->ctx->device;
  void* work = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (dev >= 0 && dev < kMaxDevices) work = g_scratch_ptr[dev];
  }
  if (!work) return fail(SPARC_EDEVICE, "fd_hamiltonian_apply_noalloc: no static scratch on device %d", dev);
  const size_t need = sparc_workspace_bytes(H, n_s, SPARC_OP_APPLY);
  if (H->n_proj > 0 && need > kScratchBytes)
    return fail(SPARC_ENOMEM,
                "fd_hamiltonian_apply_noalloc: the projections of %d states need %zu bytes, more than the %zu bytes "
                "of static scratch (use fd_hamiltonian_apply with a workspace)",
                n_s, need, kScratchBytes);
  SPARC_TRY(nl_project(H, X, ldx, n_s, work));
  return ham_step(H, X, ldx, nullptr, 0, Y, ldy, n_s, 1.0, 0.0, 0.0, work, STEP_NO_TUNE);
}

}  // extern "C"
