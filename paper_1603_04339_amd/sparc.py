"""Thin ctypes binding of libsparc_hip (argument marshalling only).

Every function here forwards to the C-ABI entry point of the same name in
include/sparc_hip.h; all arithmetic runs in the library's HIP kernels.  PyTorch
supplies device memory and the stream: orbital blocks are CUDA(HIP) tensors of
shape (n_s, ld) whose row n is orbital n, i.e. exactly the column-major
N_d x n_s block with leading dimension ld that the library expects.

If the shared library has not been built the import fails with an error; there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsparc_hip.so")

OK, EINVAL, ESHAPE, ENOMEM, ENOTSPD, ENOCONV, EDEVICE, ENAN = 0, -1, -2, -3, -4, -5, -6, -7
R64, R32, C128, C64 = 0, 1, 2, 3
GEMM_NATIVE, GEMM_BF16X3, GEMM_BF16X6 = 0, 1, 2
OP_APPLY, OP_FILTER, OP_RR, OP_LANCZOS, OP_FORCES = 0, 1, 2, 3, 4
ELEC_JELLIUM, ELEC_PSEUDOCHARGE = 0, 1

TORCH_DTYPE = {R64: torch.float64, R32: torch.float32, C128: torch.complex128, C64: torch.complex64}


class SparcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class sparc_grid(C.Structure):
    _fields_ = [("n", C.c_int32 * 3), ("L", C.c_double * 3), ("n_o", C.c_int32), ("kpt", C.c_double * 3),
                ("bc", C.c_int32 * 3)]


class sparc_atoms(C.Structure):
    _fields_ = [("n_atoms", C.c_int32), ("R", C.POINTER(C.c_double)), ("vloc_depth", C.POINTER(C.c_double)),
                ("vloc_width", C.POINTER(C.c_double)), ("n_chan", C.c_int32),
                ("chan_atom", C.POINTER(C.c_int32)), ("chan_l", C.POINTER(C.c_int32)),
                ("chan_gamma", C.POINTER(C.c_double)), ("chan_rc", C.POINTER(C.c_double)),
                ("Z", C.POINTER(C.c_double)), ("psd_rc", C.POINTER(C.c_double)),
                ("psd_rc_ref", C.POINTER(C.c_double))]


class sparc_scf_params(C.Structure):
    _fields_ = [("n_s", C.c_int32), ("degree", C.c_int32), ("n_first_passes", C.c_int32),
                ("max_iter", C.c_int32), ("lanczos_steps", C.c_int32), ("mix_history", C.c_int32),
                ("kT", C.c_double), ("mix", C.c_double), ("tol", C.c_double), ("n_elec", C.c_double),
                ("poisson_tol", C.c_double), ("filt", C.c_int), ("rr", C.c_int), ("final_fp64_pass", C.c_int32),
                ("rho_init_dev", C.c_void_p), ("x0_dev", C.c_void_p), ("lanczos_v0_dev", C.c_void_p),
                ("electrostatics", C.c_int32), ("eps_b", C.c_double), ("kerker_k0", C.c_double)]


class sparc_scf_result(C.Structure):
    _fields_ = [("energy", C.c_double), ("mu", C.c_double), ("iterations", C.c_int32), ("converged", C.c_int32),
                ("rho_dev", C.c_void_p), ("ritz_dev", C.c_void_p), ("x_dev", C.c_void_p),
                ("history", C.POINTER(C.c_double)), ("phi_dev", C.c_void_p)]


# entry points: name -> (restype, argtypes)
_SIGS = {
    "sparc_ctx_create": (C.c_int, [C.c_int, C.c_void_p, C.POINTER(C.c_void_p)]),
    "sparc_ctx_destroy": (None, [C.c_void_p]),
    "sparc_ctx_sync": (C.c_int, [C.c_void_p]),
    "sparc_ctx_set_timing": (C.c_int, [C.c_void_p, C.c_int]),
    "sparc_ctx_kernel_time": (C.c_int, [C.c_void_p, C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_int64)]),
    "sparc_last_error": (C.c_char_p, []),
    "sparc_status_string": (C.c_char_p, [C.c_int]),
    "sparc_ham_create": (C.c_int, [C.c_void_p, C.POINTER(sparc_grid), C.POINTER(sparc_atoms), C.c_int,
                                   C.POINTER(C.c_void_p)]),
    "sparc_ham_destroy": (None, [C.c_void_p]),
    "sparc_ham_set_veff": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sparc_ham_get_vloc": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sparc_ham_info": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int64)]),
    "sparc_workspace_bytes": (C.c_size_t, [C.c_void_p, C.c_int32, C.c_int32]),
    "fd_hamiltonian_apply": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64, C.c_int32,
                                       C.c_void_p, C.c_size_t]),
    "fd_hamiltonian_apply_noalloc_max_bytes": (C.c_size_t, []),
    "fd_hamiltonian_apply_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_int64,
                                               C.c_int32]),
    "chebyshev_filter": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_double,
                                   C.c_double, C.c_void_p, C.c_size_t]),
    "rayleigh_ritz": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int, C.c_void_p, C.c_void_p,
                                C.c_size_t, C.POINTER(C.c_int32)]),
    "lanczos_bounds": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t,
                                 C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "density_from_orbitals": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int64),
                                        C.c_int32, C.c_int, C.c_void_p, C.c_int64, C.c_double, C.c_void_p]),
    "sparc_fermi": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.POINTER(C.c_double), C.c_double,
                              C.c_double, C.c_void_p, C.POINTER(C.c_double)]),
    "sparc_stream_triad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int32,
                                     C.POINTER(C.c_double)]),
    "sparc_filter_plan_workspace_bytes": (C.c_size_t, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int32),
                                                        C.POINTER(C.c_int32)]),
    "sparc_filter_plan_create": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                           C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32,
                                           C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)]),
    "sparc_filter_plan_run": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "sparc_filter_plan_destroy": (None, [C.c_void_p]),
    "chebyshev_filter_batched": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                           C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                           C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_void_p, C.c_size_t]),
    "sparc_rr_batched_workspace_bytes": (C.c_size_t, [C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_int32)]),
    "rayleigh_ritz_batched": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(C.c_void_p),
                                        C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.c_int, C.POINTER(C.c_void_p),
                                        C.c_void_p, C.c_size_t]),
    "sparc_ctx_set_autotune": (C.c_int, [C.c_void_p, C.c_int]),
    "sparc_sad_density": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]),
    "sparc_forces_local": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sparc_band_structure": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                                       C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_double, C.c_int32,
                                       C.c_void_p, C.c_void_p]),
    "sparc_dos": (C.c_int, [C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_double,
                            C.c_void_p]),
    "sparc_forces_nonlocal": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_void_p,
                                        C.c_void_p, C.c_size_t]),
    "sparc_psd_boxes": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_void_p]),
    "sparc_pseudocharge": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "sparc_forces_psd": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sparc_dnet_num_params": (C.c_int64, []),
    "sparc_dnet_create": (C.c_int, [C.c_void_p, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_void_p)]),
    "sparc_dnet_destroy": (None, [C.c_void_p]),
    "sparc_dnet_set_precision": (C.c_int, [C.c_void_p, C.c_int32]),
    "sparc_dnet_set_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sparc_dnet_get_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "sparc_dnet_scale_density": (C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_void_p]),
    "sparc_dnet_prepare_input": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_void_p]),
    "sparc_dnet_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p]),
    "sparc_dnet_loss_grad": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.POINTER(C.c_double),
                                       C.c_void_p]),
    "sparc_dnet_adam_step": (C.c_int, [C.c_void_p, C.c_double]),
    "sparc_dnet_train_step": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_double,
                                        C.POINTER(C.c_double)]),
    "sparc_dnet_predict_density": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_double, C.c_double, C.c_double,
                                             C.c_void_p, C.POINTER(C.c_int32)]),
    "sparc_scf_run": (C.c_int, [C.c_void_p, C.POINTER(sparc_grid), C.POINTER(sparc_atoms),
                                C.POINTER(sparc_scf_params), C.POINTER(sparc_scf_result)]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (once) and declare every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1603_04339_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def exported_symbols():
    return list(_SIGS.keys())


def _check(status: int):
    if status != OK:
        raise SparcError(status, load().sparc_last_error().decode())


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _dptr(arr):
    return arr.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(arr):
    return arr.ctypes.data_as(C.POINTER(C.c_int32))


class Context:
    """Device + stream (torch's current stream on that device by default)."""

    def __init__(self, device: int = 0, stream=None):
        lib = load()
        if stream is None:
            stream = torch.cuda.current_stream(device)
        self.stream = stream
        h = C.c_void_p()
        _check(lib.sparc_ctx_create(device, C.c_void_p(stream.cuda_stream), C.byref(h)))
        self.handle = h
        self.device = device

    def sync(self):
        _check(load().sparc_ctx_sync(self.handle))

    def set_timing(self, enable: bool):
        _check(load().sparc_ctx_set_timing(self.handle, int(bool(enable))))

    def kernel_time(self, kernel: str):
        """(total milliseconds, launches) of a named kernel since set_timing."""
        ms, n = C.c_double(), C.c_int64()
        _check(load().sparc_ctx_kernel_time(self.handle, kernel.encode(), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def close(self):
        if self.handle:
            load().sparc_ctx_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def make_grid(n, L, n_o=6, kpt=(0.0, 0.0, 0.0), bc=(0, 0, 0)):
    """Grid struct; bc per direction: 0 Bloch-periodic, 1 zero Dirichlet."""
    g = sparc_grid()
    for s in range(3):
        g.n[s] = int(n[s])
        g.L[s] = float(L[s])
        g.kpt[s] = float(kpt[s])
        g.bc[s] = int(bc[s])
    g.n_o = int(n_o)
    return g


class _Atoms:
    """Keeps the numpy arrays alive while the C struct points at them."""

    def __init__(self, cell):
        self.R = np.ascontiguousarray(cell.positions, dtype=np.float64).reshape(-1)
        self.D = np.ascontiguousarray(cell.depth, dtype=np.float64)
        self.W = np.ascontiguousarray(cell.width, dtype=np.float64)
        self.ca = np.ascontiguousarray(cell.chan_atom, dtype=np.int32)
        self.cl = np.ascontiguousarray(cell.chan_l, dtype=np.int32)
        self.cg = np.ascontiguousarray(cell.chan_gamma, dtype=np.float64)
        self.cr = np.ascontiguousarray(cell.chan_rc, dtype=np.float64)
        self.Z = np.ascontiguousarray(cell.Z, dtype=np.float64)
        prc, prr = getattr(cell, "psd_rc", None), getattr(cell, "psd_rc_ref", None)
        self.prc = None if prc is None else np.ascontiguousarray(prc, dtype=np.float64)
        self.prr = None if prr is None else np.ascontiguousarray(prr, dtype=np.float64)
        a = sparc_atoms()
        a.n_atoms = len(self.D)
        a.R, a.vloc_depth, a.vloc_width = _dptr(self.R), _dptr(self.D), _dptr(self.W)
        a.n_chan = len(self.ca)
        a.chan_atom, a.chan_l = _iptr(self.ca), _iptr(self.cl)
        a.chan_gamma, a.chan_rc, a.Z = _dptr(self.cg), _dptr(self.cr), _dptr(self.Z)
        if self.prc is not None:
            a.psd_rc = _dptr(self.prc)
        if self.prr is not None:
            a.psd_rc_ref = _dptr(self.prr)
        self.struct = a


class Hamiltonian:
    """One (cell, k, dtype) Hamiltonian (sparc_ham)."""

    def __init__(self, ctx: Context, cell, dtype: int = R64, kpt=(0.0, 0.0, 0.0), n_o: int = 6):
        lib = load()
        self.ctx = ctx
        self.dtype = dtype
        self.grid = make_grid(cell.n, cell.L, n_o, kpt, getattr(cell, "bc", (0, 0, 0)))
        self._atoms = _Atoms(cell)
        h = C.c_void_p()
        _check(lib.sparc_ham_create(ctx.handle, C.byref(self.grid), C.byref(self._atoms.struct), dtype, C.byref(h)))
        self.handle = h
        nd, npj, ne = C.c_int64(), C.c_int32(), C.c_int64()
        _check(lib.sparc_ham_info(h, C.byref(nd), C.byref(npj), C.byref(ne)))
        self.n_d, self.n_proj, self.n_entries = nd.value, npj.value, ne.value
        self.dV = float(np.prod([cell.L[s] / cell.n[s] for s in range(3)]))

    def set_veff(self, veff):
        _check(load().sparc_ham_set_veff(self.handle, _ptr(veff)))

    def get_vloc(self, out):
        _check(load().sparc_ham_get_vloc(self.handle, _ptr(out)))
        return out

    def close(self):
        if self.handle:
            load().sparc_ham_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sparc_workspace_bytes(ham: Hamiltonian, n_s: int, op: int) -> int:
    return int(load().sparc_workspace_bytes(ham.handle, n_s, op))


def workspace(ham: Hamiltonian, n_s: int, op: int, device=None):
    nb = max(sparc_workspace_bytes(ham, n_s, op), 256)
    return torch.empty(nb, dtype=torch.uint8, device=device or f"cuda:{ham.ctx.device}")


def _ld(X):
    """Leading dimension of an (n_s, ld) block; a single row's stride is
    arbitrary in torch, its row length is what the library checks."""
    return X.shape[1] if X.shape[0] == 1 else X.stride(0)


def _block(X, ham):
    if X.dtype != TORCH_DTYPE[ham.dtype]:
        raise TypeError(f"block dtype {X.dtype} does not match the Hamiltonian's {TORCH_DTYPE[ham.dtype]}")
    if X.dim() == 1:
        return X, X.shape[0], 1
    if X.stride(1) != 1:
        raise ValueError("orbital blocks must be (n_s, ld) with unit stride along the grid")
    return X, _ld(X), X.shape[0]


def fd_hamiltonian_apply(ham: Hamiltonian, X, Y, work):
    X, ldx, ns = _block(X, ham)
    Y, ldy, _ = _block(Y, ham)
    _check(load().fd_hamiltonian_apply(ham.handle, _ptr(X), ldx, _ptr(Y), ldy, ns, _ptr(work), work.numel()))
    return Y


def fd_hamiltonian_apply_noalloc(ham: Hamiltonian, X, Y):
    X, ldx, ns = _block(X, ham)
    Y, ldy, _ = _block(Y, ham)
    _check(load().fd_hamiltonian_apply_noalloc(ham.handle, _ptr(X), ldx, _ptr(Y), ldy, ns))
    return Y


def noalloc_max_bytes() -> int:
    return int(load().fd_hamiltonian_apply_noalloc_max_bytes())


def chebyshev_filter(ham: Hamiltonian, X, degree: int, lambda_cut: float, lambda_max: float, work):
    X, ldx, ns = _block(X, ham)
    _check(load().chebyshev_filter(ham.handle, _ptr(X), ldx, ns, int(degree), float(lambda_cut),
                                   float(lambda_max), _ptr(work), work.numel()))
    return X


def rayleigh_ritz(ham: Hamiltonian, X, ritz, work, mode: int = GEMM_NATIVE):
    X, ldx, ns = _block(X, ham)
    info = C.c_int32(0)
    st = load().rayleigh_ritz(ham.handle, _ptr(X), ldx, ns, int(mode), _ptr(ritz), _ptr(work), work.numel(),
                              C.byref(info))
    _check(st)
    return ritz


def lanczos_bounds(ham: Hamiltonian, v0, steps: int, work):
    lo, hi = C.c_double(), C.c_double()
    _check(load().lanczos_bounds(ham.handle, _ptr(v0), int(steps), _ptr(work), work.numel(), C.byref(lo),
                                 C.byref(hi)))
    return lo.value, hi.value


def forces_local(ham: Hamiltonian, rho, F):
    """Adds the local force component (Ha/bohr) to F, a device FP64 tensor of shape
    (n_atoms, 3); rho: device FP64 density [N_d]."""
    _check(load().sparc_forces_local(ham.handle, _ptr(rho), _ptr(F)))
    return F


def forces_nonlocal(ham: Hamiltonian, X, occ_w, F, work):
    """Adds the non-local force component of the block X (n_s, ld) with weights occ_w
    (device FP64 [n_s], w_b g_nb) to F; work: workspace(ham, n_s, OP_FORCES)."""
    X, ldx, ns = _block(X, ham)
    _check(load().sparc_forces_nonlocal(ham.handle, _ptr(X), ldx, ns, _ptr(occ_w), _ptr(F), _ptr(work),
                                        work.numel()))
    return F


def density_from_orbitals(ctx: Context, Xs, occ_w, dV: float, rho, dtype: int):
    nk = len(Xs)
    ptrs = (C.c_void_p * nk)(*[X.data_ptr() for X in Xs])
    lds = (C.c_int64 * nk)(*[_ld(X) for X in Xs])
    ns = Xs[0].shape[0]
    nd = Xs[0].shape[1]
    _check(load().density_from_orbitals(ctx.handle, nk, ptrs, lds, ns, dtype, _ptr(occ_w), nd, float(dV),
                                        _ptr(rho)))
    return rho


def sparc_fermi(ctx: Context, lam, wk, n_elec: float, kT: float, occ_w=None):
    nk, ns = lam.shape
    w = np.ascontiguousarray(wk, dtype=np.float64)
    mu = C.c_double()
    _check(load().sparc_fermi(ctx.handle, nk, ns, _ptr(lam), _dptr(w), float(n_elec), float(kT), _ptr(occ_w),
                              C.byref(mu)))
    return mu.value


def stream_triad(ctx: Context, a, b, c, reps: int = 10) -> float:
    """sparc_stream_triad on three equal FP64 device tensors; returns ms per launch."""
    ms = C.c_double()
    _check(load().sparc_stream_triad(ctx.handle, _ptr(a), _ptr(b), _ptr(c), a.numel(), int(reps), C.byref(ms)))
    return ms.value


def _arr(ctype, vals):
    return (ctype * len(vals))(*vals)


def _batch_args(hams, Xs, n_s, degree=None):
    H = _arr(C.c_void_p, [h.handle.value for h in hams])
    X = _arr(C.c_void_p, [x.data_ptr() for x in Xs])
    ld = _arr(C.c_int64, [_ld(x) for x in Xs])
    ns = _arr(C.c_int32, list(n_s))
    dg = _arr(C.c_int32, list(degree)) if degree is not None else None
    return H, X, ld, ns, dg


class FilterPlan:
    """Batched Chebyshev filter over several problems (sparc_filter_plan)."""

    def __init__(self, ctx: Context, hams, Xs, degree, use_graph: bool = True):
        lib = load()
        for h, x in zip(hams, Xs):
            _block(x, h)
        n_s = [x.shape[0] for x in Xs]
        self._args = _batch_args(hams, Xs, n_s, degree)
        H, X, ld, ns, dg = self._args
        nb = lib.sparc_filter_plan_workspace_bytes(len(hams), H, ns, dg)
        self.work = torch.empty(max(int(nb), 256), dtype=torch.uint8, device=f"cuda:{ctx.device}")
        h = C.c_void_p()
        _check(lib.sparc_filter_plan_create(ctx.handle, len(hams), H, X, ld, ns, dg, int(use_graph),
                                            _ptr(self.work), self.work.numel(), C.byref(h)))
        self.handle = h
        self.n = len(hams)
        self._keep = (list(hams), list(Xs))   # the plan holds raw pointers into these

    def run(self, lambda_cut, lambda_max):
        lc = _arr(C.c_double, [float(v) for v in lambda_cut])
        lm = _arr(C.c_double, [float(v) for v in lambda_max])
        _check(load().sparc_filter_plan_run(self.handle, lc, lm))

    def close(self):
        if self.handle:
            load().sparc_filter_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def chebyshev_filter_batched(ctx: Context, hams, Xs, degree, lambda_cut, lambda_max):
    lib = load()
    n_s = [x.shape[0] for x in Xs]
    H, X, ld, ns, dg = _batch_args(hams, Xs, n_s, degree)
    nb = lib.sparc_filter_plan_workspace_bytes(len(hams), H, ns, dg)
    work = torch.empty(max(int(nb), 256), dtype=torch.uint8, device=f"cuda:{ctx.device}")
    _check(lib.chebyshev_filter_batched(ctx.handle, len(hams), H, X, ld, ns, dg,
                                        _arr(C.c_double, [float(v) for v in lambda_cut]),
                                        _arr(C.c_double, [float(v) for v in lambda_max]), _ptr(work), work.numel()))


def rr_batched_workspace(ctx: Context, hams, Xs):
    n_s = [x.shape[0] for x in Xs]
    H, _, _, ns, _ = _batch_args(hams, Xs, n_s)
    nb = load().sparc_rr_batched_workspace_bytes(len(hams), H, ns)
    return torch.empty(max(int(nb), 256), dtype=torch.uint8, device=f"cuda:{ctx.device}")


def rayleigh_ritz_batched(ctx: Context, hams, Xs, ritz, mode: int = GEMM_NATIVE, work=None):
    lib = load()
    n_s = [x.shape[0] for x in Xs]
    H, X, ld, ns, _ = _batch_args(hams, Xs, n_s)
    if work is None:
        work = rr_batched_workspace(ctx, hams, Xs)
    R = _arr(C.c_void_p, [r.data_ptr() for r in ritz])
    _check(lib.rayleigh_ritz_batched(ctx.handle, len(hams), H, X, ld, ns, int(mode), R, _ptr(work), work.numel()))


def set_autotune(ctx: Context, enable: bool):
    _check(load().sparc_ctx_set_autotune(ctx.handle, int(bool(enable))))


def sparc_scf_run(ctx: Context, cell, params: dict, rho_out, ritz_out, x_out=None, n_o: int = 6, phi_out=None):
    """Minimal SCF through the library; params keys follow sparc_scf_params.
    phi_out (optional device FP64 [N_d]) receives V_H or phi of the final density."""
    lib = load()
    grid = make_grid(cell.n, cell.L, n_o, bc=getattr(cell, "bc", (0, 0, 0)))
    atoms = _Atoms(cell)
    p = sparc_scf_params()
    for k, v in params.items():
        if k.endswith("_dev"):
            setattr(p, k, C.c_void_p(v.data_ptr()) if v is not None else None)
        else:
            setattr(p, k, v)
    res = sparc_scf_result()
    res.rho_dev = C.c_void_p(rho_out.data_ptr())
    res.ritz_dev = C.c_void_p(ritz_out.data_ptr())
    res.x_dev = C.c_void_p(x_out.data_ptr()) if x_out is not None else None
    res.phi_dev = C.c_void_p(phi_out.data_ptr()) if phi_out is not None else None
    hist = np.zeros(3 * max(1, params.get("max_iter", 1)))
    res.history = _dptr(hist)
    st = lib.sparc_scf_run(ctx.handle, C.byref(grid), C.byref(atoms.struct), C.byref(p), C.byref(res))
    out = {"energy": res.energy, "mu": res.mu, "iterations": res.iterations, "converged": bool(res.converged),
           "history": hist[:3 * max(res.iterations, 0)].reshape(-1, 3), "status": st}
    if st not in (OK, ENOCONV):
        _check(st)
    return out


def band_structure(ctx: Context, cell, veff, kpts, Xs, n_bands: int, degree: int = 20, max_passes: int = 50,
                   tol: float = 1e-8, use_graph: bool = True, n_o: int = 6):
    """Band structure at fixed potential (sparc_band_structure).  veff: device FP64
    [N_d]; kpts: (n_k, 3); Xs: list of n_k device complex128 (n_s, N_d) start blocks,
    overwritten by the Ritz vectors.  Returns (eig (n_k, n_bands), passes (n_k,),
    status) where status is OK or ENOCONV."""
    lib = load()
    grid = make_grid(cell.n, cell.L, n_o, bc=getattr(cell, "bc", (0, 0, 0)))
    atoms = _Atoms(cell)
    k = np.ascontiguousarray(kpts, dtype=np.float64).reshape(-1, 3)
    nk = k.shape[0]
    if len(Xs) != nk:
        raise ValueError("one start block per k-point")
    for X in Xs:
        if X.dtype != torch.complex128 or not X.is_contiguous() or X.shape[1] != cell.n_d:
            raise ValueError("start blocks must be contiguous complex128 (n_s, N_d)")
    ns = int(Xs[0].shape[0])
    ptrs = (C.c_void_p * nk)(*[X.data_ptr() for X in Xs])
    eig = np.zeros((nk, n_bands))
    passes = np.zeros(nk, dtype=np.int32)
    st = lib.sparc_band_structure(ctx.handle, C.byref(grid), C.byref(atoms.struct), _ptr(veff), nk, _dptr(k),
                                  ptrs, ns, int(n_bands), int(degree), int(max_passes), float(tol),
                                  1 if use_graph else 0, _dptr(eig), passes.ctypes.data_as(C.c_void_p))
    if st not in (OK, ENOCONV):
        _check(st)
    return eig, passes, st


def dos(eig, wk, energies, sigma: float):
    """Density of states D(E) (sparc_dos, host computation)."""
    eig = np.ascontiguousarray(eig, dtype=np.float64)
    wk = np.ascontiguousarray(wk, dtype=np.float64)
    E = np.ascontiguousarray(energies, dtype=np.float64)
    out = np.zeros(E.shape[0])
    _check(load().sparc_dos(eig.shape[0], eig.shape[1], _dptr(eig), _dptr(wk), E.shape[0], _dptr(E), float(sigma),
                            _dptr(out)))
    return out


def psd_boxes(ctx: Context, cell, eps_b: float = 1e-8, n_o: int = 6):
    """Truncation boxes of the pseudocharges (sparc_psd_boxes): int32 (n_atoms, 6),
    half-widths in nodes (pseudocharge x, y, z, then reference x, y, z)."""
    grid = make_grid(cell.n, cell.L, n_o, bc=getattr(cell, "bc", (0, 0, 0)))
    atoms = _Atoms(cell)
    out = np.zeros((cell.n_atoms, 6), dtype=np.int32)
    _check(load().sparc_psd_boxes(ctx.handle, C.byref(grid), C.byref(atoms.struct), float(eps_b),
                                  out.ctypes.data_as(C.c_void_p)))
    return out


def pseudocharge(ctx: Context, cell, boxes, n_o: int = 6):
    """Algorithm 1 and E_c (sparc_pseudocharge).  Returns dict(b, bref, vc: device FP64
    [N_d]; eself, eself_ref, ec: floats)."""
    grid = make_grid(cell.n, cell.L, n_o, bc=getattr(cell, "bc", (0, 0, 0)))
    atoms = _Atoms(cell)
    bx = np.ascontiguousarray(boxes, dtype=np.int32)
    out = {k: torch.zeros(cell.n_d, dtype=torch.float64, device=f"cuda:{ctx.device}") for k in ("b", "bref", "vc")}
    en = np.zeros(3)
    _check(load().sparc_pseudocharge(ctx.handle, C.byref(grid), C.byref(atoms.struct), bx.ctypes.data_as(C.c_void_p),
                                     _ptr(out["b"]), _ptr(out["bref"]), _ptr(out["vc"]), _dptr(en)))
    out.update(eself=float(en[0]), eself_ref=float(en[1]), ec=float(en[2]))
    return out


def forces_psd(ctx: Context, cell, boxes, phi, st, Floc=None, Fc=None, n_o: int = 6):
    """Adds the local and overlap-correction force components with pseudocharges
    (sparc_forces_psd) to Floc and Fc (device FP64 (n_atoms, 3), either may be None);
    st: the dict of pseudocharge() for the same boxes."""
    grid = make_grid(cell.n, cell.L, n_o, bc=getattr(cell, "bc", (0, 0, 0)))
    atoms = _Atoms(cell)
    bx = np.ascontiguousarray(boxes, dtype=np.int32)
    _check(load().sparc_forces_psd(ctx.handle, C.byref(grid), C.byref(atoms.struct), bx.ctypes.data_as(C.c_void_p),
                                   _ptr(phi), _ptr(st["b"]), _ptr(st["bref"]), _ptr(st["vc"]), _ptr(Floc), _ptr(Fc)))


def sad_density(ctx: Context, cell, rho_out, n_o: int = 6):
    """Atomic-superposition density of a cell into rho_out (device FP64, N_d)."""
    grid = make_grid(cell.n, cell.L, n_o, bc=getattr(cell, "bc", (0, 0, 0)))
    atoms = _Atoms(cell)
    _check(load().sparc_sad_density(ctx.handle, C.byref(grid), C.byref(atoms.struct), float(cell.n_elec),
                                    _ptr(rho_out)))
    return rho_out


class DensityNet:
    """Learned initial density (sparc_dnet): FP32 3-D conv net on one grid shape."""

    def __init__(self, ctx: Context, n, max_batch: int = 1):
        lib = load()
        self.ctx = ctx
        self.n = tuple(int(v) for v in n)
        self.n_d = self.n[0] * self.n[1] * self.n[2]
        self.num_params = int(lib.sparc_dnet_num_params())
        h = C.c_void_p()
        _check(lib.sparc_dnet_create(ctx.handle, (C.c_int32 * 3)(*self.n), int(max_batch), C.byref(h)))
        self.handle = h

    def set_params(self, theta):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        if t.size != self.num_params:
            raise ValueError(f"expected {self.num_params} parameters, got {t.size}")
        _check(load().sparc_dnet_set_params(self.handle, t.ctypes.data_as(C.c_void_p)))

    def set_bf16(self, enable: bool):
        """bfloat16 inference (activations and weights), FP32 sums; training stays FP32."""
        _check(load().sparc_dnet_set_precision(self.handle, 1 if enable else 0))

    def get_params(self):
        t = np.zeros(self.num_params, dtype=np.float32)
        _check(load().sparc_dnet_get_params(self.handle, t.ctypes.data_as(C.c_void_p)))
        return t

    def scale_density(self, rho, n_elec: float, dV: float, x_out):
        _check(load().sparc_dnet_scale_density(self.handle, _ptr(rho), float(n_elec), float(dV), _ptr(x_out)))
        return x_out

    def prepare_input(self, rho_sad, vloc, n_elec: float, dV: float, in_out):
        """in_out (FP32, N_d x 2) = (rho_sad / rho_bar, -vloc)."""
        _check(load().sparc_dnet_prepare_input(self.handle, _ptr(rho_sad), _ptr(vloc), float(n_elec), float(dV),
                                               _ptr(in_out)))
        return in_out

    def forward(self, x, d_out):
        B = x.numel() // (2 * self.n_d)
        _check(load().sparc_dnet_forward(self.handle, _ptr(x), B, _ptr(d_out)))
        return d_out

    def loss_grad(self, x, y, want_grad: bool = True):
        B = y.numel() // self.n_d
        loss = C.c_double()
        g = np.zeros(self.num_params, dtype=np.float32) if want_grad else None
        _check(load().sparc_dnet_loss_grad(self.handle, _ptr(x), _ptr(y), B, C.byref(loss),
                                           g.ctypes.data_as(C.c_void_p) if want_grad else None))
        return loss.value, g

    def adam_step(self, lr: float):
        _check(load().sparc_dnet_adam_step(self.handle, float(lr)))

    def train_step(self, x, y, lr: float):
        B = y.numel() // self.n_d
        loss = C.c_double()
        _check(load().sparc_dnet_train_step(self.handle, _ptr(x), _ptr(y), B, float(lr), C.byref(loss)))
        return loss.value

    def predict_density(self, rho_sad, vloc, n_elec: float, dV: float, rho_out, charge_tol: float = 1e-2):
        used = C.c_int32()
        _check(load().sparc_dnet_predict_density(self.handle, _ptr(rho_sad), _ptr(vloc), float(n_elec), float(dV),
                                                 float(charge_tol), _ptr(rho_out), C.byref(used)))
        return bool(used.value)

    def close(self):
        if self.handle:
            load().sparc_dnet_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
