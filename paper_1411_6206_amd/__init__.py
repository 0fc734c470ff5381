"""Python binding of libprior_ls.so, the MI355X (gfx950) Priori L+S reconstruction library.

Argument marshalling only: every step of the iteration runs in the library's HIP
kernels.  PyTorch provides device memory (tensors) and the HIP stream.  The names
mirror the C ABI in include/prior_ls.h:

    h = PriorLS(nx, ny, nz, nt, nc, wavelet_levels=2)     # prior_ls_create
    out, stats = h.solve(kspace, mask, sens, prior_w, ...)  # prior_ls_solve
    out, stats = h.step(n)                                  # prior_ls_step
    h.close()                                               # prior_ls_destroy

If the shared library has not been built, importing works but every call raises
LibraryMissing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libprior_ls.so")

OK, EINVAL, ESHAPE, ENOMEM, EHIP, ENONFINITE = 0, -1, -2, -3, -4, -5
GRAM_MODES = {"fp64": 0, "fp32": 1, "bf16x3": 2}
MAX_NT = 32

# every symbol include/prior_ls.h declares
EXPORTS = ("prior_ls_create", "prior_ls_solve", "prior_ls_step", "prior_ls_destroy",
           "prior_ls_strerror", "prior_ls_last_error", "prior_ls_plan_bytes",
           "prior_ls_op_dc", "prior_ls_op_svt", "prior_ls_op_sparse", "prior_ls_step_timed",
           "prior_ls_append")
NKERNELS = 7
KERNEL_NAMES = ("gram", "gram_reduce", "eig", "sparse", "backproject", "data_consistency", "stats")


class LibraryMissing(RuntimeError):
    pass


class PriorLSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class Dims(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("nx", C.c_int32), ("ny", C.c_int32),
                ("nz", C.c_int32), ("nt", C.c_int32), ("nc", C.c_int32),
                ("wavelet_levels", C.c_int32), ("gram_mode", C.c_int32),
                ("reserved", C.c_int32), ("hbm_budget", C.c_uint64)]


class Params(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("lambda_L", C.c_double), ("lambda_S", C.c_double),
                ("lambda_p", C.c_double), ("tol", C.c_double), ("lambda_L_relative", C.c_int32),
                ("max_iter", C.c_int32), ("check_every", C.c_int32), ("use_graph", C.c_int32)]


class Inputs(C.Structure):
    _fields_ = [("kspace", C.c_void_p), ("mask", C.c_void_p), ("sens", C.c_void_p),
                ("prior_w", C.c_void_p), ("sigma_prev", C.POINTER(C.c_double)),
                ("L0", C.c_void_p), ("S0", C.c_void_p)]


class Outputs(C.Structure):
    _fields_ = [("L", C.c_void_p), ("S", C.c_void_p), ("X", C.c_void_p), ("M", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("iters", C.c_int32), ("converged", C.c_int32),
                ("nonfinite", C.c_int32), ("sigma_count", C.c_int32),
                ("eig_sweeps", C.c_int32), ("reserved", C.c_int32),
                ("rel_change", C.c_double), ("resid_norm", C.c_double),
                ("nuclear_norm", C.c_double), ("l1_weighted", C.c_double),
                ("objective", C.c_double), ("tau_L", C.c_double),
                ("sigma", C.c_double * MAX_NT), ("ms", C.c_double)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_
             if k not in ("sigma", "struct_size", "reserved")}
        d["sigma"] = list(self.sigma)[: self.sigma_count]
        return d


_lib = None


def lib():
    """Load libprior_ls.so (raises LibraryMissing if it was never built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} is not built; run paper_1411_6206_amd.build.build()")
    L = C.CDLL(LIB_PATH)
    H = C.c_void_p
    L.prior_ls_create.argtypes = [C.POINTER(Dims), C.c_void_p, C.POINTER(H)]
    L.prior_ls_create.restype = C.c_int
    L.prior_ls_solve.argtypes = [H, C.POINTER(Inputs), C.POINTER(Params), C.POINTER(Outputs),
                                 C.POINTER(Stats)]
    L.prior_ls_solve.restype = C.c_int
    L.prior_ls_step.argtypes = [H, C.c_int32, C.POINTER(Outputs), C.POINTER(Stats)]
    L.prior_ls_step.restype = C.c_int
    L.prior_ls_destroy.argtypes = [H]
    L.prior_ls_destroy.restype = None
    L.prior_ls_strerror.argtypes = [C.c_int]
    L.prior_ls_strerror.restype = C.c_char_p
    L.prior_ls_last_error.argtypes = [H]
    L.prior_ls_last_error.restype = C.c_char_p
    L.prior_ls_plan_bytes.argtypes = [C.POINTER(Dims)]
    L.prior_ls_plan_bytes.restype = C.c_uint64
    L.prior_ls_op_dc.argtypes = [H, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]
    L.prior_ls_op_dc.restype = C.c_int
    L.prior_ls_op_svt.argtypes = [H, C.c_void_p, C.c_void_p, C.POINTER(C.c_double)]
    L.prior_ls_op_svt.restype = C.c_int
    L.prior_ls_op_sparse.argtypes = [H, C.c_void_p, C.c_void_p, C.c_void_p]
    L.prior_ls_op_sparse.restype = C.c_int
    L.prior_ls_step_timed.argtypes = [H, C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                      C.POINTER(Stats)]
    L.prior_ls_step_timed.restype = C.c_int
    L.prior_ls_append.argtypes = [H, C.c_void_p, C.c_void_p, C.POINTER(Params),
                                  C.POINTER(Outputs), C.POINTER(Stats)]
    L.prior_ls_append.restype = C.c_int
    _lib = L
    return L


def make_dims(nx, ny, nz, nt, nc, wavelet_levels=2, gram_mode="fp64", hbm_budget=0):
    gm = GRAM_MODES[gram_mode] if isinstance(gram_mode, str) else int(gram_mode)
    return Dims(C.sizeof(Dims), nx, ny, nz, nt, nc, wavelet_levels, gm, 0, hbm_budget)


def plan_bytes(nx, ny, nz, nt, nc, wavelet_levels=2, gram_mode="fp64"):
    d = make_dims(nx, ny, nz, nt, nc, wavelet_levels, gram_mode)
    return int(lib().prior_ls_plan_bytes(C.byref(d)))


def strerror(status):
    return lib().prior_ls_strerror(status).decode()


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensors must be contiguous")
    return C.c_void_p(t.data_ptr())


def _current_stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class PriorLS:
    """One problem geometry (prior_ls_create); owns the device state until close()."""

    def __init__(self, nx, ny, nz, nt, nc, wavelet_levels=2, gram_mode="fp64",
                 hbm_budget=0, stream=None):
        L = lib()
        self._h = C.c_void_p()
        self.dims = make_dims(nx, ny, nz, nt, nc, wavelet_levels, gram_mode, hbm_budget)
        self.shape = (nt, nz, ny, nx)
        st = _current_stream() if stream is None else C.c_void_p(stream)
        rc = L.prior_ls_create(C.byref(self.dims), st, C.byref(self._h))
        if rc != OK:
            raise PriorLSError(rc, f"prior_ls_create: {L.prior_ls_last_error(None).decode()}")

    def _check(self, rc, what):
        if rc != OK:
            raise PriorLSError(rc, f"{what}: {lib().prior_ls_last_error(self._h).decode()}")

    def _outputs(self, want: Sequence[str]):
        import torch
        outs = {k: torch.empty(self.shape, dtype=torch.complex64, device="cuda") for k in want}
        o = Outputs(*(_ptr(outs.get(k)) for k in ("L", "S", "X", "M")))
        return outs, o

    def solve(self, kspace, mask, sens=None, prior_w=None, sigma_prev=None, L0=None, S0=None,
              lambda_L=0.01, lambda_S=0.01, lambda_p=0.0, lambda_L_relative=True, max_iter=50,
              tol=0.0, check_every=10, use_graph=True, outputs=("L", "S", "X", "M")):
        """prior_ls_solve.  Tensors: complex64 / uint8 CUDA tensors in the ABI layouts."""
        import torch
        sp = None
        if sigma_prev is not None:
            vals = [float(v) for v in sigma_prev]
            sp = (C.c_double * len(vals))(*vals)
        ins = Inputs(_ptr(kspace), _ptr(mask), _ptr(sens), _ptr(prior_w),
                     C.cast(sp, C.POINTER(C.c_double)) if sp is not None else None,
                     _ptr(L0), _ptr(S0))
        prm = Params(C.sizeof(Params), float(lambda_L), float(lambda_S), float(lambda_p),
                     float(tol), 1 if lambda_L_relative else 0, int(max_iter), int(check_every),
                     1 if use_graph else 0)
        outs, o = self._outputs(outputs)
        st = Stats()
        st.struct_size = C.sizeof(Stats)
        rc = lib().prior_ls_solve(self._h, C.byref(ins), C.byref(prm), C.byref(o), C.byref(st))
        torch.cuda.current_stream().synchronize()
        self._check(rc, "prior_ls_solve")
        return outs, st.as_dict()

    def append(self, kspace_frame, mask_frame, lambda_L=0.01, lambda_S=0.01, lambda_p=0.0,
               lambda_L_relative=True, max_iter=20, tol=0.0, check_every=10, use_graph=True,
               outputs=("L", "S", "X", "M")):
        """prior_ls_append: slide the window by one frame (kspace_frame complex64
        [nc][nz][ny][nx], mask_frame uint8 [nz][ny]) and iterate with the previous window's
        support and singular values as a-priori knowledge."""
        import torch
        prm = Params(C.sizeof(Params), float(lambda_L), float(lambda_S), float(lambda_p),
                     float(tol), 1 if lambda_L_relative else 0, int(max_iter), int(check_every),
                     1 if use_graph else 0)
        outs, o = self._outputs(outputs)
        st = Stats()
        st.struct_size = C.sizeof(Stats)
        rc = lib().prior_ls_append(self._h, _ptr(kspace_frame), _ptr(mask_frame), C.byref(prm),
                                   C.byref(o), C.byref(st))
        torch.cuda.current_stream().synchronize()
        self._check(rc, "prior_ls_append")
        return outs, st.as_dict()

    def step(self, n_iter, outputs=("L", "S", "X", "M")):
        """prior_ls_step: continue the resident iteration."""
        outs, o = self._outputs(outputs)
        st = Stats()
        st.struct_size = C.sizeof(Stats)
        rc = lib().prior_ls_step(self._h, int(n_iter), C.byref(o), C.byref(st))
        self._check(rc, "prior_ls_step")
        return outs, st.as_dict()

    def step_timed(self, n_iter):
        """prior_ls_step_timed: n_iter iterations with per-kernel hipEvent timing.
        Returns ({kernel name: summed ms}, stats)."""
        ms = (C.c_double * NKERNELS)()
        cnt = (C.c_int32 * NKERNELS)()
        st = Stats()
        st.struct_size = C.sizeof(Stats)
        rc = lib().prior_ls_step_timed(self._h, int(n_iter), ms, cnt, C.byref(st))
        self._check(rc, "prior_ls_step_timed")
        return {k: ms[i] for i, k in enumerate(KERNEL_NAMES)}, st.as_dict()

    def op_dc(self, Y):
        """prior_ls_op_dc: M = Y - A^H(A(Y) - d), step (4)."""
        import torch
        M = torch.empty_like(Y)
        r = C.c_double()
        self._check(lib().prior_ls_op_dc(self._h, _ptr(Y), _ptr(M), C.byref(r)), "prior_ls_op_dc")
        return M, r.value

    def op_svt(self, Cmat):
        """prior_ls_op_svt: steps (1)-(2) on the Casorati matrix of Cmat."""
        import torch
        Lout = torch.empty_like(Cmat)
        sig = (C.c_double * MAX_NT)()
        self._check(lib().prior_ls_op_svt(self._h, _ptr(Cmat), _ptr(Lout), sig), "prior_ls_op_svt")
        return Lout, list(sig)[: self.shape[0]]

    def op_sparse(self, Xm, Lp):
        """prior_ls_op_sparse: S = T^-1 soft(T(Xm - Lp), lambda_S (1 - w)), step (3)."""
        import torch
        S = torch.empty_like(Xm)
        self._check(lib().prior_ls_op_sparse(self._h, _ptr(Xm), _ptr(Lp), _ptr(S)),
                    "prior_ls_op_sparse")
        return S

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().prior_ls_destroy(self._h)
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_device(problem, device="cuda"):
    """Device tensors of a synthetic problem (complex64 / uint8) in the ABI layouts."""
    import torch
    import numpy as np

    def c64(a):
        return None if a is None else torch.from_numpy(np.ascontiguousarray(a, np.complex64)).to(device)

    def u8(a):
        return None if a is None else torch.from_numpy(np.ascontiguousarray(a, np.uint8)).to(device)

    return dict(kspace=c64(problem.kspace), mask=u8(problem.mask), sens=c64(problem.sens),
                prior_w=u8(problem.prior_w))
