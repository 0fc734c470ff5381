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
TRANSFORMS = {"haar": 0, "tfft": 1, "db4": 2}
MAX_NT = 64

# every symbol include/prior_ls.h declares
EXPORTS = ("prior_ls_create", "prior_ls_solve", "prior_ls_step", "prior_ls_destroy",
           "prior_ls_strerror", "prior_ls_last_error", "prior_ls_plan_bytes",
           "prior_ls_op_dc", "prior_ls_op_svt", "prior_ls_op_sparse", "prior_ls_step_timed",
           "prior_ls_append", "prior_ls_server_create", "prior_ls_server_submit",
           "prior_ls_server_wait", "prior_ls_server_info", "prior_ls_server_destroy",
           "prior_ls_tune", "prior_ls_set_tuning", "prior_ls_get_tuning",
           "prior_ls_batch_create", "prior_ls_batch_solve", "prior_ls_batch_step",
           "prior_ls_batch_last_error", "prior_ls_batch_destroy", "prior_ls_svt_noalloc")
NKERNELS = 8
KERNEL_NAMES = ("gram", "gram_reduce", "eig", "sparse", "backproject", "data_consistency", "stats",
                "change")


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
                ("transform", C.c_int32), ("hbm_budget", C.c_uint64)]


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


class Tuning(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("gram_blocks", C.c_int32), ("bp_grid", C.c_int32),
                ("sparse_fork", C.c_int32), ("sparse_grid", C.c_int32),
                ("ms_per_iteration", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_
                if k not in ("struct_size",)}


class ServerConfig(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("hbm_budget", C.c_uint64),
                ("max_active", C.c_int32), ("reserved", C.c_int32)]


class Request(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("dims", Dims), ("first", Params), ("next", Params),
                ("n_append", C.c_int32), ("reserved", C.c_int32),
                ("kspace0", C.c_void_p), ("mask0", C.c_void_p),
                ("kspace_frames", C.c_void_p), ("mask_frames", C.c_void_p),
                ("sens", C.c_void_p), ("out", Outputs), ("stats", C.POINTER(Stats)),
                ("latency_ms", C.POINTER(C.c_double))]


class Result(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("status", C.c_int32), ("reused_plan", C.c_int32),
                ("queue_ms", C.c_double), ("run_ms", C.c_double), ("total_ms", C.c_double),
                ("state_bytes", C.c_uint64), ("message", C.c_char * 160)]


class ServerStats(C.Structure):
    _fields_ = [("struct_size", C.c_size_t), ("budget", C.c_uint64), ("used", C.c_uint64),
                ("peak_used", C.c_uint64), ("submitted", C.c_int64), ("completed", C.c_int64),
                ("failed", C.c_int64), ("reused", C.c_int64), ("evicted", C.c_int64),
                ("queued", C.c_int32), ("active", C.c_int32), ("peak_active", C.c_int32),
                ("resident_idle", C.c_int32)]


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
    L.prior_ls_tune.argtypes = [H, C.POINTER(Inputs), C.POINTER(Params), C.POINTER(Tuning)]
    L.prior_ls_tune.restype = C.c_int
    L.prior_ls_set_tuning.argtypes = [H, C.POINTER(Tuning)]
    L.prior_ls_set_tuning.restype = C.c_int
    L.prior_ls_get_tuning.argtypes = [H, C.POINTER(Tuning)]
    L.prior_ls_get_tuning.restype = C.c_int
    B = C.c_void_p
    L.prior_ls_batch_create.argtypes = [C.POINTER(H), C.c_int32, C.POINTER(B)]
    L.prior_ls_batch_create.restype = C.c_int
    L.prior_ls_batch_solve.argtypes = [B, C.POINTER(Inputs), C.POINTER(Params), C.POINTER(Outputs),
                                       C.POINTER(Stats)]
    L.prior_ls_batch_solve.restype = C.c_int
    L.prior_ls_batch_step.argtypes = [B, C.c_int32, C.POINTER(Outputs), C.POINTER(Stats)]
    L.prior_ls_batch_step.restype = C.c_int
    L.prior_ls_batch_last_error.argtypes = [B]
    L.prior_ls_batch_last_error.restype = C.c_char_p
    L.prior_ls_batch_destroy.argtypes = [B]
    L.prior_ls_batch_destroy.restype = None
    L.prior_ls_svt_noalloc.argtypes = [C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_double,
                                       C.c_int32, C.c_double, C.c_void_p, C.c_void_p,
                                       C.c_void_p, C.c_void_p]
    L.prior_ls_svt_noalloc.restype = C.c_int
    S = C.c_void_p
    L.prior_ls_server_create.argtypes = [C.POINTER(ServerConfig), C.POINTER(S)]
    L.prior_ls_server_create.restype = C.c_int
    L.prior_ls_server_submit.argtypes = [S, C.POINTER(Request), C.POINTER(C.c_int64)]
    L.prior_ls_server_submit.restype = C.c_int
    L.prior_ls_server_wait.argtypes = [S, C.c_int64, C.POINTER(Result)]
    L.prior_ls_server_wait.restype = C.c_int
    L.prior_ls_server_info.argtypes = [S, C.POINTER(ServerStats)]
    L.prior_ls_server_info.restype = C.c_int
    L.prior_ls_server_destroy.argtypes = [S]
    L.prior_ls_server_destroy.restype = None
    _lib = L
    return L


def _sigma_prev_ptr(sigma_prev):
    """(pointer, keep-alive) for sigma_prev: a float64 CUDA tensor is passed as device memory,
    anything else is copied into a host array."""
    if sigma_prev is None:
        return None, None
    if hasattr(sigma_prev, "is_cuda") and sigma_prev.is_cuda:
        import torch
        if sigma_prev.dtype != torch.float64 or not sigma_prev.is_contiguous():
            raise ValueError("a device sigma_prev must be a contiguous float64 tensor")
        return C.cast(C.c_void_p(sigma_prev.data_ptr()), C.POINTER(C.c_double)), sigma_prev
    vals = [float(v) for v in sigma_prev]
    arr = (C.c_double * len(vals))(*vals)
    return C.cast(arr, C.POINTER(C.c_double)), arr


def make_dims(nx, ny, nz, nt, nc, wavelet_levels=2, gram_mode="fp64", hbm_budget=0,
              transform="haar"):
    gm = GRAM_MODES[gram_mode] if isinstance(gram_mode, str) else int(gram_mode)
    tf = TRANSFORMS[transform] if isinstance(transform, str) else int(transform)
    return Dims(C.sizeof(Dims), nx, ny, nz, nt, nc, wavelet_levels, gm, tf, hbm_budget)


def plan_bytes(nx, ny, nz, nt, nc, wavelet_levels=2, gram_mode="fp64", transform="haar"):
    d = make_dims(nx, ny, nz, nt, nc, wavelet_levels, gram_mode, transform=transform)
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
                 hbm_budget=0, stream=None, transform="haar"):
        L = lib()
        self._h = C.c_void_p()
        self.dims = make_dims(nx, ny, nz, nt, nc, wavelet_levels, gram_mode, hbm_budget,
                              transform)
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
        sp = _sigma_prev_ptr(sigma_prev)
        ins = Inputs(_ptr(kspace), _ptr(mask), _ptr(sens), _ptr(prior_w), sp[0],
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

    def tune(self, kspace, mask, sens=None, prior_w=None, sigma_prev=None, lambda_L=0.01,
             lambda_S=0.01, lambda_p=0.0, lambda_L_relative=True, check_every=10, cache=None):
        """prior_ls_tune: time candidate launch shapes on this problem and keep the fastest;
        leaves the problem loaded (as solve with max_iter = 0).  cache: a JSON file (default
        $PRIOR_LS_TUNE_CACHE) of earlier choices keyed by device, geometry and chunk length;
        a hit is applied without measuring (the problem is then loaded by a 0-iteration
        solve).  Returns the choice as a dict."""
        import json
        import torch
        cache = cache or os.environ.get("PRIOR_LS_TUNE_CACHE")
        d = self.dims
        key = (f"{torch.cuda.get_device_name()}|{d.nx}x{d.ny}x{d.nz}x{d.nt}x{d.nc}|J{d.wavelet_levels}"
               f"|T{d.transform}|gram{d.gram_mode}|chunk{check_every}")
        book = {}
        if cache and os.path.exists(cache):
            with open(cache) as fh:
                book = json.load(fh)
        if key in book:
            t = Tuning(C.sizeof(Tuning), int(book[key]["gram_blocks"]), int(book[key]["bp_grid"]),
                       int(book[key]["sparse_fork"]), int(book[key].get("sparse_grid", 0)),
                       float(book[key]["ms_per_iteration"]))
            self._check(lib().prior_ls_set_tuning(self._h, C.byref(t)), "prior_ls_set_tuning")
            self.solve(kspace, mask, sens, prior_w, sigma_prev, lambda_L=lambda_L,
                       lambda_S=lambda_S, lambda_p=lambda_p, lambda_L_relative=lambda_L_relative,
                       max_iter=0, check_every=check_every, outputs=())
            return dict(t.as_dict(), cached=True)
        sp = _sigma_prev_ptr(sigma_prev)
        ins = Inputs(_ptr(kspace), _ptr(mask), _ptr(sens), _ptr(prior_w), sp[0], None, None)
        prm = Params(C.sizeof(Params), float(lambda_L), float(lambda_S), float(lambda_p), 0.0,
                     1 if lambda_L_relative else 0, 0, int(check_every), 1)
        t = Tuning()
        t.struct_size = C.sizeof(Tuning)
        rc = lib().prior_ls_tune(self._h, C.byref(ins), C.byref(prm), C.byref(t))
        torch.cuda.current_stream().synchronize()
        self._check(rc, "prior_ls_tune")
        if cache:
            book[key] = t.as_dict()
            with open(cache, "w") as fh:
                json.dump(book, fh, indent=1)
        return dict(t.as_dict(), cached=False)

    def set_tuning(self, gram_blocks=0, bp_grid=0, sparse_fork=0, sparse_grid=0):
        t = Tuning(C.sizeof(Tuning), int(gram_blocks), int(bp_grid), int(sparse_fork),
                   int(sparse_grid), 0.0)
        self._check(lib().prior_ls_set_tuning(self._h, C.byref(t)), "prior_ls_set_tuning")

    def get_tuning(self):
        t = Tuning()
        t.struct_size = C.sizeof(Tuning)
        self._check(lib().prior_ls_get_tuning(self._h, C.byref(t)), "prior_ls_get_tuning")
        return t.as_dict()

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


class Batch:
    """prior_ls_batch_*: several PriorLS handles advanced together, one launch per kernel
    of an iteration for all of them.  They share the phase-encode plane, transform, Gram
    mode and Gram tile class; nx, nt and nc may differ.  The handles stay owned by the
    caller and must outlive the batch."""

    def __init__(self, solvers: Sequence["PriorLS"]):
        L = lib()
        self.solvers = list(solvers)
        n = len(self.solvers)
        arr = (C.c_void_p * n)(*[s._h.value for s in self.solvers])
        self._b = C.c_void_p()
        rc = L.prior_ls_batch_create(arr, n, C.byref(self._b))
        if rc != OK:
            raise PriorLSError(rc, f"prior_ls_batch_create: {L.prior_ls_last_error(None).decode()}")

    def _check(self, rc, what):
        if rc != OK:
            raise PriorLSError(rc, f"{what}: {lib().prior_ls_batch_last_error(self._b).decode()}")

    def _outputs(self, want):
        outs, os_ = [], []
        for s in self.solvers:
            o, oc = s._outputs(want)
            outs.append(o)
            os_.append(oc)
        return outs, (Outputs * len(os_))(*os_)

    def solve(self, problems, params, outputs=("L", "S", "X", "M")):
        """problems: per problem a dict of device tensors (kspace, mask, sens, prior_w and
        optionally sigma_prev, L0, S0); params: one Params for all or one per problem.
        Returns (outputs, stats) lists."""
        import torch
        n = len(self.solvers)
        if len(problems) != n:
            raise ValueError("one problem per handle")
        prms = list(params) if isinstance(params, (list, tuple)) else [params] * n
        keep, ins = [], []
        for p in problems:
            sp = _sigma_prev_ptr(p.get("sigma_prev"))
            keep.append(sp)
            ins.append(Inputs(_ptr(p["kspace"]), _ptr(p["mask"]), _ptr(p.get("sens")),
                              _ptr(p.get("prior_w")), sp[0],
                              _ptr(p.get("L0")), _ptr(p.get("S0"))))
        in_arr = (Inputs * n)(*ins)
        prm_arr = (Params * n)(*prms)
        outs, o_arr = self._outputs(outputs)
        st = (Stats * n)()
        for k in range(n):
            st[k].struct_size = C.sizeof(Stats)
        rc = lib().prior_ls_batch_solve(self._b, in_arr, prm_arr, o_arr, st)
        torch.cuda.current_stream().synchronize()
        self._check(rc, "prior_ls_batch_solve")
        return outs, [st[k].as_dict() for k in range(n)]

    def step(self, n_iter, outputs=("L", "S", "X", "M")):
        import torch
        n = len(self.solvers)
        outs, o_arr = self._outputs(outputs)
        st = (Stats * n)()
        for k in range(n):
            st[k].struct_size = C.sizeof(Stats)
        rc = lib().prior_ls_batch_step(self._b, int(n_iter), o_arr, st)
        torch.cuda.current_stream().synchronize()
        self._check(rc, "prior_ls_batch_step")
        return outs, [st[k].as_dict() for k in range(n)]

    def close(self):
        if getattr(self, "_b", None) and self._b.value:
            lib().prior_ls_batch_destroy(self._b)
            self._b = C.c_void_p()

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


def svt_noalloc(Cmat, lambda_L=0.01, lambda_L_relative=True, lambda_p=0.0, sigma_prev=None,
                gram_mode="fp64", out=None, sigma=None, stream=None):
    """prior_ls_svt_noalloc: steps (1)-(2) on the Casorati matrix of Cmat (complex64 CUDA
    tensor [nt][...], each frame contiguous) without a handle and without allocating in the
    library; L (out, allocated here by torch when None) and the singular values (sigma, a
    float64 CUDA tensor of nt entries, allocated here when None) are written on `stream`
    (default: torch's current stream).  sigma_prev: float64 CUDA tensor, descending."""
    import torch
    nt = Cmat.shape[0]
    n_vox = Cmat.numel() // nt
    Lout = torch.empty_like(Cmat) if out is None else out
    sig = torch.empty(nt, dtype=torch.float64, device=Cmat.device) if sigma is None else sigma
    gm = GRAM_MODES[gram_mode] if isinstance(gram_mode, str) else int(gram_mode)
    st = _current_stream() if stream is None else C.c_void_p(stream)
    rc = lib().prior_ls_svt_noalloc(_ptr(Cmat), int(n_vox), int(nt), gm, float(lambda_L),
                                    1 if lambda_L_relative else 0, float(lambda_p),
                                    _ptr(sigma_prev), _ptr(Lout), _ptr(sig), st)
    if rc != OK:
        raise PriorLSError(rc, f"prior_ls_svt_noalloc: {lib().prior_ls_last_error(None).decode()}")
    return Lout, sig


def make_params(lambda_L=0.01, lambda_S=0.01, lambda_p=0.0, lambda_L_relative=True, max_iter=20,
                tol=0.0, check_every=10, use_graph=True):
    return Params(C.sizeof(Params), float(lambda_L), float(lambda_S), float(lambda_p),
                  float(tol), 1 if lambda_L_relative else 0, int(max_iter), int(check_every),
                  1 if use_graph else 0)


class Server:
    """prior_ls_server_*: continuous batching of recursive reconstructions.

    submit() queues one sequence (first window + appended frames, CUDA tensors) and returns
    a ticket; the tensors are kept referenced until wait(ticket) returns its result."""

    def __init__(self, hbm_budget=0, max_active=4):
        self._s = C.c_void_p()
        cfg = ServerConfig(C.sizeof(ServerConfig), int(hbm_budget), int(max_active), 0)
        rc = lib().prior_ls_server_create(C.byref(cfg), C.byref(self._s))
        if rc != OK:
            raise PriorLSError(rc, "prior_ls_server_create: " +
                               lib().prior_ls_last_error(None).decode())
        self._live = {}

    def submit(self, dims, kspace0, mask0, kspace_frames=None, mask_frames=None, sens=None,
               first=None, append_params=None, outputs=("L", "S", "X", "M"), out=None,
               sync=True):
        """dims: a Dims (make_dims); kspace0 complex64 [nc][nt][nz][ny][nx], mask0 uint8
        [nt][nz][ny], kspace_frames complex64 [n][nc][nz][ny][nx], mask_frames uint8
        [n][nz][ny]; first / append_params: Params (make_params).  out: preallocated output
        tensors by name (else `outputs` are allocated).  sync: synchronize the current
        stream first (the inputs must be complete before the server reads them); with
        sync=False and `out` given, submit makes no GPU call at all."""
        n = 0 if kspace_frames is None else int(kspace_frames.shape[0])
        if out is None:
            import torch
            shape = (dims.nt, dims.nz, dims.ny, dims.nx)
            outs = {k: torch.empty(shape, dtype=torch.complex64, device="cuda") for k in outputs}
        else:
            outs = dict(out)
        stats = (Stats * (n + 1))()
        for st in stats:
            st.struct_size = C.sizeof(Stats)
        lat = (C.c_double * (n + 1))()
        req = Request(C.sizeof(Request), dims, first or make_params(max_iter=50),
                      append_params or make_params(max_iter=20), n, 0,
                      _ptr(kspace0), _ptr(mask0), _ptr(kspace_frames), _ptr(mask_frames),
                      _ptr(sens), Outputs(*(_ptr(outs.get(k)) for k in ("L", "S", "X", "M"))),
                      C.cast(stats, C.POINTER(Stats)), C.cast(lat, C.POINTER(C.c_double)))
        if sync:
            import torch
            torch.cuda.current_stream().synchronize()  # inputs ready before the server reads
        t = C.c_int64()
        rc = lib().prior_ls_server_submit(self._s, C.byref(req), C.byref(t))
        if rc != OK:
            raise PriorLSError(rc, "prior_ls_server_submit: " +
                               lib().prior_ls_last_error(None).decode())
        self._live[t.value] = (req, outs, stats, lat,
                               (kspace0, mask0, kspace_frames, mask_frames, sens))
        return t.value

    def wait(self, ticket):
        """Blocks until the request is done; returns (outputs, result dict)."""
        r = Result()
        r.struct_size = C.sizeof(Result)
        rc = lib().prior_ls_server_wait(self._s, int(ticket), C.byref(r))
        if rc != OK:
            raise PriorLSError(rc, "prior_ls_server_wait")
        req, outs, stats, lat, _ = self._live.pop(ticket)
        res = {"status": r.status, "reused_plan": bool(r.reused_plan), "queue_ms": r.queue_ms,
               "run_ms": r.run_ms, "total_ms": r.total_ms, "state_bytes": r.state_bytes,
               "message": r.message.decode(), "latency_ms": list(lat),
               "windows": [st.as_dict() for st in stats]}
        return outs, res

    def info(self):
        st = ServerStats()
        st.struct_size = C.sizeof(ServerStats)
        rc = lib().prior_ls_server_info(self._s, C.byref(st))
        if rc != OK:
            raise PriorLSError(rc, "prior_ls_server_info")
        return {k: getattr(st, k) for k, _ in st._fields_ if k != "struct_size"}

    def close(self):
        if getattr(self, "_s", None) and self._s.value:
            lib().prior_ls_server_destroy(self._s)
            self._s = C.c_void_p()
            self._live.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
