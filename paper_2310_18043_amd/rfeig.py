"""Python binding of the rfeig C ABI (``include/rfeig.h``).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides device memory (complex128 CUDA tensors) and the stream.
The library must be built (``python -m paper_2310_18043_amd.build``); if it is
missing or fails to load, importing this module raises.

Blocks of vectors are column-major n x k.  A torch tensor ``X`` of shape
(n, k) is column-major when ``X.T`` is contiguous; ``block(n, k)`` allocates
one and ``as_colmajor`` converts.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# RFEIG_LIBRARY names another build of the library (default: the in-tree one)
LIB_PATH = os.environ.get("RFEIG_LIBRARY") or os.path.join(HERE, "librfeig.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "rfeig.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"rfeig library not built: {LIB_PATH} is missing "
                      "(run python -m paper_2310_18043_amd.build)")
_lib = ctypes.CDLL(LIB_PATH)

RF_OK, RF_ERR_ARG, RF_ERR_NOMEM, RF_ERR_SINGULAR, RF_ERR_NOCONV, RF_ERR_DEVICE, RF_ERR_STATE = range(7)


class RfCsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("colind", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


class RfOpts(ctypes.Structure):
    _fields_ = [("c_re", ctypes.c_double), ("c_im", ctypes.c_double), ("r", ctypes.c_double),
                ("p", ctypes.c_int32), ("q", ctypes.c_int32), ("w", ctypes.c_int32),
                ("sigma_re", ctypes.c_double), ("sigma_im", ctypes.c_double),
                ("tau", ctypes.c_double), ("tau_g", ctypes.c_double),
                ("gmres_tol", ctypes.c_double),
                ("max_subspace_it", ctypes.c_int32), ("max_krylov_blocks", ctypes.c_int32),
                ("subblock", ctypes.c_int32), ("expected_count", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("trsm_cols", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("q_max", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("refine", ctypes.c_int32),
                ("no_graph", ctypes.c_int32), ("solve_form", ctypes.c_int32)]


class RfFilterInfo(ctypes.Structure):
    _fields_ = [("krylov_steps", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("max_residual", ctypes.c_double), ("inner_columns", ctypes.c_int64),
                ("ms_total", ctypes.c_double)]


class RfResult(ctypes.Structure):
    _fields_ = [("lambda_", ctypes.c_void_p), ("X", ctypes.c_void_p), ("ldx", ctypes.c_int64),
                ("err", ctypes.c_void_p), ("flags", ctypes.c_void_p),
                ("count", ctypes.c_int32), ("sweeps", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("krylov_steps", ctypes.c_int32 * 16),
                ("ms_filter", ctypes.c_double), ("ms_hsrr", ctypes.c_double)]


class RfKernelStats(ctypes.Structure):
    _fields_ = [("solve_launches", ctypes.c_int64), ("solve_columns", ctypes.c_int64),
                ("solve_ms", ctypes.c_double), ("factor_launches", ctypes.c_int64),
                ("factor_ms", ctypes.c_double)]


_P = ctypes.c_void_p
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class RfAllocator(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("ctx", ctypes.c_void_p)]


_lib.rf_profile_enable.argtypes = [_P, ctypes.c_int32]
_lib.rf_profile_enable.restype = ctypes.c_int
_lib.rf_profile_read.argtypes = [_P, ctypes.POINTER(RfKernelStats)]
_lib.rf_profile_read.restype = ctypes.c_int
_lib.rf_default_opts.argtypes = [ctypes.POINTER(RfOpts)]
_lib.rf_default_opts.restype = None
_lib.rf_plan_create.argtypes = [ctypes.POINTER(RfCsr), ctypes.POINTER(RfCsr),
                                ctypes.POINTER(RfOpts), ctypes.POINTER(RfAllocator), _P,
                                ctypes.POINTER(_P)]
_lib.rf_plan_create.restype = ctypes.c_int
_lib.rf_factor_shifts.argtypes = [_P]
_lib.rf_factor_shifts.restype = ctypes.c_int
_lib.rf_apply_inner.argtypes = [_P, _P, ctypes.c_int64, ctypes.c_int32, _P, ctypes.c_int64]
_lib.rf_apply_inner.restype = ctypes.c_int
_lib.rf_apply_inner_noalloc.argtypes = [_P, _P, ctypes.c_int64, ctypes.c_int32, _P, ctypes.c_int64]
_lib.rf_apply_inner_noalloc.restype = ctypes.c_int
_lib.rf_filter_apply.argtypes = [_P, _P, ctypes.c_int64, ctypes.c_int32, _P, ctypes.c_int64,
                                 ctypes.POINTER(RfFilterInfo)]
_lib.rf_filter_apply.restype = ctypes.c_int
_lib.rf_solve_region.argtypes = [_P, _P, ctypes.c_int64, ctypes.POINTER(RfResult)]
_lib.rf_solve_region.restype = ctypes.c_int
_lib.rf_solve_region_adaptive.argtypes = [_P, _P, ctypes.c_int64, ctypes.POINTER(RfResult)]
_lib.rf_solve_region_adaptive.restype = ctypes.c_int
_lib.rf_plan_n.argtypes = [_P]
_lib.rf_plan_n.restype = ctypes.c_int64
_lib.rf_plan_device_bytes.argtypes = [_P]
_lib.rf_plan_device_bytes.restype = ctypes.c_int64
_lib.rf_plan_destroy.argtypes = [_P]
_lib.rf_plan_destroy.restype = None
_lib.rf_status_str.argtypes = [ctypes.c_int]
_lib.rf_status_str.restype = ctypes.c_char_p
_lib.rf_last_error.argtypes = [_P]
_lib.rf_last_error.restype = ctypes.c_char_p
_lib.rf_solve_regions.argtypes = [ctypes.c_int32, ctypes.POINTER(_P), ctypes.c_int32,
                                  ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_int64), _P,
                                  ctypes.POINTER(ctypes.c_int)]
_lib.rf_solve_regions.restype = ctypes.c_int
_lib.rf_plan_create_adjoint.argtypes = [_P, _P, ctypes.POINTER(_P)]
_lib.rf_plan_create_adjoint.restype = ctypes.c_int
_lib.rf_eig_vjp.argtypes = [_P, ctypes.c_int32, _P, _P, ctypes.c_int64, ctypes.c_int32, _P, _P,
                            ctypes.c_int64, _P, _P, _P, _P, _P]
_lib.rf_eig_vjp.restype = ctypes.c_int
_lib.rf_batch_create.argtypes = [ctypes.POINTER(RfCsr), ctypes.POINTER(RfCsr),
                                 ctypes.POINTER(RfOpts), ctypes.c_int32,
                                 ctypes.POINTER(RfAllocator), _P, ctypes.POINTER(_P)]
_lib.rf_batch_create.restype = ctypes.c_int
_lib.rf_batch_factor.argtypes = [_P]
_lib.rf_batch_factor.restype = ctypes.c_int
_lib.rf_batch_plan.argtypes = [_P, ctypes.c_int32]
_lib.rf_batch_plan.restype = _P
_lib.rf_batch_size.argtypes = [_P]
_lib.rf_batch_size.restype = ctypes.c_int32
_lib.rf_batch_solve.argtypes = [_P, ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(RfResult), ctypes.POINTER(ctypes.c_int),
                                ctypes.c_int32]
_lib.rf_batch_solve.restype = ctypes.c_int
_lib.rf_batch_device_bytes.argtypes = [_P]
_lib.rf_batch_device_bytes.restype = ctypes.c_int64
_lib.rf_batch_last_error.argtypes = [_P]
_lib.rf_batch_last_error.restype = ctypes.c_char_p
_lib.rf_batch_destroy.argtypes = [_P]
_lib.rf_batch_destroy.restype = None


def library_path() -> str:
    return LIB_PATH


def declared_symbols() -> list[str]:
    """Every function name declared in include/rfeig.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(rf_[a-z_]+)\s*\(", text)))


class RfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_lib.rf_status_str(status).decode()}: {msg}")
        self.status = status


def _torch():
    import torch
    return torch


def block(n: int, k: int, device="cuda"):
    """Uninitialised column-major complex128 n x k block on the device."""
    torch = _torch()
    return torch.empty((k, n), dtype=torch.complex128, device=device).T


def as_colmajor(X):
    """Column-major complex128 device copy of X (n x k) unless it already is one."""
    torch = _torch()
    if X.dim() == 1:
        X = X[:, None]
    if X.dtype != torch.complex128:
        X = X.to(torch.complex128)
    if not X.is_cuda:
        X = X.cuda()
    if X.T.is_contiguous():
        return X
    return X.T.contiguous().T


def _ld(X) -> int:
    # leading dimension of a column-major view: stride of the column index
    return int(X.stride(1)) if X.dim() == 2 and X.shape[1] > 1 else int(X.shape[0])


class TorchAllocator:
    """rf_allocator callbacks backed by PyTorch's caching allocator, so that every
    device buffer of a plan is torch memory (counted by torch.cuda.memory_allocated)
    and is returned to torch's cache when the plan is destroyed.  Blocks are
    allocated on the plan's stream; the library drains its streams before it frees."""

    def __init__(self, stream=None):
        torch = _torch()
        self.device = torch.cuda.current_device()
        self.stream = stream
        self.live = {}

        def _alloc(nbytes, ctx):
            try:
                ptr = torch.cuda.caching_allocator_alloc(int(nbytes), device=self.device,
                                                         stream=self.stream)
            except Exception:             # out of memory: the library reports RF_ERR_NOMEM
                return None
            self.live[int(ptr)] = int(nbytes)
            return int(ptr)

        def _free(ptr, ctx):
            if ptr is None:
                return
            self.live.pop(int(ptr), None)
            torch.cuda.caching_allocator_delete(int(ptr))

        # the ctypes function objects must outlive every plan that holds them
        self._alloc_fn = ALLOC_FN(_alloc)
        self._free_fn = FREE_FN(_free)
        self.struct = RfAllocator(self._alloc_fn, self._free_fn, None)

    @property
    def live_bytes(self) -> int:
        return sum(self.live.values())


def _allocator_arg(allocator, stream):
    """(pointer to pass, object to keep alive): allocator is "torch" (default), None
    (hipMalloc inside the library) or an object with a ``struct`` RfAllocator."""
    if allocator is None:
        return None, None
    if isinstance(allocator, str):
        if allocator != "torch":
            raise ValueError(f"unknown allocator {allocator!r}")
        allocator = TorchAllocator(stream)
    return ctypes.byref(allocator.struct), allocator


class _HostCsr:
    """Keeps host arrays alive for the duration of plan creation."""

    def __init__(self, M):
        import scipy.sparse as sp
        M = sp.csr_matrix(M, dtype=np.complex128)
        M.sort_indices()
        self.rowptr = np.ascontiguousarray(M.indptr, dtype=np.int32)
        self.colind = np.ascontiguousarray(M.indices, dtype=np.int32)
        self.val = np.ascontiguousarray(M.data, dtype=np.complex128)
        self.s = RfCsr(M.shape[0], int(M.nnz), self.rowptr.ctypes.data, self.colind.ctypes.data,
                       self.val.ctypes.data)


def make_opts(c: complex, r: float, p: int = 4, q: int = 8, w: int = 32, **opts) -> RfOpts:
    """rf_opts for disk (c, r): defaults of rf_default_opts, then the given fields."""
    o = RfOpts()
    _lib.rf_default_opts(ctypes.byref(o))
    o.c_re, o.c_im, o.r = float(np.real(c)), float(np.imag(c)), float(r)
    o.p, o.q, o.w = int(p), int(q), int(w)
    for key, val in opts.items():
        if key == "sigma":
            o.sigma_re, o.sigma_im = float(np.real(val)), float(np.imag(val))
        elif hasattr(o, key):
            setattr(o, key, val)
        else:
            raise TypeError(f"unknown option {key}")
    return o


class Plan:
    """rf_plan_create: pencil (A, B) as scipy sparse matrices, disk (c, r), rules p, q, width w."""

    def __init__(self, A, B, c: complex, r: float, p: int = 4, q: int = 8, w: int = 32,
                 stream=None, allocator="torch", tuned=True, **opts):
        torch = _torch()
        if tuned:
            # launch shapes from the autotuner's table (tune.py) where the caller left
            # them automatic
            from . import tune
            entry = tune.lookup(A, B, p, q, w, int(opts.get("precision", 0)))
            if entry:
                for key in ("tile", "trsm_cols", "subblock"):
                    if not opts.get(key):
                        opts[key] = int(entry[key])
        o = make_opts(c, r, p, q, w, **opts)
        self.opts = o
        self._owned = True
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        ha, hb = _HostCsr(A), _HostCsr(B)
        handle = _P()
        aptr, self.allocator = _allocator_arg(allocator, stream)
        st = _lib.rf_plan_create(ctypes.byref(ha.s), ctypes.byref(hb.s), ctypes.byref(o), aptr,
                                 _P(stream.cuda_stream), ctypes.byref(handle))
        if st != RF_OK:
            msg = _lib.rf_last_error(handle).decode() if handle.value else ""
            if handle.value:
                _lib.rf_plan_destroy(handle)
            raise RfError(st, msg or "rf_plan_create failed")
        self._h = handle
        self.n = int(_lib.rf_plan_n(handle))
        self.w = int(w)

    # -- helpers --------------------------------------------------------------
    def _check(self, st, allow=()):
        if st != RF_OK and st not in allow:
            raise RfError(st, _lib.rf_last_error(self._h).decode())
        return st

    @property
    def device_bytes(self) -> int:
        return int(_lib.rf_plan_device_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            if self._owned:
                _lib.rf_plan_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile_enable(self, on: bool = True):
        self._check(_lib.rf_profile_enable(self._h, 1 if on else 0))

    def profile_read(self) -> dict:
        st = RfKernelStats()
        self._check(_lib.rf_profile_read(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in RfKernelStats._fields_}

    # -- the four calls -------------------------------------------------------
    def factor_shifts(self):
        self._check(_lib.rf_factor_shifts(self._h))

    def apply_inner(self, X, out=None):
        X = as_colmajor(X)
        k = X.shape[1]
        Z = block(self.n, k) if out is None else out
        self._check(_lib.rf_apply_inner(self._h, _P(X.data_ptr()), _ld(X), k,
                                        _P(Z.data_ptr()), _ld(Z)))
        return Z

    def apply_inner_noalloc(self, X, out):
        """rf_apply_inner_noalloc: Z = G(X) into the caller's block ``out`` with the
        library's static work array; enqueued on the plan stream, not synchronized."""
        X = as_colmajor(X)
        k = X.shape[1]
        self._check(_lib.rf_apply_inner_noalloc(self._h, _P(X.data_ptr()), _ld(X), k,
                                                _P(out.data_ptr()), _ld(out)))
        return out

    def filter_apply(self, Y, out=None, allow_noconv=False):
        Y = as_colmajor(Y)
        U = block(self.n, Y.shape[1]) if out is None else out
        info = RfFilterInfo()
        st = _lib.rf_filter_apply(self._h, _P(Y.data_ptr()), _ld(Y), Y.shape[1],
                                  _P(U.data_ptr()), _ld(U), ctypes.byref(info))
        self._check(st, allow=(RF_ERR_NOCONV,) if allow_noconv else ())
        return U, {"krylov_steps": info.krylov_steps, "converged": bool(info.converged),
                   "max_residual": info.max_residual, "inner_columns": info.inner_columns,
                   "ms": info.ms_total}

    def adjoint(self, stream=None):
        """rf_plan_create_adjoint: plan of (A^H, B^H) over D(conj c, r) whose solves use
        the conjugate transposes of this plan's factors (factor_shifts on it transposes
        them; this plan must be factorized first)."""
        torch = _torch()
        stream = self.stream if stream is None else stream
        handle = _P()
        st = _lib.rf_plan_create_adjoint(self._h, _P(stream.cuda_stream), ctypes.byref(handle))
        if st != RF_OK:
            msg = _lib.rf_last_error(handle).decode() if handle.value else ""
            if handle.value:
                _lib.rf_plan_destroy(handle)
            raise RfError(st, msg or "rf_plan_create_adjoint failed")
        P = Plan.__new__(Plan)
        P._h = handle
        P._owned = True
        P.allocator = self.allocator          # the adjoint plan uses the same callbacks
        P._parent = self                      # whose factors it transposes: kept alive
        P.opts = self.opts
        P.stream = stream
        P.n = self.n
        P.w = self.w
        return P

    def eig_vjp(self, lam, X, mu, Yl, g, nnz_a, nnz_b=None):
        """rf_eig_vjp: (gA, gB, denom, pair) with gA[e] = sum_i g_i d lambda_i / d A_e
        over the stored entries of A (CSR order), likewise gB (None if nnz_b is None)."""
        torch = _torch()
        lam = np.ascontiguousarray(np.asarray(lam, dtype=np.complex128))
        mu = np.ascontiguousarray(np.asarray(mu, dtype=np.complex128))
        g = np.ascontiguousarray(np.asarray(g, dtype=np.complex128))
        s, sl = len(lam), len(mu)
        if X.dim() == 1:
            X = X[:, None]
        if Yl.dim() == 1:
            Yl = Yl[:, None]
        X = as_colmajor(X)
        Yl = as_colmajor(Yl)
        gA = torch.empty(int(nnz_a), dtype=torch.complex128, device="cuda")
        gB = None if nnz_b is None else torch.empty(int(nnz_b), dtype=torch.complex128,
                                                    device="cuda")
        denom = np.zeros(s, dtype=np.complex128)
        pair = np.zeros(max(s, 1), dtype=np.int32)
        self._check(_lib.rf_eig_vjp(self._h, s, lam.ctypes.data, _P(X.data_ptr()), _ld(X), sl,
                                    mu.ctypes.data, _P(Yl.data_ptr()), _ld(Yl), g.ctypes.data,
                                    _P(gA.data_ptr()), _P(gB.data_ptr() if gB is not None else None),
                                    denom.ctypes.data, pair.ctypes.data))
        return gA, gB, denom, pair[:s]

    def solve_region(self, Y0=None, allow_noconv=False):
        """Alg. composite: subspace iteration with the composite filter."""
        return self._region(_lib.rf_solve_region, Y0, allow_noconv)

    def solve_region_adaptive(self, Y0=None, allow_noconv=False):
        """Alg. composite2: no subspace iteration, the outer node count doubles from q
        to the plan's q_max on one shared Krylov basis."""
        return self._region(_lib.rf_solve_region_adaptive, Y0, allow_noconv)

    def _result(self):
        """An rf_result whose arrays live in the returned holder."""
        w = self.w
        h = {"lam": np.zeros(2 * w), "err": np.zeros(w), "flags": np.zeros(w, dtype=np.int32),
             "X": block(self.n, w)}
        res = RfResult()
        res.lambda_ = h["lam"].ctypes.data
        res.X = h["X"].data_ptr()
        res.ldx = self.n
        res.err = h["err"].ctypes.data
        res.flags = h["flags"].ctypes.data
        return res, h

    @staticmethod
    def _unpack(res, h):
        lam, err, X = h["lam"], h["err"], h["X"]
        lamc = lam[0::2] + 1j * lam[1::2]
        k = res.count
        return {"lam": lamc[:k], "X": X[:, :k], "err": err[:k], "count": k,
                "all_lam": lamc, "all_err": err, "flags": h["flags"], "all_X": X,
                "sweeps": res.sweeps, "converged": bool(res.converged),
                "krylov_steps": list(res.krylov_steps[:min(res.sweeps, 16)]),
                "ms_filter": res.ms_filter, "ms_hsrr": res.ms_hsrr}

    def _region(self, fn, Y0, allow_noconv):
        res, h = self._result()
        if Y0 is not None:
            Y0 = as_colmajor(Y0)
            st = fn(self._h, _P(Y0.data_ptr()), _ld(Y0), ctypes.byref(res))
        else:
            st = fn(self._h, None, 0, ctypes.byref(res))
        self._check(st, allow=(RF_ERR_NOCONV,) if allow_noconv else ())
        return self._unpack(res, h)


class _DiskPlan(Plan):
    """Plan of one disk of a Batch (handle owned by the batch)."""

    def __init__(self, batch, d: int, opts: RfOpts):
        self._batch = batch          # keeps the batch (and the handle) alive
        self._owned = False
        self.opts = opts
        self._h = _P(_lib.rf_batch_plan(batch._h, d))
        if not self._h.value:
            raise RfError(RF_ERR_ARG, f"no disk {d}")
        self.n = int(_lib.rf_plan_n(self._h))
        self.w = int(opts.w)


class Batch:
    """rf_batch_create: one pencil, many disks.  ``disks`` is a list of dicts with the
    keys c, r and optionally p, q, w and any rf_opts field."""

    def __init__(self, A, B, disks, stream=None, allocator="torch", **common):
        torch = _torch()
        n = len(disks)
        arr = (RfOpts * n)()
        for d, spec in enumerate(disks):
            kw = dict(common)
            kw.update(spec)
            arr[d] = make_opts(**kw)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        ha, hb = _HostCsr(A), _HostCsr(B)
        handle = _P()
        aptr, self.allocator = _allocator_arg(allocator, stream)
        st = _lib.rf_batch_create(ctypes.byref(ha.s), ctypes.byref(hb.s), arr, n, aptr,
                                  _P(stream.cuda_stream), ctypes.byref(handle))
        if st != RF_OK:
            msg = _lib.rf_batch_last_error(handle).decode() if handle.value else ""
            if handle.value:
                _lib.rf_batch_destroy(handle)
            raise RfError(st, msg or "rf_batch_create failed")
        self._h = handle
        self.opts = arr
        self.plans = [_DiskPlan(self, d, arr[d]) for d in range(n)]

    def __len__(self):
        return len(self.plans)

    def _check(self, st, allow=()):
        if st != RF_OK and st not in allow:
            raise RfError(st, _lib.rf_batch_last_error(self._h).decode())
        return st

    @property
    def device_bytes(self) -> int:
        return int(_lib.rf_batch_device_bytes(self._h))

    def factor(self):
        self._check(_lib.rf_batch_factor(self._h))

    def solve(self, Y0s=None, threads: int = 0, allow_noconv=False):
        """rf_batch_solve: every disk's Alg. composite; one result dict per disk."""
        torch = _torch()
        n = len(self.plans)
        ys = (_P * n)()
        lds = (ctypes.c_int64 * n)()
        keep = []
        if Y0s is not None:
            for d, Y in enumerate(Y0s):
                if Y is None:
                    continue
                Y = as_colmajor(Y)
                keep.append(Y)
                ys[d] = Y.data_ptr()
                lds[d] = _ld(Y)
        torch.cuda.synchronize()     # start blocks complete before the disk streams read them
        results = (RfResult * n)()
        holders = []
        for d, P in enumerate(self.plans):
            res, h = P._result()
            results[d] = res
            holders.append(h)
        status = (ctypes.c_int * n)()
        st = _lib.rf_batch_solve(self._h, ys, lds, results, status, int(threads))
        allow = (RF_ERR_NOCONV,) if allow_noconv else ()
        for d in range(n):
            if status[d] != RF_OK and status[d] not in allow:
                raise RfError(status[d], _lib.rf_batch_last_error(self._h).decode())
        if st != RF_OK and st not in allow:
            self._check(st)
        out = []
        for d in range(n):
            r = Plan._unpack(results[d], holders[d])
            r["status"] = int(status[d])
            out.append(r)
        return out

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            for P in getattr(self, "plans", []):
                P._h = _P()
            _lib.rf_batch_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_regions(plans, Y0s=None, factor=False, allow_noconv=False):
    """rf_solve_regions: Alg. composite on several independent plans at once (each on
    its own host thread and the plan's stream); factor=True refactorizes first."""
    torch = _torch()
    n = len(plans)
    hs = (_P * n)(*[P._h for P in plans])
    ys = (_P * n)()
    lds = (ctypes.c_int64 * n)()
    keep = []
    if Y0s is not None:
        for d, Y in enumerate(Y0s):
            if Y is None:
                continue
            Y = as_colmajor(Y)
            keep.append(Y)
            ys[d] = Y.data_ptr()
            lds[d] = _ld(Y)
    torch.cuda.synchronize()         # start blocks complete before the plans' streams read them
    results = (RfResult * n)()
    holders = []
    for d, P in enumerate(plans):
        res, h = P._result()
        results[d] = res
        holders.append(h)
    status = (ctypes.c_int * n)()
    st = _lib.rf_solve_regions(n, hs, 1 if factor else 0, ys, lds,
                               ctypes.cast(results, _P), status)
    allow = (RF_ERR_NOCONV,) if allow_noconv else ()
    for d in range(n):
        if status[d] != RF_OK and status[d] not in allow:
            raise RfError(status[d], _lib.rf_last_error(plans[d]._h).decode())
    if st != RF_OK and st not in allow:
        raise RfError(st, "rf_solve_regions failed")
    out = []
    for d in range(n):
        r = Plan._unpack(results[d], holders[d])
        r["status"] = int(status[d])
        out.append(r)
    return out


# ---------------------------------------------------------------------------
# differentiation form: eigenvalues inside a disk as a differentiable function of
# the stored entries of A and B
# ---------------------------------------------------------------------------

def _csr_with_values(pattern, vals):
    import scipy.sparse as sp
    M = sp.csr_matrix((np.asarray(vals, dtype=np.complex128), pattern.indices, pattern.indptr),
                      shape=pattern.shape)
    return M


def disk_eigenvalues(a_vals, b_vals, A_pattern, B_pattern, c, r, Y0=None, Y0_adj=None,
                     **plan_opts):
    """Converged eigenvalues inside D(c, r) of the pencil whose stored entries (CSR
    order of the sorted patterns) are the complex128 tensors a_vals, b_vals, as a
    torch function with a backward pass: the gradient comes from rf_eig_vjp with the
    left vectors of the adjoint pencil, solved by the same filter.

    Returns a complex128 CPU tensor of the converged eigenvalues in the order the
    solver returns them; the gradients come back on the devices of a_vals, b_vals."""
    torch = _torch()
    return _DiskEig.apply(a_vals, b_vals, A_pattern, B_pattern, complex(c), float(r), Y0,
                          Y0_adj, plan_opts)


def _disk_eig_class():
    torch = _torch()

    class DiskEig(torch.autograd.Function):
        @staticmethod
        def forward(ctx, a_vals, b_vals, A_pattern, B_pattern, c, r, Y0, Y0_adj, plan_opts):
            A = _csr_with_values(A_pattern, a_vals.detach().cpu().numpy())
            B = _csr_with_values(B_pattern, b_vals.detach().cpu().numpy())
            opts = dict(plan_opts)
            P = Plan(A, B, c, r, **opts)
            # the adjoint on a stream of its own: both problems are solved concurrently
            Pa = P.adjoint(stream=torch.cuda.Stream())
            res, resa = solve_regions([P, Pa], [Y0, Y0_adj])
            ctx.state = (P, Pa, res, resa, A.nnz, B.nnz, a_vals.device, b_vals.device)
            return torch.from_numpy(np.array(res["lam"], dtype=np.complex128))

        @staticmethod
        def backward(ctx, grad_lam):
            P, Pa, res, resa, nnz_a, nnz_b, dev_a, dev_b = ctx.state
            # torch's convention for complex: grad_in = sum_i grad_i * conj(d lambda_i / d z)
            g = np.conj(grad_lam.detach().cpu().numpy().astype(np.complex128))
            gA, gB, _, _ = P.eig_vjp(res["lam"], res["X"], resa["lam"], resa["X"], g,
                                     nnz_a, nnz_b)
            return (gA.conj().to(dev_a), gB.conj().to(dev_b), None, None, None, None, None, None,
                    None)

    return DiskEig


class _LazyFn:
    _cls = None

    def apply(self, *args):
        if _LazyFn._cls is None:
            _LazyFn._cls = _disk_eig_class()
        return _LazyFn._cls.apply(*args)


_DiskEig = _LazyFn()
