"""Thin Python binding of the h2ulv C-ABI (include/h2ulv.h).

Argument marshalling only: every step of the factorization and solve runs in
the HIP library.  torch supplies device memory and the current stream.  The
library must be built (``python -m paper_2208_10907_amd.build``); loading fails
loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os
from pathlib import Path

import numpy as np

LIB_PATH = Path(__file__).resolve().parent / "_lib" / "libh2ulv.so"

OK = 0
ERR_INVALID_ARG = -1
ERR_OOM = -2
ERR_HIP = -3
ERR_SINGULAR = -4
ERR_DUPLICATE_POINTS = -5
ERR_NOT_CONVERGED = -6
ERR_RANK_CHECK = -7

LAPLACE = 0
YUKAWA = 1
ADVECTION = 2
FP64 = 0
MIXED = 1

# every symbol include/h2ulv.h declares
EXPORTS = [
    "h2ulv_params_default", "h2ulv_factorize", "h2ulv_factorize_batch", "h2ulv_solve",
    "h2ulv_matvec_exact", "h2ulv_refine", "h2ulv_get_stats", "h2ulv_get_levels",
    "h2ulv_get_perm", "h2ulv_get_ranks", "h2ulv_get_skeleton", "h2ulv_get_basis",
    "h2ulv_get_column_skeleton", "h2ulv_get_column_basis", "h2ulv_solve_repeated",
    "h2ulv_destroy", "h2ulv_structure_create", "h2ulv_structure_levels",
    "h2ulv_structure_perm", "h2ulv_structure_lists", "h2ulv_structure_geometry",
    "h2ulv_structure_destroy", "h2ulv_status_string", "h2ulv_last_error",
    "h2ulv_profile_enable", "h2ulv_profile_read", "h2ulv_rankmodel_create",
    "h2ulv_rankmodel_destroy", "h2ulv_rankmodel_set_params", "h2ulv_rankmodel_get_params",
    "h2ulv_rankmodel_forward", "h2ulv_rankmodel_gradient", "h2ulv_rankmodel_adam_step",
    "h2ulv_rankmodel_train", "h2ulv_rankmodel_save", "h2ulv_rankmodel_load",
    "h2ulv_get_features", "h2ulv_get_sketch_info",
    "h2ulv_release_cache", "h2ulv_refine_gmres", "h2ulv_refine_block_gmres",
    "h2ulv_gemm_tile_rates",
    "h2ulv_matvec_exact_noalloc",
]

NFEAT = 16
MLP_NPARAM = 9473


class Params(C.Structure):
    _fields_ = [
        ("struct_size", C.c_int32), ("kernel", C.c_int32), ("alpha", C.c_double),
        ("diag", C.c_double), ("eta", C.c_double), ("leaf_size", C.c_int32),
        ("rank_cap", C.c_int32), ("tol", C.c_double), ("far_sample", C.c_int32),
        ("precision", C.c_int32), ("verbose", C.c_int32), ("oversample", C.c_int32),
        ("rank_model", C.c_void_p), ("sketch_seed", C.c_uint64), ("fill_in", C.c_int32),
        ("partition", C.c_int32), ("structure", C.c_int32), ("bases", C.c_int32),
        ("sketch_fallback", C.c_int32), ("sketch_min_level", C.c_int32),
        ("drift", C.c_double * 3),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("levels", C.c_int32), ("max_rank", C.c_int32), ("root_size", C.c_int32),
        ("reserved", C.c_int32), ("n", C.c_int64), ("flops_fill", C.c_double),
        ("flops_basis", C.c_double), ("flops_couple", C.c_double),
        ("flops_rotate", C.c_double), ("flops_elim", C.c_double), ("flops_root", C.c_double),
        ("kernel_evals", C.c_double), ("time_setup_s", C.c_double),
        ("time_factor_s", C.c_double), ("device_bytes", C.c_double), ("logabsdet", C.c_double),
    ]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}
        d["flops"] = (self.flops_fill + self.flops_basis + self.flops_couple + self.flops_rotate
                      + self.flops_elim + self.flops_root)
        return d


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    """h2ulv_allocator: device memory from the caller."""
    _fields_ = [("ctx", C.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN)]


def make_allocator(alloc, free) -> Allocator:
    """An h2ulv_allocator from two Python functions: alloc(nbytes, stream) ->
    device address (0 on failure), free(ptr, stream).  An exception in alloc
    counts as a failed allocation.  The returned object keeps the callbacks
    alive; keep it as long as any factor made with it."""
    def _a(ctx, nbytes, stream):
        try:
            return int(alloc(int(nbytes), stream or 0)) or None
        except Exception:  # noqa: BLE001 - no exception may cross the C boundary
            return None

    def _f(ctx, ptr, stream):
        try:
            free(int(ptr), stream or 0)
        except Exception:  # noqa: BLE001
            pass

    a = Allocator(None, ALLOC_FN(_a), FREE_FN(_f))
    a._refs = (_a, _f, alloc, free)
    return a


_TORCH_ALLOCATOR = None


def torch_allocator() -> Allocator:
    """The torch caching allocator behind the library's device memory:
    blocks are drawn on (and stream-ordered by) the stream of each call."""
    global _TORCH_ALLOCATOR
    if _TORCH_ALLOCATOR is None:
        import torch

        def alloc(nbytes, stream):
            return torch.cuda.caching_allocator_alloc(nbytes, stream=stream or None)

        def free(ptr, stream):
            torch.cuda.caching_allocator_delete(ptr)

        _TORCH_ALLOCATOR = make_allocator(alloc, free)
    return _TORCH_ALLOCATOR


def _allocator(allocator):
    """'torch' -> the torch caching allocator, None -> the library's own cache,
    or an Allocator."""
    if allocator is None:
        return None
    if isinstance(allocator, str):
        if allocator != "torch":
            raise ValueError(f"unknown allocator {allocator!r}")
        return torch_allocator()
    return allocator


class KernelProfile(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("time_ms", C.c_double),
                ("flops", C.c_double), ("bytes", C.c_double)]


class H2ULVError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"h2ulv status {status}: {msg}")
        self.status = status


_lib = None


def lib() -> C.CDLL:
    """Load libh2ulv.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not LIB_PATH.exists():
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2208_10907_amd.build`")
    L = C.CDLL(str(LIB_PATH))
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    sig = {
        "h2ulv_params_default": (i32, [P(Params)]),
        "h2ulv_factorize": (i32, [vp, i64, P(Params), P(Allocator), vp, P(vp)]),
        "h2ulv_factorize_batch": (i32, [i32, P(vp), P(i64), P(Params), P(Allocator), vp,
                                        P(vp)]),
        "h2ulv_solve": (i32, [vp, vp, i32, i64, vp]),
        "h2ulv_matvec_exact": (i32, [vp, vp, i64, vp, i64, i32, vp]),
        "h2ulv_matvec_exact_noalloc": (i32, [vp, vp, i64, vp, i64, i32, vp]),
        "h2ulv_refine": (i32, [vp, vp, i64, vp, i64, i32, dbl, i32, P(i32), P(dbl), vp]),
        "h2ulv_get_stats": (i32, [vp, P(Stats)]),
        "h2ulv_get_levels": (i32, [vp, P(i32)]),
        "h2ulv_get_perm": (i32, [vp, vp]),
        "h2ulv_get_ranks": (i32, [vp, i32, vp, vp]),
        "h2ulv_get_skeleton": (i32, [vp, i32, i32, vp]),
        "h2ulv_get_basis": (i32, [vp, i32, i32, vp]),
        "h2ulv_get_column_skeleton": (i32, [vp, i32, i32, vp]),
        "h2ulv_get_column_basis": (i32, [vp, i32, i32, vp]),
        "h2ulv_solve_repeated": (i32, [vp, vp, i32, i64, vp]),
        "h2ulv_destroy": (None, [vp]),
        "h2ulv_structure_create": (i32, [vp, i64, P(Params), P(vp)]),
        "h2ulv_structure_levels": (i32, [vp, P(i32)]),
        "h2ulv_structure_perm": (i32, [vp, vp]),
        "h2ulv_structure_lists": (i32, [vp, i32, vp, vp, vp, vp]),
        "h2ulv_structure_geometry": (i32, [vp, i32, vp, vp]),
        "h2ulv_structure_destroy": (None, [vp]),
        "h2ulv_status_string": (C.c_char_p, [i32]),
        "h2ulv_last_error": (C.c_char_p, []),
        "h2ulv_profile_enable": (i32, [i32]),
        "h2ulv_profile_read": (i32, [P(KernelProfile), i32, P(i32)]),
        "h2ulv_rankmodel_create": (i32, [C.c_uint64, P(vp)]),
        "h2ulv_rankmodel_destroy": (None, [vp]),
        "h2ulv_rankmodel_set_params": (i32, [vp, vp]),
        "h2ulv_rankmodel_get_params": (i32, [vp, vp]),
        "h2ulv_rankmodel_forward": (i32, [vp, vp, i64, vp, vp]),
        "h2ulv_rankmodel_gradient": (i32, [vp, vp, vp, i64, vp, P(C.c_float), vp]),
        "h2ulv_rankmodel_adam_step": (i32, [vp, vp, C.c_float, vp]),
        "h2ulv_rankmodel_train": (i32, [vp, vp, vp, i64, i32, C.c_float, P(C.c_float), vp]),
        "h2ulv_rankmodel_save": (i32, [vp, C.c_char_p]),
        "h2ulv_rankmodel_load": (i32, [C.c_char_p, P(vp)]),
        "h2ulv_get_features": (i32, [vp, i32, vp, vp]),
        "h2ulv_get_sketch_info": (i32, [vp, i32, vp, vp, vp]),
        "h2ulv_release_cache": (i32, []),
        "h2ulv_gemm_tile_rates": (i32, [P(dbl)]),
        "h2ulv_refine_gmres": (i32, [vp, vp, i64, vp, i64, i32, dbl, i32, i32, P(i32), P(dbl),
                                     vp]),
        "h2ulv_refine_block_gmres": (i32, [vp, vp, i64, vp, i64, i32, dbl, i32, i32, P(i32),
                                           P(dbl), vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status: int) -> None:
    if status != OK:
        msg = lib().h2ulv_last_error().decode(errors="replace")
        raise H2ULVError(status, msg)


def make_params(kernel=LAPLACE, alpha=0.0, diag=1e3, eta=1.0, leaf=256, tol=1e-8,
                rank_cap=0, far_sample=32, precision=FP64, verbose=0, rank_model=None,
                sketch_seed=0, oversample=8, fill_in=True, partition="kd",
                structure="h2", drift=(0.0, 0.0, 0.0), bases="auto",
                sketch_fallback=True, sketch_min_level=0) -> Params:
    p = Params()
    _check(lib().h2ulv_params_default(C.byref(p)))
    p.kernel, p.alpha, p.diag, p.eta = int(kernel), float(alpha), float(diag), float(eta)
    p.leaf_size, p.rank_cap, p.tol = int(leaf), int(rank_cap), float(tol)
    p.far_sample, p.precision, p.verbose = int(far_sample), int(precision), int(verbose)
    p.oversample, p.sketch_seed = int(oversample), int(sketch_seed)
    p.fill_in = 1 if fill_in else 0
    p.partition = {"kd": 0, "kmeans": 1}[partition]
    p.structure = {"h2": 0, "blr2": 1}[structure]
    p.bases = {"auto": 0, "separate": 1}[bases]
    p.sketch_fallback = 1 if sketch_fallback else 0
    p.sketch_min_level = int(sketch_min_level)
    for c in range(3):
        p.drift[c] = float(drift[c])
    p.rank_model = rank_model._h.value if rank_model is not None else None
    p._model_ref = rank_model  # keeps the model alive as long as the parameters
    return p


def params_from_problem(prob, precision=FP64, verbose=0, **kw) -> Params:
    return make_params(prob.kernel, prob.alpha, prob.diag, prob.eta, prob.leaf, prob.tol,
                       prob.rank_cap, prob.far_sample, precision, verbose, **kw)


def _f32(x):
    import torch
    x = torch.as_tensor(x)
    return x.to(device="cuda", dtype=torch.float32).contiguous()


class RankModel:
    """The rank MLP (16 features -> 3 x 64 ReLU -> 1) with its parameters on
    the GPU; forward, gradient, Adam and the training loop run in the library."""

    def __init__(self, seed: int = 0):
        h = C.c_void_p()
        _check(lib().h2ulv_rankmodel_create(int(seed), C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.h2ulv_rankmodel_destroy(h)
            self._h = None

    def save(self, path) -> None:
        """Write the model and its Adam state to a file (h2ulv_rankmodel_save)."""
        _check(lib().h2ulv_rankmodel_save(self._h, os.fsencode(path)))

    @classmethod
    def load(cls, path) -> "RankModel":
        """A model read from a file that save() wrote (h2ulv_rankmodel_load)."""
        h = C.c_void_p()
        _check(lib().h2ulv_rankmodel_load(os.fsencode(path), C.byref(h)))
        obj = cls.__new__(cls)
        obj._h = h
        return obj

    def get_params(self) -> np.ndarray:
        out = np.empty(MLP_NPARAM, dtype=np.float32)
        _check(lib().h2ulv_rankmodel_get_params(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_params(self, theta) -> None:
        th = np.ascontiguousarray(theta, dtype=np.float32)
        if th.size != MLP_NPARAM:
            raise ValueError(f"expected {MLP_NPARAM} parameters")
        _check(lib().h2ulv_rankmodel_set_params(self._h, th.ctypes.data_as(C.c_void_p)))

    def forward(self, feat, stream=None):
        import torch
        f = _f32(feat).reshape(-1, NFEAT)
        y = torch.empty(f.shape[0], dtype=torch.float32, device="cuda")
        _check(lib().h2ulv_rankmodel_forward(self._h, C.c_void_p(f.data_ptr()), f.shape[0],
                                             C.c_void_p(y.data_ptr()), _stream(stream)))
        return y

    def gradient(self, feat, target, stream=None):
        import torch
        f = _f32(feat).reshape(-1, NFEAT)
        t = _f32(target).reshape(-1)
        g = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
        loss = C.c_float(0.0)
        _check(lib().h2ulv_rankmodel_gradient(self._h, C.c_void_p(f.data_ptr()),
                                              C.c_void_p(t.data_ptr()), f.shape[0],
                                              C.c_void_p(g.data_ptr()), C.byref(loss),
                                              _stream(stream)))
        return g, float(loss.value)

    def adam_step(self, grad, lr: float, stream=None) -> None:
        g = _f32(grad)
        _check(lib().h2ulv_rankmodel_adam_step(self._h, C.c_void_p(g.data_ptr()), float(lr),
                                               _stream(stream)))

    def train(self, feat, target, steps: int, lr: float = 3e-3, stream=None) -> float:
        f = _f32(feat).reshape(-1, NFEAT)
        t = _f32(target).reshape(-1)
        loss = C.c_float(0.0)
        _check(lib().h2ulv_rankmodel_train(self._h, C.c_void_p(f.data_ptr()),
                                           C.c_void_p(t.data_ptr()), f.shape[0], int(steps),
                                           float(lr), C.byref(loss), _stream(stream)))
        return float(loss.value)


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _dev_points(points):
    import torch
    if not isinstance(points, torch.Tensor):
        points = torch.as_tensor(np.ascontiguousarray(points, dtype=np.float64))
    pts = points.to(device="cuda", dtype=torch.float64).contiguous()
    if pts.ndim != 2 or pts.shape[1] != 3:
        raise ValueError("points must be N x 3")
    return pts


class Factor:
    """Owns one h2ulv_factor handle."""

    def __init__(self, handle: int, pts, allocator=None):
        self._h = C.c_void_p(handle)
        self._pts = pts
        self._alloc = allocator  # must outlive the handle
        self.n = int(pts.shape[0])

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.h2ulv_destroy(h)
            self._h = None

    # -- vectors: torch (n,) or (n, nrhs) tensors on the GPU -----------------
    @staticmethod
    def _colmajor(b):
        """A fresh (nrhs, n) buffer (== n x nrhs column-major); never a view of b,
        since the library writes into it."""
        import torch
        b = b.to(device="cuda", dtype=torch.float64)
        vec = b.ndim == 1
        bm = b.reshape(b.shape[0], -1)
        out = torch.empty((bm.shape[1], bm.shape[0]), dtype=torch.float64, device=b.device)
        out.copy_(bm.t())
        return vec, out

    @staticmethod
    def _back(vec, bt):
        out = bt.t()
        return out[:, 0].contiguous() if vec else out.contiguous()

    def solve(self, b, stream=None):
        vec, bt = self._colmajor(b)
        _check(lib().h2ulv_solve(self._h, C.c_void_p(bt.data_ptr()), bt.shape[0], self.n,
                                 _stream(stream)))
        return self._back(vec, bt)

    def solve_repeated(self, b, stream=None):
        """solve() through the factor's recorded HIP graph for this number of
        right-hand sides (recorded on the first call); identical results."""
        vec, bt = self._colmajor(b)
        _check(lib().h2ulv_solve_repeated(self._h, C.c_void_p(bt.data_ptr()), bt.shape[0],
                                          self.n, _stream(stream)))
        return self._back(vec, bt)

    def matvec(self, x, stream=None):
        import torch
        vec, xt = self._colmajor(x)
        yt = torch.empty_like(xt)
        _check(lib().h2ulv_matvec_exact(self._h, C.c_void_p(xt.data_ptr()), self.n,
                                        C.c_void_p(yt.data_ptr()), self.n, xt.shape[0],
                                        _stream(stream)))
        return self._back(vec, yt)

    def matvec_noalloc(self, x, y, stream=None):
        """y = A x through the allocation-free entry point; x and y are caller-owned
        column-major device arrays (n x nrhs, Fortran order) and nothing is
        allocated or synchronised."""
        _check(lib().h2ulv_matvec_exact_noalloc(self._h, C.c_void_p(x.data_ptr()), x.stride(1),
                                                C.c_void_p(y.data_ptr()), y.stride(1),
                                                x.shape[1], _stream(stream)))
        return y

    def refine(self, b, rtol=1e-10, max_iter=20, stream=None, raise_on_fail=True):
        import torch
        vec, bt = self._colmajor(b)
        xt = torch.empty_like(bt)
        it = C.c_int32(0)
        rr = C.c_double(0.0)
        st = lib().h2ulv_refine(self._h, C.c_void_p(bt.data_ptr()), self.n,
                                C.c_void_p(xt.data_ptr()), self.n, bt.shape[0], float(rtol),
                                int(max_iter), C.byref(it), C.byref(rr), _stream(stream))
        if st != OK and (raise_on_fail or st != ERR_NOT_CONVERGED):
            _check(st)
        return self._back(vec, xt), int(it.value), float(rr.value)

    def refine_gmres(self, b, rtol=1e-10, max_iter=60, restart=30, stream=None,
                     raise_on_fail=True):
        """Refinement whose correction equation is solved by GMRES preconditioned
        with the ULV solve.  Returns (x, steps, relres)."""
        import torch
        vec, bt = self._colmajor(b)
        xt = torch.empty_like(bt)
        it = C.c_int32(0)
        rr = C.c_double(0.0)
        st = lib().h2ulv_refine_gmres(self._h, C.c_void_p(bt.data_ptr()), self.n,
                                      C.c_void_p(xt.data_ptr()), self.n, bt.shape[0],
                                      float(rtol), int(max_iter), int(restart), C.byref(it),
                                      C.byref(rr), _stream(stream))
        if st != OK and (raise_on_fail or st != ERR_NOT_CONVERGED):
            _check(st)
        return self._back(vec, xt), int(it.value), float(rr.value)

    def refine_block_gmres(self, b, rtol=1e-10, max_iter=200, restart=128, stream=None,
                           raise_on_fail=True):
        """Refinement whose correction equations (all columns together) are solved
        by block GMRES preconditioned with the ULV solve.  Returns (x, block
        steps, relres)."""
        import torch
        vec, bt = self._colmajor(b)
        xt = torch.empty_like(bt)
        it = C.c_int32(0)
        rr = C.c_double(0.0)
        st = lib().h2ulv_refine_block_gmres(self._h, C.c_void_p(bt.data_ptr()), self.n,
                                            C.c_void_p(xt.data_ptr()), self.n, bt.shape[0],
                                            float(rtol), int(max_iter), int(restart),
                                            C.byref(it), C.byref(rr), _stream(stream))
        if st != OK and (raise_on_fail or st != ERR_NOT_CONVERGED):
            _check(st)
        return self._back(vec, xt), int(it.value), float(rr.value)

    # -- inspection ---------------------------------------------------------
    def stats(self) -> dict:
        s = Stats()
        _check(lib().h2ulv_get_stats(self._h, C.byref(s)))
        return s.as_dict()

    def levels(self) -> int:
        L = C.c_int32()
        _check(lib().h2ulv_get_levels(self._h, C.byref(L)))
        return int(L.value)

    def perm(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int64)
        _check(lib().h2ulv_get_perm(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def ranks(self, lev: int):
        m = np.empty(1 << lev, dtype=np.int32)
        k = np.empty(1 << lev, dtype=np.int32)
        _check(lib().h2ulv_get_ranks(self._h, lev, m.ctypes.data_as(C.c_void_p),
                                     k.ctypes.data_as(C.c_void_p)))
        return m, k

    def skeleton(self, lev: int, box: int) -> np.ndarray:
        _, k = self.ranks(lev)
        out = np.empty(max(int(k[box]), 1), dtype=np.int64)
        _check(lib().h2ulv_get_skeleton(self._h, lev, box, out.ctypes.data_as(C.c_void_p)))
        return out[: int(k[box])]

    def column_skeleton(self, lev: int, box: int) -> np.ndarray:
        """Column skeleton of a box (separate bases; the row skeleton otherwise)."""
        _, k = self.ranks(lev)
        out = np.empty(max(int(k[box]), 1), dtype=np.int64)
        _check(lib().h2ulv_get_column_skeleton(self._h, lev, box,
                                               out.ctypes.data_as(C.c_void_p)))
        return out[: int(k[box])]

    def column_basis(self, lev: int, box: int) -> np.ndarray:
        """V = [V^S V^R] of a box (separate bases; U otherwise)."""
        m, _ = self.ranks(lev)
        mm = int(m[box])
        out = np.empty((mm, mm), dtype=np.float64, order="F")
        if mm:
            _check(lib().h2ulv_get_column_basis(self._h, lev, box,
                                                out.ctypes.data_as(C.c_void_p)))
        return out

    def features(self, lev: int):
        """(features (2^lev x 16, float32), targets log2(1 + k)) of a level."""
        nb = 1 << lev
        F = np.empty((nb, NFEAT), dtype=np.float32)
        T = np.empty(nb, dtype=np.float32)
        _check(lib().h2ulv_get_features(self._h, lev, F.ctypes.data_as(C.c_void_p),
                                        T.ctypes.data_as(C.c_void_p)))
        return F, T

    def sketch_info(self, lev: int):
        """(predicted rank, sketch columns, outcome) per box of a level."""
        nb = 1 << lev
        a, b, c = (np.empty(nb, dtype=np.int32) for _ in range(3))
        _check(lib().h2ulv_get_sketch_info(self._h, lev, a.ctypes.data_as(C.c_void_p),
                                           b.ctypes.data_as(C.c_void_p),
                                           c.ctypes.data_as(C.c_void_p)))
        return a, b, c

    def basis(self, lev: int, box: int) -> np.ndarray:
        m, _ = self.ranks(lev)
        mm = int(m[box])
        out = np.empty((mm, mm), dtype=np.float64, order="F")
        if mm:
            _check(lib().h2ulv_get_basis(self._h, lev, box, out.ctypes.data_as(C.c_void_p)))
        return out


def release_cache() -> None:
    """Hand the library's cached device memory back to the runtime."""
    _check(lib().h2ulv_release_cache())


def factorize(points, params: Params | None = None, stream=None, allocator="torch",
              **kw) -> Factor:
    """Factorize the kernel matrix of `points` (N x 3) on the current GPU.
    allocator: 'torch' (the torch caching allocator supplies the device memory),
    None (the library's own caching allocator) or an Allocator."""
    if params is None:
        params = make_params(**kw)
    pts = _dev_points(points)
    al = _allocator(allocator)
    h = C.c_void_p()
    _check(lib().h2ulv_factorize(C.c_void_p(pts.data_ptr()), pts.shape[0], C.byref(params),
                                 C.byref(al) if al is not None else None, _stream(stream),
                                 C.byref(h)))
    return Factor(h.value, pts, al)


def factorize_batch(points_list, params: Params, stream=None, allocator="torch") -> list:
    """Factorize several independent problems with shared batched launches."""
    pts = [_dev_points(p) for p in points_list]
    n = len(pts)
    al = _allocator(allocator)
    ptrs = (C.c_void_p * n)(*[p.data_ptr() for p in pts])
    ns = (C.c_int64 * n)(*[p.shape[0] for p in pts])
    hs = (C.c_void_p * n)()
    _check(lib().h2ulv_factorize_batch(n, ptrs, ns, C.byref(params),
                                       C.byref(al) if al is not None else None,
                                       _stream(stream), hs))
    return [Factor(hs[i], pts[i], al) for i in range(n)]


class Structure:
    """Host-only cluster tree and near/far lists (no GPU needed)."""

    def __init__(self, points, params: Params):
        X = np.ascontiguousarray(points, dtype=np.float64)
        h = C.c_void_p()
        _check(lib().h2ulv_structure_create(X.ctypes.data_as(C.c_void_p), X.shape[0],
                                            C.byref(params), C.byref(h)))
        self._h = h
        self.n = X.shape[0]
        L = C.c_int32()
        _check(lib().h2ulv_structure_levels(h, C.byref(L)))
        self.L = int(L.value)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.h2ulv_structure_destroy(h)
            self._h = None

    def perm(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int64)
        _check(lib().h2ulv_structure_perm(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def lists(self, lev: int):
        nb = 1 << lev
        npt = np.empty(nb + 1, dtype=np.int64)
        fpt = np.empty(nb + 1, dtype=np.int64)
        _check(lib().h2ulv_structure_lists(self._h, lev, npt.ctypes.data_as(C.c_void_p), None,
                                           fpt.ctypes.data_as(C.c_void_p), None))
        nix = np.empty(max(int(npt[-1]), 1), dtype=np.int32)
        fix = np.empty(max(int(fpt[-1]), 1), dtype=np.int32)
        _check(lib().h2ulv_structure_lists(self._h, lev, npt.ctypes.data_as(C.c_void_p),
                                           nix.ctypes.data_as(C.c_void_p),
                                           fpt.ctypes.data_as(C.c_void_p),
                                           fix.ctypes.data_as(C.c_void_p)))
        near = [nix[npt[i]:npt[i + 1]].tolist() for i in range(nb)]
        far = [fix[fpt[i]:fpt[i + 1]].tolist() for i in range(nb)]
        return near, far

    def geometry(self, lev: int):
        nb = 1 << lev
        c = np.empty(nb * 3, dtype=np.float64)
        r = np.empty(nb, dtype=np.float64)
        _check(lib().h2ulv_structure_geometry(self._h, lev, c.ctypes.data_as(C.c_void_p),
                                              r.ctypes.data_as(C.c_void_p)))
        return c.reshape(nb, 3), r


def profile_enable(on: bool = True) -> None:
    """Start (or stop) recording per-kernel launch times with HIP events."""
    _check(lib().h2ulv_profile_enable(1 if on else 0))


def gemm_tile_rates() -> dict:
    """Autotuned full-tile rates (TFLOP/s) of the GEMM tile shapes on the current
    device (0 where not measured yet)."""
    out = (C.c_double * 6)()
    _check(lib().h2ulv_gemm_tile_rates(out))
    names = ["f64_64x64", "f64_64x128", "f64_128x64", "f64_128x128", "f32_64x64", "f32_128x128"]
    return {n: round(float(v), 2) for n, v in zip(names, out)}


def profile_read() -> dict:
    """Per-kernel launches, summed time (ms), algorithmic flops and bytes."""
    arr = (KernelProfile * 64)()
    cnt = C.c_int32(0)
    _check(lib().h2ulv_profile_read(arr, 64, C.byref(cnt)))
    out = {}
    for i in range(min(cnt.value, 64)):
        r = arr[i]
        out[r.name.decode()] = {"launches": int(r.launches), "time_ms": float(r.time_ms),
                                "flops": float(r.flops), "bytes": float(r.bytes)}
    return out
