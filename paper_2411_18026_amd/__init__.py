"""MI355X proxy-surface fast direct solver for 2D elastic scattering by
traction-free cavities (Galerkin P1, Burton-Miller BIE).

Thin Python binding over the C ABI declared in ``include/fds.h``: argument
marshalling only.  Every arithmetic step runs in the HIP kernels of
``libfds.so``; there is no fallback.  PyTorch provides device memory and the
stream.

Conventions: a geometry is a list of ``(n_i, 2)`` vertex arrays (closed,
counter-clockwise); unknown ``2 t + i`` is component ``i`` at global node
``t``; right-hand sides and solutions are complex128 tensors of shape
``(nrhs, N_unk)`` on the GPU (row k = column k of the column-major C view).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfds.so")
_lib = None


class FdsError(RuntimeError):
    """A library call returned a non-zero fds_status (``code``)."""

    def __init__(self, msg, code=None):
        super().__init__(msg)
        self.code = code


class _C64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class _Geometry(ctypes.Structure):
    _fields_ = [("n_curves", ctypes.c_int32), ("n_nodes", ctypes.POINTER(ctypes.c_int32)),
                ("xy", ctypes.POINTER(ctypes.c_double))]


class _Options(ctypes.Structure):
    _fields_ = [("leaf_nodes", ctypes.c_int32), ("n_proxy", ctypes.c_int32), ("root_level", ctypes.c_int32),
                ("solve_graph", ctypes.c_int32), ("proxy_ratio", ctypes.c_double), ("alpha", _C64),
                ("use_alpha", ctypes.c_int32), ("precision", ctypes.c_int32), ("ir_max_iter", ctypes.c_int32),
                ("proxy_fixed", ctypes.c_int32), ("ir_rtol", ctypes.c_double), ("ir_dtol", ctypes.c_double),
                ("rank_mode", ctypes.c_int32), ("oversample", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("predictor", ctypes.POINTER(ctypes.c_float)), ("autotune", ctypes.c_int32),
                ("mfma_sweeps", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("root_level", ctypes.c_int32), ("n_unknowns", ctypes.c_int64),
                ("root_size", ctypes.c_int64), ("max_rank", ctypes.c_int32), ("max_proxy", ctypes.c_int32),
                ("factor_seconds", ctypes.c_double), ("assembly_seconds", ctypes.c_double),
                ("id_seconds", ctypes.c_double), ("merge_seconds", ctypes.c_double),
                ("root_seconds", ctypes.c_double), ("factor_bytes", ctypes.c_int64),
                ("kernel_evals", ctypes.c_int64), ("class_seconds", ctypes.c_double * 6),
                ("class_evals", ctypes.c_int64 * 6), ("class_launches", ctypes.c_int64 * 6),
                ("precision", ctypes.c_int32), ("ir_iterations", ctypes.c_int32), ("ir_residual", ctypes.c_double),
                ("ir_correction", ctypes.c_double), ("rank_mode", ctypes.c_int32), ("reserved2", ctypes.c_int32),
                ("cells_compressed", ctypes.c_int64), ("cells_sketched", ctypes.c_int64),
                ("cells_fallback_rank", ctypes.c_int64), ("cells_fallback_judge", ctypes.c_int64),
                ("predict_seconds", ctypes.c_double), ("tune_chunk", ctypes.c_int32 * 4),
                ("tune_gemm_cols", ctypes.c_int32 * 4), ("tune_seconds", ctypes.c_double),
                ("pair_kernel_seconds", ctypes.c_double * 12), ("pair_kernel_evals", ctypes.c_int64 * 12),
                ("pair_kernel_launches", ctypes.c_int64 * 12)]

# the pair-integration kernels in the order of fds_stats.pair_kernel_*
PAIR_KERNELS = ["k_regular<0, false>", "k_regular<0, true>", "k_regular<1, false>", "k_regular<1, true>",
                "k_regular<2, false>", "k_regular<2, true>", "k_regular<3, false>", "k_regular<3, true>",
                "k_regular_wave10", "k_special<1>", "k_special2<2>", "k_special2<3>"]


class _RankRecord(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_int32), ("level", ctypes.c_int32), ("rank", ctypes.c_int32 * 4),
                ("k_pred", ctypes.c_int32), ("fallback", ctypes.c_int32), ("feat", ctypes.c_double * 6)]


PREC_FP64, PREC_MIXED = 0, 1
RANK_ADAPTIVE, RANK_LEARNED = 0, 1
MLP_PARAMS, MLP_BLOB = 8833, 8846
ENOCONV = 6


EXPORTS = ["fds_options_default", "fds_build", "fds_size", "fds_rhs_plane", "fds_solve", "fds_apply", "fds_get_stats",
           "fds_get_ranks", "fds_get_skeleton", "fds_get_rank_log", "fds_destroy", "fds_strerror", "fds_last_error",
           "fds_entries", "fds_special_eval", "fds_cpqr_batched", "fds_interp_batched", "fds_lu_batched", "fds_rid_batched", "fds_mlp_init",
           "fds_mlp_forward", "fds_mlp_loss_grad", "fds_mlp_train", "fds_release_cache", "fds_cached_bytes",
           "fds_field", "fds_set_allocator", "fds_solve_noalloc"]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p)
_allocator_refs = None      # the ctypes callbacks in use (kept alive)


def use_torch_allocator():
    """Route every device buffer of the library through PyTorch's caching
    allocator (fds_set_allocator).  Call before the first factorisation or
    after every factor has been destroyed."""
    global _allocator_refs
    import torch

    def _alloc(nbytes, device, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), int(device), int(stream or 0))
        except Exception:      # out of memory: the library reports FDS_ENOMEM
            return None

    def _free(ptr, nbytes, device, stream, ctx):
        torch.cuda.caching_allocator_delete(int(ptr))

    refs = (_ALLOC_FN(_alloc), _FREE_FN(_free))
    _check(load().fds_set_allocator(refs[0], refs[1], None))
    _allocator_refs = refs


def use_library_allocator():
    """Back to the library's own block cache."""
    global _allocator_refs
    _check(load().fds_set_allocator(_ALLOC_FN(), _FREE_FN(), None))
    _allocator_refs = None


def lib_path() -> str:
    return _LIB_PATH


def load():
    """Load libfds.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise FdsError(f"{_LIB_PATH} is missing: build it with `python -m paper_2411_18026_amd.build`")
    # the library works on PyTorch's device memory and streams: let PyTorch
    # bring in the HIP runtime first so that both share one
    import torch  # noqa: F401
    L = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.fds_options_default.argtypes = [ctypes.POINTER(_Options)]
    L.fds_build.argtypes = [ctypes.POINTER(_Geometry), dbl, dbl, dbl, dbl, dbl, ctypes.POINTER(_Options), vp,
                            ctypes.POINTER(vp)]
    L.fds_size.argtypes = [vp, ctypes.POINTER(i64)]
    L.fds_rhs_plane.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl), vp, i64, vp]
    L.fds_solve.argtypes = [vp, i32, vp, i64, vp, i64, vp]
    L.fds_solve_noalloc.argtypes = [vp, i32, vp, i64, vp, i64, vp]
    L.fds_get_stats.argtypes = [vp, ctypes.POINTER(_Stats)]
    L.fds_get_ranks.argtypes = [vp, ctypes.POINTER(i32), i64]
    L.fds_get_skeleton.argtypes = [vp, i32, ctypes.POINTER(i64), ctypes.POINTER(i64), i64, ctypes.POINTER(i64)]
    L.fds_destroy.argtypes = [vp]
    L.fds_destroy.restype = None
    L.fds_strerror.argtypes = [ctypes.c_int]
    L.fds_strerror.restype = ctypes.c_char_p
    L.fds_last_error.argtypes = []
    L.fds_last_error.restype = ctypes.c_char_p
    L.fds_entries.argtypes = [ctypes.POINTER(_Geometry), dbl, dbl, dbl, dbl, ctypes.POINTER(_Options), i64,
                              ctypes.POINTER(i64), i64, ctypes.POINTER(i64), vp, i64, vp]
    L.fds_apply.argtypes = [vp, i32, vp, i64, vp, i64, vp]
    pi64, pi32, pf = ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float)
    L.fds_lu_batched.argtypes = [i32, vp, pi64, pi64, vp, pi64, pi32, vp]
    L.fds_get_rank_log.argtypes = [vp, ctypes.POINTER(_RankRecord), i64, pi64]
    L.fds_rid_batched.argtypes = [i32, vp, pi64, pi64, pi64, pi64, pi64, ctypes.c_uint64, dbl, pi32, pi64, pi32, pi32,
                                  ctypes.POINTER(dbl), vp]
    L.fds_mlp_init.argtypes = [pf, i64, vp, vp, ctypes.c_uint64, vp]
    L.fds_mlp_forward.argtypes = [pf, i64, vp, vp, i32, vp]
    L.fds_mlp_loss_grad.argtypes = [pf, i64, vp, vp, pf, pf, vp]
    L.fds_mlp_train.argtypes = [pf, i64, vp, vp, i32, i64, ctypes.c_float, ctypes.c_uint64, pf, vp]
    L.fds_special_eval.argtypes = [i64, vp, dbl, vp, vp, vp]
    L.fds_field.argtypes = [ctypes.POINTER(_Geometry), dbl, dbl, dbl, dbl, i32, vp, i64, i64, vp,
                            ctypes.POINTER(i32), ctypes.POINTER(dbl), vp, i64, pi64, vp]
    L.fds_release_cache.argtypes = []
    L.fds_release_cache.restype = None
    L.fds_cached_bytes.argtypes = []
    L.fds_cached_bytes.restype = i64
    L.fds_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, vp]
    L.fds_cpqr_batched.argtypes = [i32, vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64), vp,
                                   ctypes.POINTER(i64), ctypes.POINTER(i64), dbl, i32, vp, vp]
    L.fds_interp_batched.argtypes = [i32, vp, pi64, pi64, pi64, vp, pi64, pi32, vp, pi64, vp]
    _lib = L
    return L


def _check(code):
    if code != 0:
        L = load()
        raise FdsError(f"{L.fds_strerror(code).decode()} ({code}): {L.fds_last_error().decode()}", code)


def _geometry(curves):
    arrs = [np.ascontiguousarray(c, dtype=np.float64).reshape(-1, 2) for c in curves]
    n = np.array([len(a) for a in arrs], dtype=np.int32)
    xy = np.ascontiguousarray(np.concatenate(arrs).ravel())
    g = _Geometry(len(arrs), n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                  xy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return g, (n, xy)


def _options(leaf=64, n_proxy=64, root_level=1, proxy_ratio=1.5, alpha=None, solve_graph=False, mixed=False,
             ir_max_iter=None, ir_rtol=None, ir_dtol=None, predictor=None, oversample=None, seed=None, autotune=True,
             mfma_sweeps=True, proxy_fixed=False):
    o = _Options()
    load().fds_options_default(ctypes.byref(o))
    o.leaf_nodes, o.n_proxy, o.root_level, o.proxy_ratio = int(leaf), int(n_proxy), int(root_level), float(proxy_ratio)
    o.solve_graph = int(bool(solve_graph))
    o.precision = PREC_MIXED if mixed else PREC_FP64
    if ir_max_iter is not None:
        o.ir_max_iter = int(ir_max_iter)
    if ir_rtol is not None:
        o.ir_rtol = float(ir_rtol)
    if ir_dtol is not None:
        o.ir_dtol = float(ir_dtol)
    if predictor is not None:
        blob = _blob(predictor)
        o.rank_mode = RANK_LEARNED
        o.predictor = blob.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        o._keep_blob = blob
    if oversample is not None:
        o.oversample = int(oversample)
    if seed is not None:
        o.seed = int(seed)
    o.autotune = int(bool(autotune))
    o.mfma_sweeps = int(bool(mfma_sweeps))
    o.proxy_fixed = int(bool(proxy_fixed))
    if alpha is not None:
        a = complex(alpha)
        o.alpha = _C64(a.real, a.imag)
        o.use_alpha = 1
    return o


def _blob(b):
    b = np.ascontiguousarray(b, dtype=np.float32)
    if b.shape != (MLP_BLOB,):
        raise FdsError(f"a predictor is {MLP_BLOB} float32 values")
    return b


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(int(stream))


def _cuda_c128(t):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.complex128 and t.is_contiguous()):
        raise FdsError("expected a contiguous complex128 CUDA tensor")
    return t


class NotConverged(FdsError):
    """Iterative refinement of the mixed form hit its step limit; ``x`` holds
    the last iterate."""

    def __init__(self, msg, x):
        super().__init__(msg, 6)
        self.x = x


class Factor:
    """Factorisation of the Galerkin Burton-Miller system of a scatterer.

    ``mixed=True`` selects the mixed-precision form (FP32 elimination and
    sweeps, FP64 assembly / IDs / root LU, iterative refinement of every
    solve against the FP64 compressed operator)."""

    def __init__(self, curves, omega, lam, mu, rho, tol, leaf=64, n_proxy=64, root_level=1, proxy_ratio=1.5,
                 alpha=None, stream=None, solve_graph=False, mixed=False, ir_max_iter=None, ir_rtol=None,
                 ir_dtol=None, predictor=None, oversample=None, seed=None, autotune=True, mfma_sweeps=True,
                 proxy_fixed=False):
        L = load()
        g, self._keep = _geometry(curves)
        o = _options(leaf, n_proxy, root_level, proxy_ratio, alpha, solve_graph, mixed, ir_max_iter, ir_rtol,
                     ir_dtol, predictor, oversample, seed, autotune, mfma_sweeps, proxy_fixed)
        h = ctypes.c_void_p()
        _check(L.fds_build(ctypes.byref(g), omega, lam, mu, rho, tol, ctypes.byref(o), _stream(stream),
                           ctypes.byref(h)))
        self._h = h
        n = ctypes.c_int64()
        _check(L.fds_size(h, ctypes.byref(n)))
        self.n_unknowns = int(n.value)

    def close(self):
        if getattr(self, "_h", None):
            load().fds_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def rhs_plane(self, kinds, angles, out=None, stream=None):
        import torch
        kinds = np.ascontiguousarray(kinds, dtype=np.int32)
        angles = np.ascontiguousarray(angles, dtype=np.float64)
        nrhs = len(kinds)
        if out is None:
            out = torch.empty((nrhs, self.n_unknowns), dtype=torch.complex128, device="cuda")
        _cuda_c128(out)
        _check(load().fds_rhs_plane(self._h, nrhs, kinds.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                    angles.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    ctypes.c_void_p(out.data_ptr()), self.n_unknowns, _stream(stream)))
        return out

    def solve(self, rhs, out=None, stream=None):
        import torch
        one = rhs.dim() == 1
        r = rhs.reshape(1, -1) if one else rhs
        _cuda_c128(r)
        if out is None:
            out = torch.empty_like(r)
        code = load().fds_solve(self._h, r.shape[0], ctypes.c_void_p(r.data_ptr()), self.n_unknowns,
                                ctypes.c_void_p(out.data_ptr()), self.n_unknowns, _stream(stream))
        if code == ENOCONV:
            raise NotConverged(load().fds_last_error().decode(), out[0] if one else out)
        _check(code)
        return out[0] if one else out

    def solve_noalloc(self, rhs, out, stream=None):
        """fds_solve_noalloc: as ``solve`` for a plain FP64 factor, with the
        sweeps' level vectors in the library's fixed device scratch; ``out``
        (the shape of ``rhs``) is required.  Asynchronous on ``stream``."""
        one = rhs.dim() == 1
        r = rhs.reshape(1, -1) if one else rhs
        o = out.reshape(1, -1) if one else out
        _cuda_c128(r)
        _cuda_c128(o)
        if o.shape != r.shape:
            raise FdsError("out must have the shape of rhs")
        _check(load().fds_solve_noalloc(self._h, r.shape[0], ctypes.c_void_p(r.data_ptr()), self.n_unknowns,
                                        ctypes.c_void_p(o.data_ptr()), self.n_unknowns, _stream(stream)))
        return out

    def apply(self, x, out=None, stream=None):
        """y = A_c x with the FP64 compressed operator (mixed-form factors)."""
        import torch
        one = x.dim() == 1
        v = x.reshape(1, -1) if one else x
        _cuda_c128(v)
        if out is None:
            out = torch.empty_like(v)
        _check(load().fds_apply(self._h, v.shape[0], ctypes.c_void_p(v.data_ptr()), self.n_unknowns,
                                ctypes.c_void_p(out.data_ptr()), self.n_unknowns, _stream(stream)))
        return out[0] if one else out

    def stats(self):
        s = _Stats()
        _check(load().fds_get_stats(self._h, ctypes.byref(s)))
        out = {}
        for f, _ in _Stats._fields_:
            if f.startswith("reserved"):
                continue
            v = getattr(s, f)
            out[f] = list(v) if hasattr(v, "__len__") else v
        return out

    def rank_log(self):
        """Per compressed cell: dict of arrays cell, level, rank (n x 4),
        k_pred, fallback, feat (n x 6)."""
        L = load()
        n = ctypes.c_int64()
        _check(L.fds_get_rank_log(self._h, None, 0, ctypes.byref(n)))
        recs = (_RankRecord * max(1, n.value))()
        _check(L.fds_get_rank_log(self._h, recs, n.value, ctypes.byref(n)))
        recs = recs[:n.value]
        return {"cell": np.array([r.cell for r in recs], np.int32),
                "level": np.array([r.level for r in recs], np.int32),
                "rank": np.array([list(r.rank) for r in recs], np.int32).reshape(-1, 4),
                "k_pred": np.array([r.k_pred for r in recs], np.int32),
                "fallback": np.array([r.fallback for r in recs], np.int32),
                "feat": np.array([list(r.feat) for r in recs], np.float64).reshape(-1, 6)}

    def ranks(self):
        st = self.stats()
        ncell = (2 << st["levels"]) - 1
        out = np.zeros(4 * ncell, dtype=np.int32)
        _check(load().fds_get_ranks(self._h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), len(out)))
        return out.reshape(ncell, 4)

    def skeleton(self, cell):
        cap = 1 << 16
        r = np.zeros(cap, np.int64)
        c = np.zeros(cap, np.int64)
        n = ctypes.c_int64()
        _check(load().fds_get_skeleton(self._h, int(cell), r.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                       c.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), cap, ctypes.byref(n)))
        return r[:n.value].copy(), c[:n.value].copy()


def release_cache():
    """Hand the library's cached device blocks back to the runtime."""
    load().fds_release_cache()


def cached_bytes() -> int:
    """Bytes of device memory held by the library's block cache."""
    return int(load().fds_cached_bytes())


def entries(curves, omega, lam, mu, rho, rows, cols, alpha=None, stream=None):
    """Galerkin entries A(rows, cols) computed by the GPU assembly kernels;
    returns a complex128 CUDA tensor of shape (len(rows), len(cols))."""
    import torch
    L = load()
    g, keep = _geometry(curves)
    o = _options(alpha=alpha)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = torch.empty((len(cols), len(rows)), dtype=torch.complex128, device="cuda")   # column-major nr x nc
    _check(L.fds_entries(ctypes.byref(g), omega, lam, mu, rho, ctypes.byref(o), len(rows),
                         rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(cols),
                         cols.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.c_void_p(out.data_ptr()),
                         len(rows), _stream(stream)))
    return out.t()


def field(curves, omega, lam, mu, rho, x, targets, kinds=None, angles=None, stream=None):
    """Displacement at ``targets`` (M x 2 points of the solid) from boundary
    solutions ``x`` ((nrhs, 2N) or (2N,) complex128 CUDA tensor) by the
    integral representation, computed by the GPU field kernels.  With
    ``kinds``/``angles`` (the plane wave of each solution) the incident
    field is added.  Returns (out, n_near): out of shape (nrhs, M, 2)
    complex128 on the GPU (or (M, 2) for a single vector), n_near the number
    of targets closer to some element than 1/64 of its length."""
    import torch
    L = load()
    g, keep = _geometry(curves)
    one = x.dim() == 1
    X = x.reshape(1, -1) if one else x
    _cuda_c128(X)
    t = torch.as_tensor(targets, dtype=torch.float64).reshape(-1, 2).to("cuda").contiguous()
    nrhs, M = X.shape[0], t.shape[0]
    out = torch.empty((nrhs, max(M, 1), 2), dtype=torch.complex128, device="cuda")
    kp = ap = None
    if kinds is not None:
        k = np.ascontiguousarray(kinds, dtype=np.int32)
        a = np.ascontiguousarray(angles, dtype=np.float64)
        if len(k) != nrhs or len(a) != nrhs:
            raise ValueError("one incident wave per solution")
        kp = k.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        ap = a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    nn = ctypes.c_int64()
    _check(L.fds_field(ctypes.byref(g), omega, lam, mu, rho, nrhs, ctypes.c_void_p(X.data_ptr()), X.stride(0), M,
                       ctypes.c_void_p(t.data_ptr()), kp, ap, ctypes.c_void_p(out.data_ptr()), 2 * max(M, 1),
                       ctypes.byref(nn), _stream(stream)))
    out = out[:, :M]
    return (out[0] if one else out), int(nn.value)


def special_eval(x, beta, stream=None):
    """(J0, J1, Y0, Y1) and (E, chi) evaluated by the device special functions."""
    import torch
    L = load()
    x = x.to(device="cuda", dtype=torch.float64).contiguous()
    out = torch.empty((x.numel(), 4), dtype=torch.float64, device="cuda")
    outc = torch.empty((x.numel(), 2), dtype=torch.complex128, device="cuda")
    _check(L.fds_special_eval(x.numel(), ctypes.c_void_p(x.data_ptr()), float(beta), ctypes.c_void_p(out.data_ptr()),
                              ctypes.c_void_p(outc.data_ptr()), _stream(stream)))
    return out, outc


def cpqr_batched(mats, tol, kmax=None, stop_at_tol=True, stream=None, interp=False):
    """Column-pivoted QR of a list of complex matrices on the GPU.  Returns
    (pivots, ranks, R-factors) with R the top ``rank`` rows of the reduced
    matrix in pivoted column order; with ``interp`` also the interpolation
    matrix W (rank x n) of each ID, M ~ M[:, piv[:rank]] W."""
    import torch
    L = load()
    ms = [np.asarray(m, dtype=np.complex128) for m in mats]
    offs, mm, nn, pvo, km = [], [], [], [], []
    o = p = 0
    for i, m in enumerate(ms):
        offs.append(o)
        mm.append(m.shape[0])
        nn.append(m.shape[1])
        pvo.append(p)
        km.append(min(m.shape) if kmax is None else int(kmax[i]))
        o += m.size
        p += m.shape[1]
    flat = np.concatenate([m.T.ravel() for m in ms])       # column-major
    dev = torch.from_numpy(flat).to("cuda")
    piv = torch.zeros(p, dtype=torch.int32, device="cuda")
    rank = torch.zeros(len(ms), dtype=torch.int32, device="cuda")
    arr = lambda v: np.ascontiguousarray(v, dtype=np.int64)
    a_off, a_m, a_n, a_pv, a_k = arr(offs), arr(mm), arr(nn), arr(pvo), arr(km)
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    _check(L.fds_cpqr_batched(len(ms), ctypes.c_void_p(dev.data_ptr()), P(a_off), P(a_m), P(a_n),
                              ctypes.c_void_p(piv.data_ptr()), P(a_pv), P(a_k), float(tol), int(bool(stop_at_tol)),
                              ctypes.c_void_p(rank.data_ptr()), _stream(stream)))
    flat_out = dev.cpu().numpy()
    pv = piv.cpu().numpy()
    rk = rank.cpu().numpy()
    res = []
    for i, m in enumerate(ms):
        A = flat_out[offs[i]:offs[i] + m.size].reshape(m.shape[1], m.shape[0]).T
        k = int(rk[i])
        res.append((pv[pvo[i]:pvo[i] + m.shape[1]].copy(), k, np.triu(A[:k, :])))
    if not interp:
        return res
    rk32 = np.ascontiguousarray(rk, dtype=np.int32)
    woff = np.concatenate([[0], np.cumsum([int(rk[i]) * nn[i] for i in range(len(ms))])]).astype(np.int64)
    w = torch.zeros(max(int(woff[-1]), 1), dtype=torch.complex128, device="cuda")
    _check(L.fds_interp_batched(len(ms), ctypes.c_void_p(dev.data_ptr()), P(a_off), P(a_m), P(a_n),
                                ctypes.c_void_p(piv.data_ptr()), P(a_pv),
                                rk32.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), ctypes.c_void_p(w.data_ptr()),
                                P(np.ascontiguousarray(woff[:-1])), _stream(stream)))
    wh = w.cpu().numpy()
    out = []
    for i, (pv_i, k, R) in enumerate(res):
        W = wh[woff[i]:woff[i] + k * nn[i]].reshape(nn[i], k).T
        out.append((pv_i, k, R, W))
    return out


def rid_batched(mats, sizes, tol, seed, gids=None, stream=None):
    """Randomized IDs with residual judge on the GPU; returns per matrix
    (piv, rank, revealed, ratio)."""
    import torch
    L = load()
    ms = [np.asarray(m, dtype=np.complex128) for m in mats]
    offs, mm, nn, pvo = [], [], [], []
    o = p = 0
    for m in ms:
        offs.append(o)
        mm.append(m.shape[0])
        nn.append(m.shape[1])
        pvo.append(p)
        o += m.size
        p += m.shape[1]
    buf = torch.from_numpy(np.concatenate([np.asfortranarray(m).ravel(order="F") for m in ms])).to("cuda")
    a64 = lambda v: np.ascontiguousarray(v, dtype=np.int64)
    offs, mm, nn, pvo, ss = a64(offs), a64(mm), a64(nn), a64(pvo), a64(sizes)
    gids = a64(np.arange(len(ms)) if gids is None else gids)
    piv = np.zeros(p, np.int32)
    rank = np.zeros(len(ms), np.int32)
    rev = np.zeros(len(ms), np.int32)
    ratio = np.zeros(len(ms), np.float64)
    P = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
    _check(L.fds_rid_batched(len(ms), ctypes.c_void_p(buf.data_ptr()), P(offs, ctypes.c_int64),
                             P(mm, ctypes.c_int64), P(nn, ctypes.c_int64), P(ss, ctypes.c_int64),
                             P(gids, ctypes.c_int64), int(seed), float(tol), P(piv, ctypes.c_int32),
                             P(pvo, ctypes.c_int64), P(rank, ctypes.c_int32), P(rev, ctypes.c_int32),
                             P(ratio, ctypes.c_double), _stream(stream)))
    return [(piv[pvo[i]:pvo[i] + nn[i]].copy(), int(rank[i]), bool(rev[i]), float(ratio[i])) for i in range(len(ms))]


def _f32_cuda(a, shape):
    import torch
    t = a if isinstance(a, torch.Tensor) else torch.as_tensor(np.asarray(a, dtype=np.float32))
    t = t.to(device="cuda", dtype=torch.float32).contiguous()
    if tuple(t.shape) != tuple(shape):
        raise FdsError(f"expected shape {shape}, got {tuple(t.shape)}")
    return t


def mlp_init(x, y, seed, stream=None):
    """A fresh predictor blob (float32 [MLP_BLOB]) for features x (n x 6) and targets y (n)."""
    n = len(y)
    xt, yt = _f32_cuda(x, (n, 6)), _f32_cuda(y, (n,))
    blob = np.zeros(MLP_BLOB, np.float32)
    _check(load().fds_mlp_init(blob.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n, ctypes.c_void_p(xt.data_ptr()),
                               ctypes.c_void_p(yt.data_ptr()), int(seed), _stream(stream)))
    return blob


def mlp_forward(blob, x, bf16=False, stream=None):
    """Predictions (float32 CUDA tensor [n]) of a predictor blob for features x (n x 6)."""
    import torch
    b = _blob(blob)
    n = len(x)
    xt = _f32_cuda(x, (n, 6))
    y = torch.empty(n, dtype=torch.float32, device="cuda")
    _check(load().fds_mlp_forward(b.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), n, ctypes.c_void_p(xt.data_ptr()),
                                  ctypes.c_void_p(y.data_ptr()), int(bool(bf16)), _stream(stream)))
    return y


def mlp_loss_grad(blob, x, y, stream=None):
    """(loss, gradient [MLP_PARAMS]) of the mean squared error over all rows."""
    b = _blob(blob)
    n = len(y)
    xt, yt = _f32_cuda(x, (n, 6)), _f32_cuda(y, (n,))
    g = np.zeros(MLP_PARAMS, np.float32)
    loss = np.zeros(1, np.float32)
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    _check(load().fds_mlp_loss_grad(P(b), n, ctypes.c_void_p(xt.data_ptr()), ctypes.c_void_p(yt.data_ptr()), P(g),
                                    P(loss), _stream(stream)))
    return float(loss[0]), g


def mlp_train(blob, x, y, steps, batch, lr, seed, stream=None):
    """Adam training on the GPU; returns (trained blob, loss history)."""
    b = _blob(blob).copy()
    n = len(y)
    xt, yt = _f32_cuda(x, (n, 6)), _f32_cuda(y, (n,))
    hist = np.zeros(max(1, steps), np.float32)
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
    _check(load().fds_mlp_train(P(b), n, ctypes.c_void_p(xt.data_ptr()), ctypes.c_void_p(yt.data_ptr()), int(steps),
                                int(batch), float(lr), int(seed), P(hist), _stream(stream)))
    return b, hist[:steps]


def lu_batched(mats, stream=None):
    """LU with partial pivoting of square complex matrices on the GPU.
    Returns per matrix (LU packed as LAPACK does, pivots, info)."""
    import torch
    L = load()
    ms = [np.asarray(m, dtype=np.complex128) for m in mats]
    offs, nn, pvo = [], [], []
    o = p = 0
    for m in ms:
        offs.append(o)
        nn.append(m.shape[0])
        pvo.append(p)
        o += m.size
        p += m.shape[0]
    dev = torch.from_numpy(np.concatenate([m.T.ravel() for m in ms])).to("cuda")
    piv = torch.zeros(p, dtype=torch.int32, device="cuda")
    info = np.zeros(len(ms), np.int32)
    a64 = lambda v: np.ascontiguousarray(v, dtype=np.int64)
    offs, nn, pvo = a64(offs), a64(nn), a64(pvo)
    P = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
    _check(L.fds_lu_batched(len(ms), ctypes.c_void_p(dev.data_ptr()), P(offs, ctypes.c_int64), P(nn, ctypes.c_int64),
                            ctypes.c_void_p(piv.data_ptr()), P(pvo, ctypes.c_int64), P(info, ctypes.c_int32),
                            _stream(stream)))
    flat = dev.cpu().numpy()
    pv = piv.cpu().numpy()
    return [(flat[offs[i]:offs[i] + m.size].reshape(m.shape[1], m.shape[0]).T.copy(), pv[pvo[i]:pvo[i] + nn[i]].copy(),
             int(info[i])) for i, m in enumerate(ms)]
