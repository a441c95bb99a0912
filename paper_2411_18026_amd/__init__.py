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
    pass


class _C64(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class _Geometry(ctypes.Structure):
    _fields_ = [("n_curves", ctypes.c_int32), ("n_nodes", ctypes.POINTER(ctypes.c_int32)),
                ("xy", ctypes.POINTER(ctypes.c_double))]


class _Options(ctypes.Structure):
    _fields_ = [("leaf_nodes", ctypes.c_int32), ("n_proxy", ctypes.c_int32), ("root_level", ctypes.c_int32),
                ("solve_graph", ctypes.c_int32), ("proxy_ratio", ctypes.c_double), ("alpha", _C64),
                ("use_alpha", ctypes.c_int32), ("precision", ctypes.c_int32), ("ir_max_iter", ctypes.c_int32),
                ("reserved1", ctypes.c_int32), ("ir_rtol", ctypes.c_double), ("ir_dtol", ctypes.c_double)]


class _Stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("root_level", ctypes.c_int32), ("n_unknowns", ctypes.c_int64),
                ("root_size", ctypes.c_int64), ("max_rank", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("factor_seconds", ctypes.c_double), ("assembly_seconds", ctypes.c_double),
                ("id_seconds", ctypes.c_double), ("merge_seconds", ctypes.c_double),
                ("root_seconds", ctypes.c_double), ("factor_bytes", ctypes.c_int64),
                ("kernel_evals", ctypes.c_int64), ("class_seconds", ctypes.c_double * 6),
                ("class_evals", ctypes.c_int64 * 6), ("class_launches", ctypes.c_int64 * 6),
                ("precision", ctypes.c_int32), ("ir_iterations", ctypes.c_int32), ("ir_residual", ctypes.c_double),
                ("ir_correction", ctypes.c_double)]

PREC_FP64, PREC_MIXED = 0, 1
ENOCONV = 6


EXPORTS = ["fds_options_default", "fds_build", "fds_size", "fds_rhs_plane", "fds_solve", "fds_apply", "fds_get_stats",
           "fds_get_ranks", "fds_get_skeleton", "fds_destroy", "fds_strerror", "fds_last_error",
           "fds_entries", "fds_special_eval", "fds_cpqr_batched"]


def lib_path() -> str:
    return _LIB_PATH


def load():
    """Load libfds.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise FdsError(f"{_LIB_PATH} is missing: build it with `python -m paper_2411_18026_amd.build`")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.fds_options_default.argtypes = [ctypes.POINTER(_Options)]
    L.fds_build.argtypes = [ctypes.POINTER(_Geometry), dbl, dbl, dbl, dbl, dbl, ctypes.POINTER(_Options), vp,
                            ctypes.POINTER(vp)]
    L.fds_size.argtypes = [vp, ctypes.POINTER(i64)]
    L.fds_rhs_plane.argtypes = [vp, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl), vp, i64, vp]
    L.fds_solve.argtypes = [vp, i32, vp, i64, vp, i64, vp]
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
    L.fds_special_eval.argtypes = [i64, vp, dbl, vp, vp, vp]
    L.fds_cpqr_batched.argtypes = [i32, vp, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i64), vp,
                                   ctypes.POINTER(i64), ctypes.POINTER(i64), dbl, i32, vp, vp]
    _lib = L
    return L


def _check(code):
    if code != 0:
        L = load()
        raise FdsError(f"{L.fds_strerror(code).decode()} ({code}): {L.fds_last_error().decode()}")


def _geometry(curves):
    arrs = [np.ascontiguousarray(c, dtype=np.float64).reshape(-1, 2) for c in curves]
    n = np.array([len(a) for a in arrs], dtype=np.int32)
    xy = np.ascontiguousarray(np.concatenate(arrs).ravel())
    g = _Geometry(len(arrs), n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                  xy.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return g, (n, xy)


def _options(leaf=64, n_proxy=64, root_level=1, proxy_ratio=1.5, alpha=None, solve_graph=False, mixed=False,
             ir_max_iter=None, ir_rtol=None, ir_dtol=None):
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
    if alpha is not None:
        a = complex(alpha)
        o.alpha = _C64(a.real, a.imag)
        o.use_alpha = 1
    return o


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
        super().__init__(msg)
        self.x = x


class Factor:
    """Factorisation of the Galerkin Burton-Miller system of a scatterer.

    ``mixed=True`` selects the mixed-precision form (FP32 elimination and
    sweeps, FP64 assembly / IDs / root LU, iterative refinement of every
    solve against the FP64 compressed operator)."""

    def __init__(self, curves, omega, lam, mu, rho, tol, leaf=64, n_proxy=64, root_level=1, proxy_ratio=1.5,
                 alpha=None, stream=None, solve_graph=False, mixed=False, ir_max_iter=None, ir_rtol=None,
                 ir_dtol=None):
        L = load()
        g, self._keep = _geometry(curves)
        o = _options(leaf, n_proxy, root_level, proxy_ratio, alpha, solve_graph, mixed, ir_max_iter, ir_rtol,
                     ir_dtol)
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


def cpqr_batched(mats, tol, kmax=None, stop_at_tol=True, stream=None):
    """Column-pivoted QR of a list of complex matrices on the GPU.  Returns
    (pivots, ranks, R-factors) with R the top ``rank`` rows of the reduced
    matrix in pivoted column order."""
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
    return res
