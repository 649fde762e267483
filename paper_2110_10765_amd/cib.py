"""Thin Python binding of libcib.so (argument marshalling only).

Every step of the computation runs in the library's HIP kernels; this module
converts Python objects to the C structs of include/cib.h, keeps host arrays
alive for the duration of a call and turns error codes into exceptions.
torch is used only for device memory and the current HIP stream.
"""
from __future__ import annotations

import ctypes
import os
import weakref
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcib.so")

CIB_OK = 0
CIB_E_INVALID = -1
CIB_E_NOMEM = -2
CIB_E_DEVICE = -3
CIB_E_NOT_CONVERGED = -4
CIB_E_OVERFLOW = -5
CIB_E_EMPTY_BASIS = -6
CIB_E_BUSY = -7
CIB_E_CANCELLED = -8
CIB_F64 = 0
CIB_F32 = 1

STATUS_NAMES = {0: "CIB_OK", -1: "CIB_E_INVALID", -2: "CIB_E_NOMEM", -3: "CIB_E_DEVICE",
                -4: "CIB_E_NOT_CONVERGED", -5: "CIB_E_OVERFLOW", -6: "CIB_E_EMPTY_BASIS",
                -7: "CIB_E_BUSY", -8: "CIB_E_CANCELLED"}

# every symbol include/cib.h declares
EXPORTS = [
    "cib_create", "cib_destroy", "cib_last_error", "cib_ctx_bytes",
    "cib_profile_enable", "cib_profile_reset", "cib_profile_query",
    "cib_build_basis", "cib_basis_info", "cib_basis_export", "cib_basis_free",
    "cib_upload_interaction", "cib_interaction_free",
    "cib_build_H", "cib_build_H_resident", "cib_matrix_info", "cib_matrix_stats",
    "cib_matrix_export", "cib_matrix_device", "cib_matrix_free",
    "cib_apply_H", "cib_apply_H_free", "cib_observables", "cib_count_states",
    "cib_count_states_noalloc", "cib_lobpcg", "cib_lanczos",
    "cib_tridiag_lowest", "cib_serve",
    "cib_precond_create", "cib_precond_info", "cib_precond_export", "cib_precond_apply", "cib_precond_free",
]


class CibError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(code, code), msg))
        self.code = code


# ------------------------------------------------------------------ C structs
class BasisSpecC(ctypes.Structure):
    _fields_ = [("n_species", ctypes.c_int32), ("nmax", ctypes.c_int32 * 2),
                ("n_particles", ctypes.c_int32 * 2), ("two_M", ctypes.c_int32),
                ("cut", ctypes.c_int32)]


class TablesC(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_void_p * 2), ("v_same", ctypes.c_void_p * 2),
                ("v_ab", ctypes.c_void_p)]


class AllocatorC(ctypes.Structure):
    _fields_ = [("alloc", ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)),
                ("free", ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)),
                ("user", ctypes.c_void_p)]


class BuildStatsC(ctypes.Structure):
    _fields_ = [("t_screen_s", ctypes.c_double), ("t_count_s", ctypes.c_double),
                ("t_scan_s", ctypes.c_double), ("t_fill_s", ctypes.c_double),
                ("t_total_s", ctypes.c_double), ("n_tiles", ctypes.c_int64),
                ("n_adjacent", ctypes.c_int64)]


class LobpcgOptsC(ctypes.Structure):
    _fields_ = [("nev", ctypes.c_int32), ("block", ctypes.c_int32), ("max_iter", ctypes.c_int32),
                ("tol", ctypes.c_double), ("seed", ctypes.c_uint64), ("x0", ctypes.c_void_p),
                ("precond", ctypes.c_void_p)]


class LobpcgInfoC(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("n_converged", ctypes.c_int32),
                ("resid", ctypes.c_double * 64), ("t_total_s", ctypes.c_double),
                ("t_spmm_s", ctypes.c_double), ("n_spmm", ctypes.c_int64)]


class LanczosOptsC(ctypes.Structure):
    _fields_ = [("nev", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("tol", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


class LanczosInfoC(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("n_converged", ctypes.c_int32),
                ("resid", ctypes.c_double * 64), ("t_total_s", ctypes.c_double),
                ("t_spmv_s", ctypes.c_double)]


class RequestC(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("arrival_s", ctypes.c_double), ("basis", BasisSpecC),
                ("tables", ctypes.POINTER(TablesC)), ("dtype", ctypes.c_int32),
                ("solve", LobpcgOptsC)]


class ResultC(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("status", ctypes.c_int32), ("dim", ctypes.c_int64),
                ("nnz_half", ctypes.c_int64), ("iters", ctypes.c_int32),
                ("evals", ctypes.c_double * 16), ("resid", ctypes.c_double * 16),
                ("t_arrive", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double)]


class ServeOptsC(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_active", ctypes.c_int32),
                ("realtime", ctypes.c_int32), ("deadline_s", ctypes.c_double),
                ("n_streams", ctypes.c_int32)]


_LIB = None


def load(path: str = LIB_PATH):
    """Load libcib.so; raises if it has not been built (no fallback exists)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    # torch ships its own HIP/HSA runtime with the same sonames as /opt/rocm's;
    # loading torch first makes libcib bind to that one runtime instead of
    # bringing a second HIP + HSA runtime into the process (which then finds
    # no device)
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError("libcib.so not found at %s: run `python -m paper_2110_10765_amd.build`" % path)
    lib = ctypes.CDLL(path)
    P, vp, i32, i64 = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "cib_create": ([ctypes.c_int, P(AllocatorC), vp, P(vp)], i32),
        "cib_destroy": ([vp], None),
        "cib_last_error": ([], ctypes.c_char_p),
        "cib_ctx_bytes": ([vp, P(i64), P(i64)], i32),
        "cib_profile_enable": ([vp, ctypes.c_int], i32),
        "cib_profile_reset": ([vp], i32),
        "cib_profile_query": ([vp, ctypes.c_char_p, P(i64), P(ctypes.c_double)], i32),
        "cib_build_basis": ([vp, P(BasisSpecC), P(vp), P(i64)], i32),
        "cib_basis_info": ([vp, P(i64), P(i32), P(i32), P(i64)], i32),
        "cib_basis_export": ([vp, vp], i32),
        "cib_basis_free": ([vp], None),
        "cib_upload_interaction": ([vp, vp, P(TablesC), P(vp)], i32),
        "cib_interaction_free": ([vp], None),
        "cib_build_H": ([vp, vp, P(TablesC), i32, P(vp), P(i64)], i32),
        "cib_build_H_resident": ([vp, vp, vp, i32, P(vp), P(i64)], i32),
        "cib_matrix_info": ([vp, P(i64), P(i64), P(i32)], i32),
        "cib_matrix_stats": ([vp, P(BuildStatsC)], i32),
        "cib_matrix_export": ([vp, vp, vp, vp], i32),
        "cib_matrix_device": ([vp, P(vp), P(vp), P(vp)], i32),
        "cib_matrix_free": ([vp], None),
        "cib_apply_H": ([vp, vp, vp, i64, vp, i64, i32], i32),
        "cib_observables": ([vp, vp, vp, i32, i32, vp, i64, i32, vp], i32),
        "cib_apply_H_free": ([vp, vp, vp, i32, vp, i64, vp, i64, i32], i32),
        "cib_count_states": ([vp, vp, i64, i32, i32, i32, vp, P(i64)], i32),
        "cib_count_states_noalloc": ([vp, vp, i64, i32, i32, i32, vp, P(i64)], i32),
        "cib_lobpcg": ([vp, vp, P(LobpcgOptsC), vp, vp, i64, P(LobpcgInfoC)], i32),
        "cib_lanczos": ([vp, vp, P(LanczosOptsC), vp, vp, i64, P(LanczosInfoC)], i32),
        "cib_tridiag_lowest": ([vp, vp, i32, i32, vp, vp], i32),
        "cib_serve": ([vp, P(RequestC), i32, P(ServeOptsC), P(ResultC)], i32),
        "cib_precond_create": ([vp, vp, vp, i32, P(vp)], i32),
        "cib_precond_info": ([vp, P(i64), P(i64), P(i32), P(i32)], i32),
        "cib_precond_export": ([vp, vp, vp], i32),
        "cib_precond_apply": ([vp, vp, vp, vp, i64, vp, i64, i32], i32),
        "cib_precond_free": ([vp], None),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _LIB = lib
    return lib


def _check(rc, allow=()):
    if rc != CIB_OK and rc not in allow:
        msg = load().cib_last_error()
        raise CibError(rc, msg.decode() if msg else "")
    return rc


def _spec_c(spec) -> BasisSpecC:
    s = BasisSpecC()
    s.n_species = int(spec.n_species)
    s.nmax[0], s.nmax[1] = int(spec.nmax[0]), int(spec.nmax[1])
    s.n_particles[0], s.n_particles[1] = int(spec.n_particles[0]), int(spec.n_particles[1])
    s.two_M = int(spec.two_M)
    s.cut = int(spec.cut)
    return s


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class _TablesHolder:
    """Keeps the float64 host arrays alive while C holds pointers to them."""

    def __init__(self, tables):
        self.arrays = [_f64(tables.eps[0]), _f64(tables.v_same[0])]
        t = TablesC()
        t.eps[0] = self.arrays[0].ctypes.data
        t.v_same[0] = self.arrays[1].ctypes.data
        if len(tables.eps) > 1:
            e1, v1, vab = _f64(tables.eps[1]), _f64(tables.v_same[1]), _f64(tables.v_ab)
            self.arrays += [e1, v1, vab]
            t.eps[1], t.v_same[1], t.v_ab = e1.ctypes.data, v1.ctypes.data, vab.ctypes.data
        self.c = t


def _dtype_code(dtype) -> int:
    if dtype in ("f64", "float64", CIB_F64):
        return CIB_F64
    if dtype in ("f32", "float32", CIB_F32):
        return CIB_F32
    import torch
    if dtype == torch.float64:
        return CIB_F64
    if dtype == torch.float32:
        return CIB_F32
    raise ValueError("dtype must be f64 or f32")


class Context:
    """cib_ctx on one device, issuing its work on a torch stream (a new
    default-priority one unless `stream` is given), so that torch tensors and
    library work can be ordered with stream waits."""

    def __init__(self, device: int = 0, stream=None, torch_allocator: bool = False, allocator=None):
        """allocator: optional (alloc(nbytes) -> int address or None,
        free(address)) Python callables for the library's device memory;
        torch_allocator=True uses torch's caching allocator."""
        lib = load()
        import torch
        if stream is None:
            stream = torch.cuda.Stream(device=device)
        self._alloc = None
        ap = None
        if torch_allocator and allocator is None:
            dev = device
            allocator = (lambda n: torch.cuda.caching_allocator_alloc(int(n), dev),
                         torch.cuda.caching_allocator_delete)
        if allocator is not None:
            alloc_fn, free_fn = allocator

            @ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
            def _a(n, user):
                try:
                    return alloc_fn(int(n))
                except Exception:
                    return None

            @ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
            def _f(p, user):
                free_fn(p)

            self._alloc = AllocatorC(_a, _f, None)
            self._hooks = (_a, _f)
            ap = ctypes.byref(self._alloc)
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib.cib_create(device, ap, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.device = device

    def close(self):
        """Free every handle still made on this context that is reachable,
        then the context.  Handles the cyclic garbage collector finalizes
        later (it clears the weak set first and runs finalizers in any order)
        are still safe: the library keeps a destroyed context until its last
        handle is freed."""
        if getattr(self, "h", None):
            for child in list(getattr(self, "_children", ())):
                child.free()
            load().cib_destroy(self.h)
            self.h = None

    def _adopt(self, child):
        if not hasattr(self, "_children"):
            self._children = weakref.WeakSet()
        self._children.add(child)
        return child

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile(self, on: bool = True):
        _check(load().cib_profile_enable(self.h, int(on)))
        _check(load().cib_profile_reset(self.h))

    def kernel_time(self, name: str):
        """(launches, total seconds) of one library kernel since profile()."""
        n, t = ctypes.c_int64(), ctypes.c_double()
        _check(load().cib_profile_query(self.h, name.encode(), ctypes.byref(n), ctypes.byref(t)))
        return n.value, t.value

    def bytes(self):
        live, peak = ctypes.c_int64(), ctypes.c_int64()
        _check(load().cib_ctx_bytes(self.h, ctypes.byref(live), ctypes.byref(peak)))
        return live.value, peak.value


class Basis:
    def __init__(self, ctx: Context, h, dim):
        self.ctx, self.h, self.dim = ctx, h, dim
        ctx._adopt(self)

    def info(self):
        d, nab = ctypes.c_int64(), ctypes.c_int64()
        w, no = (ctypes.c_int32 * 2)(), (ctypes.c_int32 * 2)()
        _check(load().cib_basis_info(self.h, ctypes.byref(d), w, no, ctypes.byref(nab)))
        return dict(dim=d.value, words=(w[0], w[1]), n_orb=(no[0], no[1]), n_ablocks=nab.value)

    def export(self) -> np.ndarray:
        inf = self.info()
        nw = inf["words"][0] + inf["words"][1]
        out = np.zeros((self.dim, nw), dtype=np.uint64)
        _check(load().cib_basis_export(self.h, out.ctypes.data))
        return out

    def free(self):
        if self.h:
            load().cib_basis_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Interaction:
    def __init__(self, ctx, h):
        self.ctx, self.h = ctx, h
        ctx._adopt(self)

    def free(self):
        if self.h:
            load().cib_interaction_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


class Matrix:
    def __init__(self, ctx: Context, h):
        self.ctx, self.h = ctx, h
        ctx._adopt(self)
        d, n, t = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        _check(load().cib_matrix_info(h, ctypes.byref(d), ctypes.byref(n), ctypes.byref(t)))
        self.dim, self.nnz, self.dtype = d.value, n.value, ("f64" if t.value == CIB_F64 else "f32")

    def stats(self):
        s = BuildStatsC()
        _check(load().cib_matrix_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in BuildStatsC._fields_}

    def export(self):
        rp = np.zeros(self.dim + 1, dtype=np.int64)
        col = np.zeros(self.nnz, dtype=np.int32)
        val = np.zeros(self.nnz, dtype=np.float64 if self.dtype == "f64" else np.float32)
        _check(load().cib_matrix_export(self.h, rp.ctypes.data, col.ctypes.data, val.ctypes.data))
        return rp, col, val

    def device_ptrs(self):
        a, b, c = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _check(load().cib_matrix_device(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def free(self):
        if self.h:
            load().cib_matrix_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ------------------------------------------------------------------ the ABI calls
def build_basis(ctx: Context, spec) -> Basis:
    s = _spec_c(spec)
    h, d = ctypes.c_void_p(), ctypes.c_int64()
    _check(load().cib_build_basis(ctx.h, ctypes.byref(s), ctypes.byref(h), ctypes.byref(d)))
    return Basis(ctx, h, d.value)


def upload_interaction(ctx: Context, basis: Basis, tables) -> Interaction:
    th = _TablesHolder(tables)
    h = ctypes.c_void_p()
    _check(load().cib_upload_interaction(ctx.h, basis.h, ctypes.byref(th.c), ctypes.byref(h)))
    return Interaction(ctx, h)


def build_H(ctx: Context, basis: Basis, tables, dtype="f64") -> Matrix:
    h, n = ctypes.c_void_p(), ctypes.c_int64()
    if isinstance(tables, Interaction):
        _check(load().cib_build_H_resident(ctx.h, basis.h, tables.h, _dtype_code(dtype),
                                           ctypes.byref(h), ctypes.byref(n)))
    else:
        th = _TablesHolder(tables)
        _check(load().cib_build_H(ctx.h, basis.h, ctypes.byref(th.c), _dtype_code(dtype),
                                  ctypes.byref(h), ctypes.byref(n)))
    return Matrix(ctx, h)


def apply_H(ctx: Context, H: Matrix, X, Y=None):
    """Y = H X for torch device tensors X (D x nvec, row-major, matrix dtype)."""
    import torch
    want = torch.float64 if H.dtype == "f64" else torch.float32
    if X.dtype != want or X.dim() != 2 or X.shape[0] != H.dim or X.stride(1) != 1:
        raise ValueError("X must be a (D, nvec) %s tensor with unit column stride" % want)
    if Y is None:
        Y = torch.empty_like(X)
    if Y.dtype != want or Y.shape != X.shape or Y.stride(1) != 1:
        raise ValueError("Y must match X")
    cur = torch.cuda.current_stream(X.device)
    ctx.stream.wait_stream(cur)          # X, Y are ready on the caller's stream
    _check(load().cib_apply_H(ctx.h, H.h, X.data_ptr(), X.stride(0), Y.data_ptr(), Y.stride(0),
                              X.shape[1]))
    cur.wait_stream(ctx.stream)          # later torch work sees Y
    X.record_stream(ctx.stream)
    Y.record_stream(ctx.stream)
    return Y


def apply_H_free(ctx: Context, basis: Basis, inter: Interaction, X, Y=None):
    """Matrix-free Y = H X for H given by (basis, uploaded interaction);
    X, Y torch device tensors (D x nvec, row-major, nvec 8 or 16, float64 or
    float32: the dtype H is evaluated in)."""
    import torch
    if X.dtype not in (torch.float64, torch.float32) or X.dim() != 2 or X.shape[0] != basis.dim \
            or X.stride(1) != 1:
        raise ValueError("X must be a (D, nvec) float64 or float32 tensor with unit column stride")
    if Y is None:
        Y = torch.empty_like(X)
    if Y.dtype != X.dtype or Y.shape != X.shape or Y.stride(1) != 1:
        raise ValueError("Y must match X")
    cur = torch.cuda.current_stream(X.device)
    ctx.stream.wait_stream(cur)
    _check(load().cib_apply_H_free(ctx.h, basis.h, inter.h, _dtype_code(X.dtype), X.data_ptr(), X.stride(0),
                                   Y.data_ptr(), Y.stride(0), X.shape[1]))
    cur.wait_stream(ctx.stream)
    return Y


def observables(ctx: Context, basis: Basis, tables_list, X):
    """a[k, v] = x_v^T O_k x_v (numpy float64, shape (m, nvec)) for the
    operators given by tables_list and the columns of the torch device tensor
    X (D x nvec, row-major, float64 or float32: the dtype the operators are
    built and applied in)."""
    import numpy as np
    import torch
    if X.dtype not in (torch.float64, torch.float32) or X.dim() != 2 or X.shape[0] != basis.dim \
            or X.stride(1) != 1:
        raise ValueError("X must be a (D, nvec) float64 or float32 tensor with unit column stride")
    holders = [_TablesHolder(t) for t in tables_list]
    arr = (TablesC * len(holders))(*[h.c for h in holders])
    out = np.zeros((len(holders), X.shape[1]), dtype=np.float64)
    cur = torch.cuda.current_stream(X.device)
    ctx.stream.wait_stream(cur)          # X is ready on the caller's stream
    _check(load().cib_observables(ctx.h, basis.h, ctypes.cast(arr, ctypes.c_void_p), len(holders),
                                  _dtype_code(X.dtype), X.data_ptr(), X.stride(0), X.shape[1],
                                  out.ctypes.data))
    return out


def count_states(ctx: Context, mbs, n_sp: int, method: int = 0, want_counts: bool = True,
                 noalloc: bool = False):
    """State-counting test on an (n, N) array of ascending uint16 index
    tuples (numpy, copied to the device): (total, per-state counts as numpy
    int32 or None).  method 0 = hybrid, 1 = tuples only, 2 = 128-bit bit
    strings.  noalloc: call cib_count_states_noalloc (library scratch in a
    static device array, n <= 2^17) instead of cib_count_states."""
    import numpy as np
    import torch
    mbs = np.ascontiguousarray(mbs, dtype=np.uint16)
    n, N = mbs.shape
    dev = torch.device("cuda", ctx.device)
    m = torch.from_numpy(mbs.view(np.int16)).to(dev)
    c = torch.empty(n, dtype=torch.int32, device=dev) if want_counts else None
    torch.cuda.current_stream(dev).synchronize()
    total = ctypes.c_int64()
    fn = load().cib_count_states_noalloc if noalloc else load().cib_count_states
    _check(fn(ctx.h, m.data_ptr(), n, N, n_sp, method, c.data_ptr() if c is not None else None,
              ctypes.byref(total)))
    return total.value, (c.cpu().numpy() if c is not None else None)


class Precond:
    """Block-diagonal preconditioner over many-body basis orbitals
    (cib_precond_create); blocks, groups, largest block and Jacobi sweeps as
    attributes."""

    def __init__(self, ctx: Context, basis: Basis, H: Matrix, max_block: int = 16):
        self.ctx, self.dim = ctx, H.dim
        h = ctypes.c_void_p()
        _check(load().cib_precond_create(ctx.h, basis.h, H.h, int(max_block), ctypes.byref(h)))
        self.h = h
        ctx._adopt(self)
        nb, ng, lg, sw = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(load().cib_precond_info(self.h, ctypes.byref(nb), ctypes.byref(ng), ctypes.byref(lg),
                                       ctypes.byref(sw)))
        self.n_blocks, self.n_groups, self.largest, self.max_sweeps = nb.value, ng.value, lg.value, sw.value

    def blocks(self):
        """(perm int32 [D], block_off int64 [n_blocks + 1]) host arrays."""
        perm = np.zeros(self.dim, dtype=np.int32)
        off = np.zeros(self.n_blocks + 1, dtype=np.int64)
        _check(load().cib_precond_export(self.h, perm.ctypes.data, off.ctypes.data))
        return perm, off

    def apply(self, R, theta, W=None):
        """W = M(theta)^-1 R; R, W float64 device tensors (D x ncol)."""
        import torch
        if W is None:
            W = torch.empty_like(R)
        th = np.ascontiguousarray(theta, dtype=np.float64)
        self.ctx.stream.wait_stream(torch.cuda.current_stream())
        _check(load().cib_precond_apply(self.ctx.h, self.h, th.ctypes.data, R.data_ptr(), R.stride(0),
                                        W.data_ptr(), W.stride(0), int(R.shape[1])))
        return W

    def free(self):
        if self.h:
            load().cib_precond_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def lobpcg(ctx: Context, H: Matrix, nev: int, block: int = 8, max_iter: int = 500, tol: float = 0.0,
           seed: int = 0, x0=None, want_vectors: bool = False, precond: Precond = None):
    """Lowest nev eigenvalues (numpy float64), info dict, and optionally the
    eigenvectors as a (D, nev) float64 device tensor.  precond: a Precond
    made for H (block-diagonal), else the diagonal preconditioner."""
    import torch
    o = LobpcgOptsC(nev, block, max_iter, tol, seed, x0.data_ptr() if x0 is not None else None,
                    precond.h if precond is not None else None)
    ctx.stream.wait_stream(torch.cuda.current_stream())
    ev = np.zeros(nev, dtype=np.float64)
    vec = None
    if want_vectors:
        vec = torch.empty((H.dim, nev), dtype=torch.float64, device="cuda:%d" % ctx.device)
    info = LobpcgInfoC()
    rc = load().cib_lobpcg(ctx.h, H.h, ctypes.byref(o), ev.ctypes.data,
                           vec.data_ptr() if vec is not None else None, nev, ctypes.byref(info))
    _check(rc, allow=(CIB_E_NOT_CONVERGED,))
    d = dict(status=rc, iters=info.iters, n_converged=info.n_converged,
             resid=np.asarray(info.resid[:nev]), t_total_s=info.t_total_s,
             t_spmm_s=info.t_spmm_s, n_spmm=info.n_spmm)
    return ev, d, vec


def lanczos(ctx: Context, H: Matrix, nev: int, max_iter: int = 300, tol: float = 0.0, seed: int = 0,
            want_vectors: bool = False):
    """Lowest nev eigenvalues by Lanczos with full reorthogonalisation
    (numpy float64), info dict, and optionally the eigenvectors as a (D, nev)
    float64 device tensor."""
    import torch
    o = LanczosOptsC(nev, max_iter, tol, seed)
    ctx.stream.wait_stream(torch.cuda.current_stream())
    ev = np.zeros(nev, dtype=np.float64)
    vec = None
    if want_vectors:
        vec = torch.empty((H.dim, nev), dtype=torch.float64, device="cuda:%d" % ctx.device)
    info = LanczosInfoC()
    rc = load().cib_lanczos(ctx.h, H.h, ctypes.byref(o), ev.ctypes.data,
                            vec.data_ptr() if vec is not None else None, nev, ctypes.byref(info))
    _check(rc, allow=(CIB_E_NOT_CONVERGED,))
    d = dict(status=rc, iters=info.iters, n_converged=info.n_converged,
             resid=np.asarray(info.resid[:nev]), t_total_s=info.t_total_s, t_spmv_s=info.t_spmv_s)
    return ev, d, vec


def tridiag_lowest(a, b, k):
    """Host step of the Lanczos solver: lowest k eigenpairs (values, n x k
    vectors) of the symmetric tridiagonal matrix with diagonal a and
    off-diagonal b (numpy float64)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    n = len(a)
    th = np.zeros(k)
    S = np.zeros((n, k))
    _check(load().cib_tridiag_lowest(a.ctypes.data, b.ctypes.data if len(b) else None, n, k,
                                     th.ctypes.data, S.ctypes.data))
    return th, S


def serve(ctx: Context, requests: Sequence[dict], hbm_budget_bytes: int = 0, max_active: int = 0,
          realtime: bool = False, deadline_s: float = 0.0, n_streams: int = 0):
    """requests: dicts with id, arrival_s, spec, tables, dtype, nev, block,
    max_iter, tol, seed.  Returns a list of result dicts in request order."""
    n = len(requests)
    reqs = (RequestC * n)()
    holders = []
    for k, r in enumerate(requests):
        th = _TablesHolder(r["tables"])
        holders.append(th)
        reqs[k].id = int(r["id"])
        reqs[k].arrival_s = float(r.get("arrival_s", 0.0))
        reqs[k].basis = _spec_c(r["spec"])
        reqs[k].tables = ctypes.pointer(th.c)
        reqs[k].dtype = _dtype_code(r.get("dtype", "f64"))
        reqs[k].solve = LobpcgOptsC(int(r.get("nev", 4)), int(r.get("block", 8)),
                                    int(r.get("max_iter", 500)), float(r.get("tol", 0.0)),
                                    int(r.get("seed", 0)), None)
    res = (ResultC * n)()
    opts = ServeOptsC(hbm_budget_bytes, max_active, int(realtime), deadline_s, n_streams)
    _check(load().cib_serve(ctx.h, reqs, n, ctypes.byref(opts), res))
    out = []
    for k in range(n):
        r = res[k]
        nev = reqs[k].solve.nev
        out.append(dict(id=r.id, status=r.status, dim=r.dim, nnz_half=r.nnz_half, iters=r.iters,
                        evals=np.asarray(r.evals[:nev]), resid=np.asarray(r.resid[:nev]),
                        t_arrive=r.t_arrive, t_admit=r.t_admit, t_done=r.t_done))
    return out
