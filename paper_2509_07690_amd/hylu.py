"""Python binding of libhylu.so (HYLU numerical factorisation on MI355X).

Argument marshalling only: every step of the factorisation and substitution
runs in the library's gfx950 kernels.  PyTorch supplies device memory and the
current stream.  If the library was not built, importing this module raises.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import warnings
import weakref

import numpy as np
# PyTorch ships its own HIP runtime (file libamdhip64.so, soname
# libamdhip64.so.7).  It has to be loaded before libhylu.so: the loader then
# binds libhylu.so to that same runtime.  In the other order the process ends
# up with two HIP runtimes, and device pointers of one are unknown to the other.
import torch  # noqa: F401,E402

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhylu.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2509_07690_amd.build_lib` "
                      "or __graft_entry__.build() (there is no CPU fallback)")

_lib = C.CDLL(LIB_PATH)

OK = 0
WARN_IR_NOT_CONVERGED = 1


class Options(C.Structure):
    _fields_ = [("ordering", C.c_int32), ("user_perm", C.c_void_p), ("static_pivot", C.c_int32),
                ("precision", C.c_int32), ("pivot_tau", C.c_double), ("ir_tol", C.c_double),
                ("ir_maxit", C.c_int32), ("sn_min", C.c_int32), ("sn_max", C.c_int32),
                ("kernel_mode", C.c_int32), ("repeated", C.c_int32), ("nd_leaf", C.c_int32),
                ("amd_dense", C.c_double), ("dense_tail", C.c_double), ("tail_min", C.c_int32),
                ("tail_max", C.c_int32), ("sn_dense", C.c_int32),
                ("sn_tile", C.c_int32), ("sn_inverse", C.c_int32), ("tail_sparse", C.c_int32), ("side_rows", C.c_int32),
                ("pipeline_rows", C.c_int32), ("group_min_rows", C.c_int32), ("group_tail_rows", C.c_int32),
                ("solve_chain", C.c_int32), ("gpu_symbolic", C.c_int32), ("pipeline_spin", C.c_int32),
                ("solve_split", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("nnz_a", C.c_int64), ("nnz_l", C.c_int64), ("nnz_u", C.c_int64),
                ("flops", C.c_uint64), ("flops_padded", C.c_uint64), ("factor_entries", C.c_int64),
                ("n_nodes", C.c_int32), ("n_supernodes", C.c_int32), ("rows_in_supernodes", C.c_int32),
                ("max_supernode", C.c_int32), ("n_levels", C.c_int32 * 4), ("n_perturbed", C.c_int32),
                ("ir_iters", C.c_int32), ("berr", C.c_double), ("pivot_tau", C.c_double),
                ("tail_rows", C.c_int32), ("tail_panels", C.c_int32), ("flops_issued", C.c_uint64),
                ("resid_1", C.c_double), ("n_dense_sn", C.c_int32), ("sn_groups", C.c_int32),
                ("tail_groups", C.c_int32), ("pipe_tasks", C.c_int32),
                ("chain_levels", C.c_int32), ("sym_ms", C.c_double), ("sym_kernel_ms", C.c_double),
                ("sym_hash", C.c_uint64), ("split_sn", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["n_levels"] = list(self.n_levels)
        return d


class KernelStats(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int32), ("ms", C.c_double), ("bytes", C.c_double),
                ("flops", C.c_double)]


class SymbolicView(C.Structure):
    _fields_ = [("perm_r", C.c_void_p), ("perm_c", C.c_void_p), ("dr", C.c_void_p), ("dc", C.c_void_p),
                ("node_ptr", C.c_void_p), ("is_sn", C.c_void_p), ("levels", C.c_void_p)]


_P = C.c_void_p
_sigs = {
    "hylu_default_options": [_P],
    "hylu_status_string": [C.c_int],
    "hylu_create": [_P, _P],
    "hylu_destroy": [_P],
    "hylu_analyze": [_P, C.c_int32, _P, _P, _P, _P],
    "hylu_factorize": [_P, _P, _P],
    "hylu_refactor": [_P, _P, _P],
    "hylu_solve": [_P, _P, _P, C.c_int32, C.c_int64, C.c_int32, _P],
    "hylu_solve_noalloc": [_P, _P, _P, C.c_int32, C.c_int64, C.c_int32, _P],
    "hylu_grad_values": [_P, _P, _P, C.c_int32, C.c_int64, _P, _P],
    "hylu_residual": [_P, _P, _P, C.c_int32, C.c_int64, C.c_int32, _P, _P, _P],
    "hylu_get_info": [_P, _P],
    "hylu_export_symbolic": [_P, _P],
    "hylu_export_factors": [_P, _P, _P, _P, _P, _P, _P, _P],
    "hylu_export_sizes": [_P, _P],
    "hylu_profile": [_P, _P, _P, _P, _P, _P, C.c_int32, _P],
}
for _name, _args in _sigs.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
_lib.hylu_status_string.restype = C.c_char_p

EXPORTED = tuple(_sigs)


# Device memory of every handle comes from PyTorch's caching allocator
# (hylu_allocator callbacks), so the library and torch share one pool.
_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class Allocator(C.Structure):
    _fields_ = [("ctx", C.c_void_p), ("alloc", _ALLOC_FN), ("free", _FREE_FN)]


def _torch_alloc(ctx, nbytes, stream):
    try:
        dev = torch.cuda.current_device()
        st = stream if stream else torch.cuda.current_stream(dev).cuda_stream
        return torch.cuda.caching_allocator_alloc(int(nbytes), dev, st)
    except Exception:         # the library reports HYLU_ERR_OOM
        return None


def _torch_free(ctx, ptr, stream):
    if ptr:
        torch.cuda.caching_allocator_delete(ptr)


_ALLOCATOR = Allocator(None, _ALLOC_FN(_torch_alloc), _FREE_FN(_torch_free))

# handles still open at exit are destroyed while torch's allocator is alive
_LIVE = weakref.WeakSet()


@atexit.register
def _close_all():
    for hd in list(_LIVE):
        hd.close()


class HyluError(RuntimeError):
    def __init__(self, code, what):
        msg = _lib.hylu_status_string(code).decode()
        super().__init__(f"{what}: {msg} ({code})")
        self.code = code


class RefinementWarning(RuntimeWarning):
    """Iterative refinement stopped above its backward-error target."""


def _chk(rc, what, allow_warn=False):
    if rc == OK:
        return rc
    if allow_warn and rc == WARN_IR_NOT_CONVERGED:
        warnings.warn(f"{what}: {_lib.hylu_status_string(rc).decode()}", RefinementWarning, stacklevel=3)
        return rc
    raise HyluError(rc, what)


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _ptr(a):
    return C.c_void_p(a.ctypes.data)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError(f"expected a contiguous {dtype} CUDA tensor")
    return C.c_void_p(t.data_ptr())


ORDERINGS = {"amd": 0, "nd": 1, "natural": 2, "user": 3, "nd_ml": 4}


def default_options(**kw) -> Options:
    o = Options()
    _chk(_lib.hylu_default_options(C.byref(o)), "default_options")
    for k, v in kw.items():
        if k == "ordering" and isinstance(v, str):
            v = ORDERINGS[v]
        if k == "precision" and isinstance(v, str):
            v = {"fp64": 0, "fp32": 1}[v]
        setattr(o, k, v)
    return o


class Handle:
    """One sparsity pattern: analyze once, factorize / refactor / solve many times.

    row_ptr, col, val are host arrays (CSR, 0-based, sorted unique columns).
    Keyword options follow hylu_options (ordering="amd"|"nd"|"nd_ml"|"natural"|"user",
    precision="fp64"|"fp32", static_pivot, sn_min, sn_max, kernel_mode, ...).
    """

    def __init__(self, row_ptr, col, val, user_perm=None, **opts):
        self.h = C.c_void_p()
        self.fact_id = 0          # bumped by every (re)factorisation
        self.last_status = OK
        _chk(_lib.hylu_create(C.byref(self.h), C.byref(_ALLOCATOR)), "create")
        _LIVE.add(self)
        rp = _np(row_ptr, np.int64)
        ci = _np(col, np.int32)
        va = _np(val, np.float64)
        self.n = rp.size - 1
        self.nnz = int(rp[-1])
        self._perm = None
        if user_perm is not None:
            self._perm = _np(user_perm, np.int32)
            opts["ordering"] = 3
            opts["user_perm"] = self._perm.ctypes.data
        self.opts = default_options(**opts)
        _chk(_lib.hylu_analyze(self.h, self.n, _ptr(rp), _ptr(ci), _ptr(va), C.byref(self.opts)), "analyze")
        self.row_ptr, self.col = rp, ci

    @classmethod
    def batch(cls, members, **opts):
        """One handle for a batch of matrices of uneven sizes (block diagonal;
        see hylu_analyze_batch).  members: sequence of (row_ptr, col, val)
        host CSR triples.  Values and right-hand sides are passed back to back
        in member order; `offsets()` gives the row and value ranges."""
        self = cls.__new__(cls)
        self.h = C.c_void_p()
        self.fact_id = 0
        self.last_status = OK
        self._perm = None
        _chk(_lib.hylu_create(C.byref(self.h), C.byref(_ALLOCATOR)), "create")
        _LIVE.add(self)
        mats = [(_np(rp, np.int64), _np(ci, np.int32), _np(va, np.float64)) for rp, ci, va in members]
        k = len(mats)
        ns = (C.c_int32 * k)(*[m[0].size - 1 for m in mats])
        rps = (C.c_void_p * k)(*[m[0].ctypes.data for m in mats])
        cis = (C.c_void_p * k)(*[m[1].ctypes.data for m in mats])
        vas = (C.c_void_p * k)(*[m[2].ctypes.data for m in mats])
        self.opts = default_options(**opts)
        _chk(_lib.hylu_analyze_batch(self.h, k, ns, rps, cis, vas, C.byref(self.opts)), "analyze_batch")
        roff, qoff = self.offsets()
        self.n, self.nnz = int(roff[-1]), int(qoff[-1])
        self.row_ptr = np.concatenate([[0]] + [m[0][1:] + q for m, q in zip(mats, qoff[:-1])]).astype(np.int64)
        self.col = np.concatenate([m[1] + r for m, r in zip(mats, roff[:-1])]).astype(np.int32)
        return self

    def offsets(self):
        """(row_off, nnz_off): member k owns rows row_off[k]:row_off[k+1] and
        values nnz_off[k]:nnz_off[k+1]."""
        cnt = C.c_int32()
        _chk(_lib.hylu_batch_offsets(self.h, C.byref(cnt), None, None), "batch_offsets")
        ro = np.empty(cnt.value + 1, np.int64)
        qo = np.empty(cnt.value + 1, np.int64)
        _chk(_lib.hylu_batch_offsets(self.h, C.byref(cnt), _ptr(ro), _ptr(qo)), "batch_offsets")
        return ro, qo

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            _lib.hylu_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- numerical phases (device tensors) --------------------------------
    def factorize(self, values, stream=None):
        import torch
        _chk(_lib.hylu_factorize(self.h, _dev_ptr(values, torch.float64), _stream(stream)), "factorize")
        self.fact_id += 1

    def refactor(self, values, stream=None):
        import torch
        _chk(_lib.hylu_refactor(self.h, _dev_ptr(values, torch.float64), _stream(stream)), "refactor")
        self.fact_id += 1

    def solve(self, b, out=None, transpose=False, stream=None):
        """b: (n,) or (n, k) float64 CUDA tensor (column-major for k > 1 means
        b.t().contiguous() layout; pass a tensor of shape (k, n) via solve_cols)."""
        import torch
        if b.dim() == 1:
            x = torch.empty_like(b) if out is None else out
            rc = _lib.hylu_solve(self.h, _dev_ptr(b, torch.float64), _dev_ptr(x, torch.float64), 1, self.n,
                                 1 if transpose else 0, _stream(stream))
            self.last_status = _chk(rc, "solve", allow_warn=True)
            return x
        return self.solve_cols(b.t().contiguous(), transpose=transpose, stream=stream).t()

    def solve_cols(self, bt, out=None, transpose=False, stream=None):
        """bt: (k, n) float64 CUDA tensor, i.e. k right-hand sides stored
        column-major as the C ABI expects; returns (k, n)."""
        import torch
        k, n = bt.shape
        assert n == self.n
        x = torch.empty_like(bt) if out is None else out
        rc = _lib.hylu_solve(self.h, _dev_ptr(bt, torch.float64), _dev_ptr(x, torch.float64), k, n,
                             1 if transpose else 0, _stream(stream))
        self.last_status = _chk(rc, "solve", allow_warn=True)
        return x

    def solve_noalloc(self, bt, out, transpose=False, stream=None):
        """hylu_solve_noalloc: bt, out (n,) or (k, n) float64 CUDA tensors
        (rows of a (k, n) tensor are right-hand sides); the library
        allocates nothing (work vectors in its fixed per-GPU scratch)."""
        import torch
        k = 1 if bt.dim() == 1 else bt.shape[0]
        rc = _lib.hylu_solve_noalloc(self.h, _dev_ptr(bt, torch.float64), _dev_ptr(out, torch.float64), k, self.n,
                                     1 if transpose else 0, _stream(stream))
        self.last_status = _chk(rc, "solve_noalloc", allow_warn=True)
        return out

    def residual(self, b, x, transpose=False, stream=None):
        """(backward error, ||Ax-b||_1/||b||_1) of x for b, each the largest
        over the columns: b, x (n,) or (k, n) float64 CUDA tensors (rows of a
        (k, n) tensor are right-hand sides).  Synchronises the stream."""
        import torch
        k = 1 if b.dim() == 1 else b.shape[0]
        eta, r1 = C.c_double(), C.c_double()
        _chk(_lib.hylu_residual(self.h, _dev_ptr(b, torch.float64), _dev_ptr(x, torch.float64), k, self.n,
                                1 if transpose else 0, _stream(stream), C.byref(eta), C.byref(r1)), "residual")
        return eta.value, r1.value

    def autotune(self, values, reps=2, stream=None):
        """Pick per-level thread counts by timing (hylu_autotune); returns the
        summed level times (ms) with the built-in and with the chosen shapes."""
        import torch
        before, after = C.c_double(), C.c_double()
        _chk(_lib.hylu_autotune(self.h, _dev_ptr(values, torch.float64), _stream(stream), int(reps),
                                C.byref(before), C.byref(after)), "autotune")
        self.fact_id += 1
        return before.value, after.value

    def grad_values(self, lam, x, out=None, stream=None):
        """dL/dval[p] = -sum_k lam[row p, k] x[col p, k]: lam, x are (n,) or
        (k, n) float64 CUDA tensors (rows of a (k, n) tensor are columns)."""
        import torch
        k = 1 if lam.dim() == 1 else lam.shape[0]
        g = torch.empty(self.nnz, dtype=torch.float64, device=lam.device) if out is None else out
        _chk(_lib.hylu_grad_values(self.h, _dev_ptr(lam, torch.float64), _dev_ptr(x, torch.float64), k, self.n,
                                   _dev_ptr(g, torch.float64), _stream(stream)), "grad_values")
        return g

    def profile(self, values, b, x, stream=None):
        """Per-kernel-class device time (HIP events around every launch of one
        eager refactorisation + solve) with algorithmic bytes and flops."""
        import torch
        arr = (KernelStats * 16)()
        cnt = C.c_int32()
        _chk(_lib.hylu_profile(self.h, _dev_ptr(values, torch.float64), _dev_ptr(b, torch.float64),
                               _dev_ptr(x, torch.float64), _stream(stream), arr, 16, C.byref(cnt)), "profile")
        return [{"name": arr[i].name.decode(), "launches": arr[i].launches, "ms": arr[i].ms,
                 "bytes": arr[i].bytes, "flops": arr[i].flops} for i in range(cnt.value)]

    # ---- inspection -------------------------------------------------------
    def info(self) -> dict:
        inf = Info()
        _chk(_lib.hylu_get_info(self.h, C.byref(inf)), "get_info")
        return inf.as_dict()

    def symbolic(self) -> dict:
        inf = self.info()
        n, nn = self.n, inf["n_nodes"]
        out = {"perm_r": np.empty(n, np.int32), "perm_c": np.empty(n, np.int32), "dr": np.empty(n),
               "dc": np.empty(n), "node_ptr": np.empty(nn + 1, np.int32), "is_sn": np.empty(nn, np.uint8),
               "levels": np.empty(4 * nn, np.int32)}
        v = SymbolicView(*[C.c_void_p(out[k].ctypes.data) for k in
                           ("perm_r", "perm_c", "dr", "dc", "node_ptr", "is_sn", "levels")])
        _chk(_lib.hylu_export_symbolic(self.h, C.byref(v)), "export_symbolic")
        out["levels"] = out["levels"].reshape(4, nn)
        return out

    def factors_raw(self) -> dict:
        inf = self.info()
        nn = inf["n_nodes"]
        nc = C.c_int64()
        _chk(_lib.hylu_export_sizes(self.h, C.byref(nc)), "export_sizes")
        out = {"vals": np.empty(inf["factor_entries"]), "voff": np.empty(nn + 1, np.int64),
               "lw": np.empty(nn, np.int32), "W": np.empty(nn, np.int32), "coff": np.empty(nn + 1, np.int64),
               "cols": np.empty(nc.value, np.int32), "piv": np.empty(self.n, np.int32)}
        _chk(_lib.hylu_export_factors(self.h, *[C.c_void_p(out[k].ctypes.data) for k in
                                                 ("vals", "voff", "lw", "W", "coff", "cols", "piv")]),
             "export_factors")
        return out


class SparseSolve(torch.autograd.Function):
    """x = A(val)^{-1} b on the handle's pattern, with a hand-written adjoint.

    forward: (re)factorise with `val` (the first call factorises with pivot
    search, later ones reuse that pivot order) and solve.
    backward: lambda = A^{-T} dL/dx by the transposed solve on the same
    factors; dL/db = lambda and dL/dval[p] = -lambda[row p] * x[col p], the
    gradient of x = A^{-1} b restricted to the stored pattern.  If the handle
    was refactorised with other values in between, it is refactorised with
    this call's values first.  b is (n,) or (n, k); val is (nnz,).
    """

    @staticmethod
    def forward(ctx, val, b, handle):
        val = val.detach().contiguous()
        if handle.fact_id == 0:
            handle.factorize(val)
        else:
            handle.refactor(val)
        x = handle.solve(b.detach().contiguous())
        ctx.handle = handle
        ctx.fact_id = handle.fact_id
        ctx.save_for_backward(val, x)
        return x

    @staticmethod
    def backward(ctx, gx):
        val, x = ctx.saved_tensors
        h = ctx.handle
        if h.fact_id != ctx.fact_id:
            h.refactor(val)
        lam = h.solve(gx.contiguous(), transpose=True)
        gval = gb = None
        if ctx.needs_input_grad[0]:
            if x.dim() == 1:
                gval = h.grad_values(lam, x)
            else:                 # (n, k): the library sums over the k columns
                gval = h.grad_values(lam.t().contiguous(), x.t().contiguous())
        if ctx.needs_input_grad[1]:
            gb = lam
        return gval, gb, None


def sparse_solve(handle: Handle, val, b):
    """Differentiable x = A(val)^{-1} b (see SparseSolve)."""
    return SparseSolve.apply(val, b, handle)


def factors_as_rows(h: Handle):
    """Panel export converted to the oracle's row conventions.

    Returns (L, U, piv) where L = (Lrow, Lkey, Lval) lists every stored
    multiplier with its row i and source row k (padding included), U = (Urow,
    Ucol, Uval) every stored entry of U_st (B = L * U_st) with its row and
    column, and piv[i] is the column of row i's pivot.
    """
    raw = h.factors_raw()
    sym = h.symbolic()
    ptr = sym["node_ptr"].astype(np.int64)
    piv = raw["piv"].astype(np.int64)
    n = h.n
    qinv = np.empty(n, np.int64)
    qinv[piv] = np.arange(n)
    m = np.diff(ptr)
    lw = raw["lw"].astype(np.int64)
    W = raw["W"].astype(np.int64)
    nn = m.size
    # per stored value: node, row within node, position within row
    sizes = m * W
    node_of_val = np.repeat(np.arange(nn), sizes)
    off = raw["voff"][:-1].astype(np.int64)
    local = np.arange(raw["vals"].size, dtype=np.int64) - off[node_of_val]
    Wv = W[node_of_val]
    a = local // Wv
    t = local % Wv
    row = ptr[node_of_val] + a
    col = raw["cols"][raw["coff"][:-1][node_of_val] + t].astype(np.int64)
    lwv = lw[node_of_val]
    mv = m[node_of_val]
    in_L = t < lwv
    in_B = (t >= lwv) & (t < lwv + mv)
    # a block column belongs to L for row i if an earlier row of the node pivoted on it
    pivot_row = qinv[col]                     # row whose pivot is this column (block columns)
    block_L = in_B & (pivot_row < row)
    is_L = in_L | block_L
    Lrow, Lkey, Lval = row[is_L], qinv[col[is_L]], raw["vals"][is_L]
    Urow, Ucol, Uval = row[~is_L], col[~is_L], raw["vals"][~is_L]
    return (Lrow, Lkey, Lval), (Urow, Ucol, Uval), piv
