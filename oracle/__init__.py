"""CPU oracle for HYLU's numerical factorisation and substitution.

TEST INFRASTRUCTURE ONLY: imported by tests, by the smoke check and by the
CPU-baseline leg of the benchmark, never by the library.  The arithmetic lives
in hylu_oracle.c (plain single-threaded FP64 C); this module only marshals
arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hylu_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no BLAS, no OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.orc_create.restype = P
        lib.orc_create.argtypes = [C.c_int32, P, P, P, P, P, P, P]
        lib.orc_destroy.argtypes = [P]
        for f in ("orc_symbolic", "orc_levels"):
            getattr(lib, f).argtypes = [P]
            getattr(lib, f).restype = C.c_int
        lib.orc_set_values.argtypes = [P, P]
        lib.orc_check_matching.argtypes = [P, C.c_double]
        lib.orc_partition.argtypes = [P, C.c_int32, C.c_int32]
        lib.orc_numeric.argtypes = [P, C.c_double, C.c_int, P]
        lib.orc_pivot_tau.argtypes = [P, C.c_double]
        lib.orc_pivot_tau.restype = C.c_double
        lib.orc_solve.argtypes = [P, P, P]
        lib.orc_solve_transposed.argtypes = [P, P, P]
        lib.orc_residual.argtypes = [P, P, P, P]
        lib.orc_residual.restype = None
        lib.orc_backward_error.argtypes = [P, P, P, P, P]
        lib.orc_backward_error.restype = None
        lib.orc_solve_ir.argtypes = [P, P, P, C.c_double, C.c_int, P]
        lib.orc_gradient_values.argtypes = [P, P, P, P]
        lib.orc_gradient_values.restype = None
        lib.orc_sizes.argtypes = [P, P]
        lib.orc_sizes.restype = None
        lib.orc_copy_b.argtypes = [P, P, P, P]
        lib.orc_copy_symbolic.argtypes = [P, P, P, P, P]
        lib.orc_copy_partition.argtypes = [P, P, P]
        lib.orc_copy_levels.argtypes = [P, P]
        lib.orc_copy_factors.argtypes = [P] + [P] * 7
        for f in ("orc_copy_b", "orc_copy_symbolic", "orc_copy_partition", "orc_copy_levels",
                  "orc_copy_factors"):
            getattr(lib, f).restype = None
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


class OracleError(RuntimeError):
    pass


def _chk(rc, what):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


class Oracle:
    """One matrix A with its (given) permutations and scalings.

    perm_r[i'] / perm_c[j'] map B's rows / columns to A's; dr / dc are indexed
    by A's rows / columns; B(i',j') = dr[pr[i']] A(pr[i'], pc[j']) dc[pc[j']].
    """

    def __init__(self, n, row_ptr, col, val, perm_r=None, perm_c=None, dr=None, dc=None):
        lib = _load()
        self.n = int(n)
        self._keep = [_c(row_ptr, np.int64), _c(col, np.int32), _c(val, np.float64),
                      _c(perm_r, np.int32), _c(perm_c, np.int32), _c(dr, np.float64),
                      _c(dc, np.float64)]
        self.h = lib.orc_create(self.n, *[_p(a) for a in self._keep])
        if not self.h:
            raise OracleError("orc_create failed")
        self.lib = lib
        self.nnz = int(self._keep[0][-1])

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.orc_destroy(h)
            self.h = None

    # -- phases -----------------------------------------------------------
    def set_values(self, val):
        v = _c(val, np.float64)
        _chk(self.lib.orc_set_values(self.h, _p(v)), "set_values")

    def check_matching(self, tol=64 * np.finfo(float).eps):
        return self.lib.orc_check_matching(self.h, tol) == 0

    def symbolic(self):
        _chk(self.lib.orc_symbolic(self.h), "symbolic")
        return self

    def partition(self, sn_min=2, sn_max=1 << 30):
        _chk(self.lib.orc_partition(self.h, sn_min, sn_max), "partition")
        return self

    def levels(self):
        _chk(self.lib.orc_levels(self.h), "levels")
        return self

    def analyse(self, sn_min=2, sn_max=1 << 30):
        return self.symbolic().partition(sn_min, sn_max).levels()

    def pivot_tau(self, rel=float(np.sqrt(np.finfo(np.float64).eps))):
        """Perturbation threshold rel * max|B| from the oracle's own B (the
        values it holds now: take it before set_values for a refactorisation)."""
        return float(self.lib.orc_pivot_tau(self.h, float(rel)))

    def numeric(self, tau, piv=None):
        pv = _c(piv, np.int32)
        _chk(self.lib.orc_numeric(self.h, float(tau), 0 if piv is not None else 1, _p(pv)), "numeric")
        return self

    def solve(self, b):
        b = _c(b, np.float64)
        x = np.empty(self.n)
        _chk(self.lib.orc_solve(self.h, _p(b), _p(x)), "solve")
        return x

    def solve_transposed(self, g):
        g = _c(g, np.float64)
        lam = np.empty(self.n)
        _chk(self.lib.orc_solve_transposed(self.h, _p(g), _p(lam)), "solve_transposed")
        return lam

    def solve_ir(self, b, tol=1e-12, maxit=10):
        b = _c(b, np.float64)
        x = np.empty(self.n)
        eta = np.zeros(1)
        it = self.lib.orc_solve_ir(self.h, _p(b), _p(x), float(tol), int(maxit), _p(eta))
        if it < 0:
            raise OracleError(f"solve_ir failed with code {it}")
        return x, int(it), float(eta[0])

    def residual(self, b, x):
        b = _c(b, np.float64); x = _c(x, np.float64)
        r = np.empty(self.n)
        self.lib.orc_residual(self.h, _p(b), _p(x), _p(r))
        return r

    def backward_error(self, b, x):
        """(eta_inf, ||Ax-b||_1/||b||_1) with compensated sums."""
        b = _c(b, np.float64); x = _c(x, np.float64)
        e = np.zeros(1); r1 = np.zeros(1)
        self.lib.orc_backward_error(self.h, _p(b), _p(x), _p(e), _p(r1))
        return float(e[0]), float(r1[0])

    def gradient_values(self, lam, x):
        lam = _c(lam, np.float64); x = _c(x, np.float64)
        g = np.empty(self.nnz)
        self.lib.orc_gradient_values(self.h, _p(lam), _p(x), _p(g))
        return g

    # -- results ----------------------------------------------------------
    def sizes(self):
        s = np.zeros(12, dtype=np.int64)
        self.lib.orc_sizes(self.h, _p(s))
        keys = ["n", "nnz_a", "nnz_l", "nnz_u", "flops", "flops_padded", "nnodes",
                "n_supernodes", "rows_in_supernodes", "nnz_l_padded", "n_perturbed", "factored"]
        return {k: int(v) for k, v in zip(keys, s)}

    def B(self):
        rp = np.empty(self.n + 1, np.int64)
        ci = np.empty(self.nnz, np.int32)
        v = np.empty(self.nnz)
        self.lib.orc_copy_b(self.h, _p(rp), _p(ci), _p(v))
        return rp, ci, v

    def symbolic_structure(self):
        s = self.sizes()
        Lp = np.empty(self.n + 1, np.int64); Li = np.empty(s["nnz_l"], np.int32)
        Up = np.empty(self.n + 1, np.int64); Ui = np.empty(s["nnz_u"], np.int32)
        self.lib.orc_copy_symbolic(self.h, _p(Lp), _p(Li), _p(Up), _p(Ui))
        return Lp, Li, Up, Ui

    def partition_arrays(self):
        nn = self.sizes()["nnodes"]
        ptr = np.empty(nn + 1, np.int32); sn = np.empty(nn, np.int32)
        self.lib.orc_copy_partition(self.h, _p(ptr), _p(sn))
        return ptr, sn

    def level_arrays(self):
        nn = self.sizes()["nnodes"]
        lev = np.empty(4 * nn, np.int32)
        self.lib.orc_copy_levels(self.h, _p(lev))
        return lev.reshape(4, nn)

    def factors(self):
        """(Fp, Fi, Fv, Sp, Si, Sv, piv): padded L by rows, U_st by rows, pivots."""
        s = self.sizes()
        n = self.n
        Fp = np.empty(n + 1, np.int64); Fi = np.empty(s["nnz_l_padded"], np.int32)
        Fv = np.empty(s["nnz_l_padded"])
        Sp = np.empty(n + 1, np.int64); Si = np.empty(s["nnz_u"], np.int32)
        Sv = np.empty(s["nnz_u"]); piv = np.empty(n, np.int32)
        self.lib.orc_copy_factors(self.h, _p(Fp), _p(Fi), _p(Fv), _p(Sp), _p(Si), _p(Sv), _p(piv))
        return Fp, Fi, Fv, Sp, Si, Sv, piv
