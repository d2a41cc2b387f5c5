"""Comparison helpers shared by the GPU parity tests (not a test module)."""
import numpy as np

import oracle


def oracle_for(h, A, sn_min=2, sn_max=1 << 30):
    """The oracle on A (the analysed values) with the permutations and
    scalings the library chose.  o.tau is the perturbation threshold the
    oracle computes from its own B; it must equal the library's."""
    sym = h.symbolic()
    o = oracle.Oracle(A.n, A.row_ptr, A.col, A.val, sym["perm_r"], sym["perm_c"], sym["dr"], sym["dc"])
    o.analyse(sn_min, sn_max)
    o.tau = checked_tau(h, o)
    return o, sym


def checked_tau(h, o):
    """tau = sqrt(eps) max|B| of the oracle's B (the analysed values), checked
    against the threshold the library reports."""
    tau = o.pivot_tau()
    assert tau == h.info()["pivot_tau"], (tau, h.info()["pivot_tau"])
    return tau


def _match(gkey, gval, okey, oval):
    order = np.argsort(gkey, kind="stable")
    gk, gv = gkey[order], gval[order]
    idx = np.searchsorted(gk, okey)
    assert np.all(idx < gk.size) and np.array_equal(gk[np.minimum(idx, gk.size - 1)], okey), \
        "an oracle entry is missing from the device factors"
    extra = np.ones(gk.size, bool)
    extra[idx] = False
    return gv[idx], gv[extra]


def compare_factors(h, o, tol=1e-11, exact=False):
    """Element-by-element comparison of L, U_st and the pivots.

    tol="derived": a bound for two different summation orders of the entries
    of L and U_st, relative to the largest entry.  An entry is a sum of at most
    k products of factor entries (k = the widest row of the factors), each at
    most max|L| max|U|; the sum's rounding error is at most k u times the sum
    of the magnitudes (u the unit roundoff), so the two orders differ by at
    most 2 k^2 u max|L| max|U| (floor 1e-11).  Errors carried in from
    earlier rows make this a working bound, not a proof; the residual check
    (compare_backward_stability) complements it."""
    from paper_2509_07690_amd import hylu
    (Lr, Lk, Lv), (Ur, Uc, Uv), piv = hylu.factors_as_rows(h)
    Fp, Fi, Fv, Sp, Si, Sv, opiv = o.factors()
    n = h.n
    assert np.array_equal(piv, opiv), "pivot order differs"
    okey = np.repeat(np.arange(n, dtype=np.int64), np.diff(Fp)) * n + Fi
    gl, gl_extra = _match(Lr * n + Lk, Lv, okey, Fv)
    okey = np.repeat(np.arange(n, dtype=np.int64), np.diff(Sp)) * n + Si
    gu, gu_extra = _match(Ur * n + Uc, Uv, okey, Sv)
    # padding the oracle does not store must hold exact zeros
    assert np.all(gl_extra == 0) and np.all(gu_extra == 0), "nonzero padding"
    if exact:
        assert np.array_equal(gl, Fv) and np.array_equal(gu, Sv)
        return 0.0
    gL = np.abs(Fv).max() if Fv.size else 0.0
    gU = np.abs(Sv).max()
    scale = max(1.0, gU, gL)
    if tol == "derived":
        k = int(max(np.diff(Fp).max() if Fv.size else 0, np.diff(Sp).max()))
        tol = max(1e-11, 2.0 * k * k * np.finfo(np.float64).eps / 2 * max(gL, 1.0) * max(gU, 1.0) / scale)
    err = max(np.abs(gl - Fv).max() if Fv.size else 0.0, np.abs(gu - Sv).max()) / scale
    assert err <= tol, f"factor difference {err:.3e} > {tol:.1e} (max|L| {gL:.3e}, max|U| {gU:.3e})"
    return err


def _residual_ratio(n, B, L, U):
    """||B - (I + L) U_st||_max / ||(I + |L|) |U_st|||_max for row-indexed
    factors: L = (row, source row, value), U = (row, column, value)."""
    import scipy.sparse as sp
    Lm = sp.csr_matrix((L[2], (L[0], L[1])), shape=(n, n))
    Um = sp.csr_matrix((U[2], (U[0], U[1])), shape=(n, n))
    R = B - Um - Lm @ Um
    D = abs(Um) + abs(Lm) @ abs(Um)
    return abs(R).max() / D.max()


def compare_backward_stability(h, o):
    """The device factors reproduce B (B Pi = L U, stored as B = L U_st) as
    closely as the oracle's own factors do: the normwise residual ratio of the
    device factors is at most 10 times the oracle's (with a floor of 4 u).
    Used where the blocked kernels sum in a different order than the
    up-looking oracle and growth in L and U amplifies the rounding
    differences between the two."""
    import scipy.sparse as sp
    from paper_2509_07690_amd import hylu
    n = h.n
    rp, ci, bv = o.B()
    B = sp.csr_matrix((bv, ci, rp), shape=(n, n))
    (Lr, Lk, Lv), (Ur, Uc, Uv), _ = hylu.factors_as_rows(h)
    g = _residual_ratio(n, B, (Lr, Lk, Lv), (Ur, Uc, Uv))
    Fp, Fi, Fv, Sp, Si, Sv, _ = o.factors()
    rows = lambda p: np.repeat(np.arange(n), np.diff(p))
    r = _residual_ratio(n, B, (rows(Fp), Fi, Fv), (rows(Sp), Si, Sv))
    assert g <= max(10.0 * r, 4 * np.finfo(np.float64).eps), (g, r)
    return g, r


def rel_diff(x, xo):
    return float(np.abs(x - xo).max() / max(np.abs(xo).max(), 1e-300))
