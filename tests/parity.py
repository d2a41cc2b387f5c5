"""Comparison helpers shared by the GPU parity tests (not a test module)."""
import numpy as np

import oracle


def oracle_for(h, A, sn_min=2, sn_max=1 << 30):
    """The oracle on A with the permutations and scalings the library chose."""
    sym = h.symbolic()
    o = oracle.Oracle(A.n, A.row_ptr, A.col, A.val, sym["perm_r"], sym["perm_c"], sym["dr"], sym["dc"])
    o.analyse(sn_min, sn_max)
    return o, sym


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
    """Element-by-element comparison of L, U_st and the pivots."""
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
    scale = max(1.0, np.abs(Sv).max(), np.abs(Fv).max() if Fv.size else 0.0)
    err = max(np.abs(gl - Fv).max() if Fv.size else 0.0, np.abs(gu - Sv).max()) / scale
    assert err <= tol, f"factor difference {err:.3e} > {tol:.1e}"
    return err


def rel_diff(x, xo):
    return float(np.abs(x - xo).max() / max(np.abs(xo).max(), 1e-300))
