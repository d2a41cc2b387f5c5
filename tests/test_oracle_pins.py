"""Pins of the CPU oracle against things other than itself.

Every check here compares the oracle with an independent computation that the
mathematics or a textbook routine fixes: dense boolean elimination, LAPACK
getrf (scipy), numpy's dense solvers, closed forms, exact integer factors,
finite differences.  A dropped term, a wrong index or a transposed operand in
the oracle fails at least one of them.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_2509_07690_amd import synth

TAU64 = np.sqrt(np.finfo(np.float64).eps)


# ---------------------------------------------------------------------------
# helpers written independently of the oracle
# ---------------------------------------------------------------------------

def fill_bool(mask):
    """Right-looking dense boolean elimination (no pivoting)."""
    M = np.array(mask, dtype=bool)
    n = M.shape[0]
    np.fill_diagonal(M, True)
    for k in range(n):
        rows = np.nonzero(M[k + 1:, k])[0] + k + 1
        if rows.size:
            M[np.ix_(rows, np.arange(k + 1, n))] |= M[k, k + 1:]
    return M


def lu_nopivot(D):
    """Dense right-looking Gaussian elimination without pivoting."""
    A = np.array(D, dtype=np.float64)
    n = A.shape[0]
    for k in range(n - 1):
        A[k + 1:, k] /= A[k, k]
        A[k + 1:, k + 1:] -= np.outer(A[k + 1:, k], A[k, k + 1:])
    L = np.tril(A, -1) + np.eye(n)
    U = np.triu(A)
    return L, U


def random_mask(n, density, seed, band=None):
    rng = np.random.default_rng(seed)
    M = rng.random((n, n)) < density
    if band is not None:
        i, j = np.indices((n, n))
        M &= np.abs(i - j) <= band
    np.fill_diagonal(M, True)
    return M


def csr_of_mask(M, vals=None):
    r, c = np.nonzero(M)
    v = np.ones(r.size) if vals is None else vals[r, c]
    return synth.csr_from_coo(M.shape[0], r, c, v)


def oracle_of(A, **kw):
    return oracle.Oracle(A.n, A.row_ptr, A.col, A.val, **kw)


def structure_to_mask(n, p, idx):
    M = np.zeros((n, n), bool)
    r = np.repeat(np.arange(n), np.diff(p))
    M[r, idx] = True
    return M


def partition_from_mask(M, sn_min=2, sn_max=1 << 30):
    """Maximal runs of rows whose U structure differs only by the leading row."""
    n = M.shape[0]
    U = [set(np.nonzero(M[i, i:])[0] + i) for i in range(n)]
    runs, r = [], 0
    while r < n:
        e = r + 1
        while e < n and U[e - 1] - {e - 1} == U[e]:
            e += 1
        runs.append((r, e))
        r = e
    ptr, sn = [0], []
    for (a, e) in runs:
        s = a
        while s < e:
            c = min(e - s, sn_max)
            if c >= sn_min:
                ptr.append(s + c); sn.append(1)
            else:
                for t in range(s, s + c):
                    ptr.append(t + 1); sn.append(0)
            s += c
    return np.array(ptr), np.array(sn)


def levels_relaxation(nnodes, edges):
    """Longest-path depth by Bellman-Ford style relaxation to a fixed point."""
    lev = np.zeros(nnodes, dtype=np.int64)
    changed = True
    while changed:
        changed = False
        for (u, v) in edges:
            if lev[u] + 1 > lev[v]:
                lev[v] = lev[u] + 1
                changed = True
    return lev


# ---------------------------------------------------------------------------
# symbolic structure, flops, supernodes, levels
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(8))
def test_symbolic_matches_dense_boolean_elimination(seed):
    n = [8, 17, 30, 45, 64, 64, 50, 64][seed]
    dens = [0.2, 0.1, 0.08, 0.05, 0.04, 0.1, 0.03, 0.02][seed]
    M0 = random_mask(n, dens, seed)
    A = csr_of_mask(M0)
    o = oracle_of(A).symbolic()
    Lp, Li, Up, Ui = o.symbolic_structure()
    M = fill_bool(M0)
    assert np.array_equal(structure_to_mask(n, Lp, Li), np.tril(M, -1))
    assert np.array_equal(structure_to_mask(n, Up, Ui), np.triu(M))


@pytest.mark.parametrize("seed", range(4))
def test_symbolic_matches_numeric_lu_pattern(seed):
    n = 40
    rng = np.random.default_rng(100 + seed)
    M0 = random_mask(n, 0.06, 100 + seed)
    D = np.where(M0, rng.standard_normal((n, n)), 0.0)
    D[np.arange(n), np.arange(n)] = 10.0 + rng.random(n)
    L, U = lu_nopivot(D)
    o = oracle_of(csr_of_mask(M0, D)).symbolic()
    Lp, Li, Up, Ui = o.symbolic_structure()
    assert np.array_equal(structure_to_mask(n, Lp, Li), np.tril(L, -1) != 0)
    assert np.array_equal(structure_to_mask(n, Up, Ui), U != 0)


def _flops_dense(n):
    """Row k of a dense n x n matrix is a source for n-1-k rows, each costing
    one division and n-1-k multiply-subtract pairs."""
    return sum(m * (1 + 2 * m) for m in range(n))


@pytest.mark.parametrize("n", [1, 2, 3, 7, 20, 33])
def test_closed_forms_dense(n):
    M = np.ones((n, n), bool)
    o = oracle_of(csr_of_mask(M)).analyse()
    s = o.sizes()
    # (2/3) n^3 - n^2/2 - n/6, evaluated exactly
    assert 6 * s["flops"] == 4 * n ** 3 - 3 * n ** 2 - n
    assert s["flops"] == _flops_dense(n)
    ptr, sn = o.partition_arrays()
    if n >= 2:
        assert list(ptr) == [0, n] and list(sn) == [1]
    lev = o.level_arrays()
    assert lev.max() == 0


@pytest.mark.parametrize("n", [2, 3, 10, 57])
def test_closed_forms_tridiagonal(n):
    M = np.eye(n, dtype=bool) | np.eye(n, k=1, dtype=bool) | np.eye(n, k=-1, dtype=bool)
    o = oracle_of(csr_of_mask(M)).analyse()
    s = o.sizes()
    assert s["flops"] == 3 * (n - 1)
    assert s["nnz_l"] == n - 1 and s["nnz_u"] == 2 * n - 1
    ptr, sn = o.partition_arrays()
    # only the last two rows form a supernode
    assert list(sn) == [0] * (n - 2) + [1] and ptr[-2] == n - 2
    lev = o.level_arrays()
    assert lev[0].max() + 1 == n - 1 and lev[1].max() + 1 == n - 1


@pytest.mark.parametrize("n", [5, 16])
def test_closed_forms_arrowhead(n):
    last = np.zeros((n, n), bool); last[-1, :] = last[:, -1] = True
    o = oracle_of(csr_of_mask(last)).analyse()
    assert o.sizes()["flops"] == 3 * (n - 1)                  # hub last: no fill
    assert o.sizes()["nnz_l"] + o.sizes()["nnz_u"] == 3 * n - 2
    first = np.zeros((n, n), bool); first[0, :] = first[:, 0] = True
    o = oracle_of(csr_of_mask(first)).analyse()
    assert 6 * o.sizes()["flops"] == 4 * n ** 3 - 3 * n ** 2 - n  # hub first: complete fill


def test_closed_forms_block_diagonal():
    sizes = [3, 5, 1, 4, 2]
    n = sum(sizes)
    M = np.zeros((n, n), bool)
    s0 = 0
    for b in sizes:
        M[s0:s0 + b, s0:s0 + b] = True
        s0 += b
    o = oracle_of(csr_of_mask(M)).analyse()
    ptr, sn = o.partition_arrays()
    assert list(ptr) == [0, 3, 8, 9, 13, 15] and list(sn) == [1, 1, 0, 1, 1]
    assert o.level_arrays().max() == 0
    assert o.sizes()["flops"] == sum(_flops_dense(b) for b in sizes)


@pytest.mark.parametrize("seed", range(6))
def test_partition_and_levels_bruteforce(seed):
    n = 48
    M0 = random_mask(n, 0.05, 200 + seed, band=12 if seed % 2 else None)
    M = fill_bool(M0)
    for sn_min, sn_max in [(2, 1 << 30), (3, 4), (2, 2)]:
        o = oracle_of(csr_of_mask(M0)).analyse(sn_min, sn_max)
        ptr, sn = o.partition_arrays()
        eptr, esn = partition_from_mask(M, sn_min, sn_max)
        assert np.array_equal(ptr, eptr) and np.array_equal(sn, esn)
        node_of = np.repeat(np.arange(len(sn)), np.diff(ptr))
        EL, EU = set(), set()
        for i in range(n):
            for k in np.nonzero(M[i, :i])[0]:
                if node_of[k] != node_of[i]:
                    EL.add((node_of[k], node_of[i]))
            for c in np.nonzero(M[i, i + 1:])[0] + i + 1:
                if node_of[c] != node_of[i]:
                    EU.add((node_of[c], node_of[i]))
        nn = len(sn)
        lev = o.level_arrays()
        assert np.array_equal(lev[0], levels_relaxation(nn, EL))
        assert np.array_equal(lev[1], levels_relaxation(nn, EU))
        assert np.array_equal(lev[2], levels_relaxation(nn, [(v, u) for (u, v) in EU]))
        assert np.array_equal(lev[3], levels_relaxation(nn, [(v, u) for (u, v) in EL]))


def test_flops_count_dense_elimination_work():
    """F equals the multiply-add and divide count of a dense right-looking
    elimination that skips structural zeros, counted operation by operation."""
    n = 40
    M0 = random_mask(n, 0.07, 7)
    M = fill_bool(M0)
    ops = 0
    for k in range(n):
        for i in range(k + 1, n):
            if M[i, k]:
                ops += 1                                   # the multiplier
                for j in range(k + 1, n):
                    if M[k, j]:
                        ops += 2                           # multiply + subtract
    assert oracle_of(csr_of_mask(M0)).analyse().sizes()["flops"] == ops


# ---------------------------------------------------------------------------
# numerical factorisation
# ---------------------------------------------------------------------------

def unpack_factors(o, n):
    """Dense L (unit, row-indexed multipliers), U_st and piv from the oracle."""
    Fp, Fi, Fv, Sp, Si, Sv, piv = o.factors()
    L = np.eye(n)
    r = np.repeat(np.arange(n), np.diff(Fp))
    L[r, Fi] = Fv
    Ust = np.zeros((n, n))
    r = np.repeat(np.arange(n), np.diff(Sp))
    Ust[r, Si] = Sv
    return L, Ust, piv


@pytest.mark.parametrize("n", [1, 2, 5, 16, 33])
def test_dense_supernode_equals_getrf_of_transpose(n):
    """One dense supernode with column pivoting = LAPACK getrf on A^T."""
    rng = np.random.default_rng(n)
    D = rng.standard_normal((n, n))
    o = oracle_of(synth.csr_from_dense(D)).analyse().numeric(1e-300)
    L, Ust, piv = unpack_factors(o, n)
    lu, ipiv = sla.lu_factor(D.T)
    perm = np.arange(n)
    for k in range(n):
        perm[k], perm[ipiv[k]] = perm[ipiv[k]], perm[k]
    assert np.array_equal(piv, perm)
    Lp = np.tril(lu, -1) + np.eye(n)       # L' of A^T[perm] = L' U'
    Up = np.triu(lu)
    U_ours = Ust[:, piv]                    # A[:, piv] = L U_ours
    d = np.diag(Up)
    np.testing.assert_allclose(L, (Up / d[:, None]).T, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(U_ours, (Lp * d[None, :]).T, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", range(5))
def test_dominant_matrix_matches_lapack_lu(seed):
    """Row- and column-dominant sparse matrices: no pivoting on either side,
    so the oracle's factors equal scipy's dense LU (which must report P = I)."""
    n = 60
    rng = np.random.default_rng(300 + seed)
    M0 = random_mask(n, 0.08, 300 + seed, band=None if seed % 2 else 6)
    D = np.where(M0, rng.uniform(-1, 1, (n, n)), 0.0)
    s = np.maximum(np.abs(D).sum(0), np.abs(D).sum(1))
    D[np.arange(n), np.arange(n)] = 2.0 * s + 1.0
    P, Ld, Ud = sla.lu(D)
    assert np.array_equal(P, np.eye(n))
    o = oracle_of(synth.csr_from_dense(D)).analyse().numeric(TAU64)
    assert o.sizes()["n_supernodes"] >= 1 or seed % 2 == 0
    L, Ust, piv = unpack_factors(o, n)
    assert np.array_equal(piv, np.arange(n))
    np.testing.assert_allclose(L, Ld, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(Ust, Ud, rtol=1e-12, atol=1e-13)


def integer_factor_case(n, density, seed, band=None):
    """A = L U with integer factors on a closed (filled) structure."""
    rng = np.random.default_rng(seed)
    M = fill_bool(random_mask(n, density, seed, band))
    L = np.where(np.tril(M, -1), rng.choice([-2, -1, 1, 2], (n, n)), 0).astype(np.int64)
    L += np.eye(n, dtype=np.int64)
    U = np.where(np.triu(M, 1), rng.integers(-3, 4, (n, n)), 0).astype(np.int64)
    U[np.arange(n), np.arange(n)] = rng.choice([-1, 1], n) * 2 ** rng.integers(2, 5, n)
    A = L @ U
    assert np.all(A[~M] == 0)
    r, c = np.nonzero(M)
    return synth.csr_from_coo(n, r, c, A[r, c].astype(np.float64)), L, U


@pytest.mark.parametrize("seed", range(6))
def test_integer_factors_bit_exact(seed):
    n = [12, 30, 50, 64, 64, 40][seed]
    A, L, U = integer_factor_case(n, [0.2, 0.08, 0.05, 0.03, 0.06, 0.1][seed], 400 + seed,
                                  band=8 if seed >= 4 else None)
    o = oracle_of(A).analyse().numeric(TAU64)
    assert o.sizes()["n_perturbed"] == 0
    Lo, Ust, piv = unpack_factors(o, n)
    assert np.array_equal(piv, np.arange(n))
    assert np.array_equal(Lo, L.astype(np.float64))
    assert np.array_equal(Ust, U.astype(np.float64))


def test_integer_factors_refactor_reuses_pivots():
    A, L, U = integer_factor_case(40, 0.1, 77)
    o = oracle_of(A).analyse().numeric(TAU64)
    piv = o.factors()[-1]
    o.numeric(TAU64, piv=piv)
    Lo, Ust, piv2 = unpack_factors(o, 40)
    assert np.array_equal(piv2, piv) and np.array_equal(Lo, L) and np.array_equal(Ust, U)


# ---------------------------------------------------------------------------
# substitution, permutations and scalings, transposed solve, gradient
# ---------------------------------------------------------------------------

def _perm_case(n, seed):
    rng = np.random.default_rng(seed)
    M0 = random_mask(n, 0.1, seed)
    D = np.where(M0, rng.uniform(-1, 1, (n, n)), 0.0)
    D[np.arange(n), np.arange(n)] = 3.0 * np.abs(D).sum(1) + 1
    q = rng.permutation(n)
    dr = rng.uniform(0.95, 1.05, n)
    dc = rng.uniform(0.95, 1.05, n)
    return synth.csr_from_dense(D), D, q, dr, dc


@pytest.mark.parametrize("seed", range(4))
def test_solve_with_permutation_and_scaling(seed):
    n = 50
    A, D, q, dr, dc = _perm_case(n, 500 + seed)
    o = oracle_of(A, perm_r=q, perm_c=q, dr=dr, dc=dc).analyse().numeric(TAU64)
    assert o.sizes()["n_perturbed"] == 0
    # B = R A C as formed by the oracle
    rp, ci, bv = o.B()
    Bd = np.zeros((n, n)); Bd[np.repeat(np.arange(n), np.diff(rp)), ci] = bv
    np.testing.assert_allclose(Bd, (dr[:, None] * D * dc[None, :])[np.ix_(q, q)], rtol=1e-15)
    # B Pi = L U_st reconstructs B
    L, Ust, piv = unpack_factors(o, n)
    np.testing.assert_allclose(L @ Ust, Bd, atol=1e-12)
    rng = np.random.default_rng(seed)
    b = rng.uniform(-1, 1, n)
    x = o.solve(b)
    np.testing.assert_allclose(x, np.linalg.solve(D, b), rtol=1e-11, atol=1e-12)
    g = rng.uniform(-1, 1, n)
    lam = o.solve_transposed(g)
    np.testing.assert_allclose(lam, np.linalg.solve(D.T, g), rtol=1e-11, atol=1e-12)
    eta, r1 = o.backward_error(b, x)
    assert eta < 1e-15 and r1 < 1e-14


def test_solve_pivoted_supernodes_against_numpy():
    """Dense-ish blocks with random values force real column pivots."""
    n = 40
    rng = np.random.default_rng(9)
    M0 = fill_bool(random_mask(n, 0.15, 9))
    D = np.where(M0, rng.standard_normal((n, n)), 0.0)
    D[np.arange(n), np.arange(n)] += 0.1
    o = oracle_of(synth.csr_from_dense(D)).analyse().numeric(1e-300)
    L, Ust, piv = unpack_factors(o, n)
    assert not np.array_equal(piv, np.arange(n))
    np.testing.assert_allclose(L @ Ust, D, atol=1e-10)
    b = rng.standard_normal(n)
    x = o.solve(b)
    np.testing.assert_allclose(D @ x, b, atol=1e-9)
    lam = o.solve_transposed(b)
    np.testing.assert_allclose(D.T @ lam, b, atol=1e-9)


def test_perturbation_counts_and_refinement():
    """[[0,1],[1,1]] without static pivoting or supernodes: one zero pivot is
    replaced by tau; refinement then recovers the solution."""
    A = synth.csr_from_dense(np.array([[0.0, 1.0], [1.0, 1.0]]))
    o = oracle_of(A).analyse(sn_min=3).numeric(TAU64)
    assert o.sizes()["n_perturbed"] == 1
    b = np.array([1.0, 3.0])
    x, it, eta = o.solve_ir(b, tol=1e-15, maxit=20)
    np.testing.assert_allclose(x, [2.0, 1.0], rtol=1e-12)
    assert it >= 1 and eta < 1e-15
    # with supernode pivoting the block pivot avoids the zero
    o2 = oracle_of(A).analyse().numeric(TAU64)
    assert o2.sizes()["n_perturbed"] == 0
    np.testing.assert_allclose(o2.solve(b), [2.0, 1.0], rtol=1e-15)


def test_matching_certificate():
    n = 30
    rng = np.random.default_rng(3)
    D = np.where(random_mask(n, 0.2, 3), rng.uniform(-1, 1, (n, n)), 0.0)
    D[np.arange(n), np.arange(n)] = rng.choice([-1.0, 1.0], n)
    o = oracle_of(synth.csr_from_dense(D))
    assert o.check_matching()
    D2 = D.copy(); D2[0, 0] = 0.5
    assert not oracle_of(synth.csr_from_dense(D2)).check_matching()
    D3 = D.copy(); D3[2, 5] = 1.5
    assert not oracle_of(synth.csr_from_dense(D3)).check_matching()
    q = rng.permutation(n)
    assert not oracle_of(synth.csr_from_dense(D), perm_r=q, perm_c=np.arange(n)).check_matching()


def test_gradient_closed_form_and_finite_differences():
    n = 30
    A, D, q, dr, dc = _perm_case(n, 900)
    rng = np.random.default_rng(901)
    b = rng.uniform(-1, 1, n)
    xt = rng.uniform(-1, 1, n)
    o = oracle_of(A, perm_r=q, perm_c=q, dr=dr, dc=dc).analyse().numeric(TAU64)
    x = o.solve(b)
    lam = o.solve_transposed(x - xt)       # dL/dx for L = 0.5 ||x - xt||^2
    g = o.gradient_values(lam, x)
    rows = A.rows()
    np.testing.assert_allclose(g, -np.outer(lam, x)[rows, A.col], rtol=1e-13, atol=1e-15)

    def loss(Dm, bb):
        xx = np.linalg.solve(Dm, bb)
        return 0.5 * np.sum((xx - xt) ** 2)

    h = 1e-6
    for p in rng.choice(A.nnz, 12, replace=False):
        Dp = D.copy(); Dp[rows[p], A.col[p]] += h
        Dm = D.copy(); Dm[rows[p], A.col[p]] -= h
        fd = (loss(Dp, b) - loss(Dm, b)) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 * max(1.0, abs(g[p]))
    for i in rng.choice(n, 5, replace=False):
        bp = b.copy(); bp[i] += h
        bm = b.copy(); bm[i] -= h
        assert abs((loss(D, bp) - loss(D, bm)) / (2 * h) - lam[i]) <= 1e-6
    # homogeneity: sum g_A * A + g_b * b = lam^T (b - A x) ~ 0
    assert abs(np.dot(g, A.val) + np.dot(lam, b)) < 1e-10


def test_config0_natural_order_solution():
    w = synth.config(0)
    o = oracle_of(w.A).analyse().numeric(TAU64)
    x = o.solve(w.b[:, 0])
    assert np.abs(x - w.x_true[:, 0]).max() < 1e-12
    eta, _ = o.backward_error(w.b[:, 0], x)
    assert eta < 1e-15


def test_pivot_tie_takes_lowest_column():
    """Hand-computed: [[1,1],[1,2]] is one supernode; row 0 ties between its
    two block columns and must take column 0, leaving column 1 to row 1."""
    A = synth.csr_from_dense(np.array([[1.0, 1.0], [1.0, 2.0]]))
    o = oracle_of(A).analyse().numeric(TAU64)
    L, Ust, piv = unpack_factors(o, 2)
    assert list(piv) == [0, 1]
    assert np.array_equal(L, [[1, 0], [1, 1]]) and np.array_equal(Ust, [[1, 1], [0, 1]])


# ---------------------------------------------------------------------------
# backward error, value reload and perturbation threshold against their
# definitions, computed here without the oracle
# ---------------------------------------------------------------------------

def _dense_eta(D, b, x):
    """Normwise backward error max|b - Dx| / (max_i sum_j |D_ij| max|x| + max|b|)
    and the paper's accuracy measure sum|Dx - b| / sum|b| (Sec. 3.3)."""
    r = b - D @ x
    eta = np.abs(r).max() / (np.abs(D).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max())
    return eta, np.abs(r).sum() / np.abs(b).sum()


@pytest.mark.parametrize("case", ["A_x_term", "b_term", "balanced"])
def test_backward_error_against_dense_definition(case):
    """Cases where each term of the denominator dominates, on a matrix whose
    largest row sum differs from its largest column sum (a transposed norm, a
    dropped ||b|| or ||A|| ||x|| term, or a 1-norm for an infinity norm each
    change the value by far more than the tolerance)."""
    n = 60
    rng = np.random.default_rng(31)
    D = np.where(random_mask(n, 0.1, 31), rng.uniform(-1, 1, (n, n)), 0.0)
    D[7, ::2] = 4.0                                   # one heavy row
    A = synth.csr_from_dense(D)
    assert np.abs(D).sum(axis=1).max() > 1.5 * np.abs(D).sum(axis=0).max()
    scale_x, scale_b = {"A_x_term": (1e3, 1e-3), "b_term": (1e-6, 1e2), "balanced": (1.0, 100.0)}[case]
    x = scale_x * rng.uniform(-1, 1, n)
    b = scale_b * rng.uniform(-1, 1, n)
    eta, r1 = oracle_of(A).backward_error(b, x)
    eta_d, r1_d = _dense_eta(D, b, x)
    assert abs(eta - eta_d) <= 1e-13 * eta_d and abs(r1 - r1_d) <= 1e-13 * r1_d
    # the terms really differ in size where they are meant to
    ax = np.abs(D).sum(axis=1).max() * np.abs(x).max()
    bx = np.abs(b).max()
    assert {"A_x_term": ax > 1e5 * bx, "b_term": bx > 1e5 * ax, "balanced": 0.1 < ax / bx < 10}[case]


def test_backward_error_exact_integers():
    """Integer A, x and b: the residual and both norms are exact, so the
    backward error is the correctly rounded quotient of two integers."""
    from fractions import Fraction
    n = 25
    rng = np.random.default_rng(32)
    D = np.where(random_mask(n, 0.2, 32), rng.integers(-9, 10, (n, n)), 0).astype(np.float64)
    A = synth.csr_from_dense(D)
    x = rng.integers(-50, 51, n).astype(np.float64)
    b = rng.integers(-70, 71, n).astype(np.float64)
    eta, r1 = oracle_of(A).backward_error(b, x)
    Di = D.astype(np.int64)
    r = b.astype(np.int64) - Di @ x.astype(np.int64)
    den = int(np.abs(Di).sum(axis=1).max()) * int(np.abs(x).max()) + int(np.abs(b).max())
    assert eta == float(Fraction(int(np.abs(r).max()), den))
    assert r1 == float(Fraction(int(np.abs(r).sum()), int(np.abs(b).sum())))


def test_set_values_matches_fresh_oracle():
    """The repeated-solve path (Sec. 3.2): new values on the same pattern
    through set_values give B, factors and solutions bit-identical to an
    oracle created with those values, with and without the pivot search, and
    B equals R A C formed here from the new values."""
    n = 60
    A, D, q, dr, dc = _perm_case(n, 77)
    rng = np.random.default_rng(78)
    v1 = A.val * rng.uniform(0.5, 1.5, A.nnz)
    o = oracle_of(A, perm_r=q, perm_c=q, dr=dr, dc=dc).analyse().numeric(TAU64)
    piv = o.factors()[-1]
    o.set_values(v1)
    A1 = synth.Csr(A.n, A.row_ptr, A.col, v1)
    f = oracle_of(A1, perm_r=q, perm_c=q, dr=dr, dc=dc).analyse()
    for a, c in zip(o.B(), f.B()):
        assert np.array_equal(a, c)
    rp, ci, bv = o.B()
    rows = A.rows()
    Bd = np.zeros((n, n))
    Bd[rows, A.col] = (dr[rows] * v1) * dc[A.col]
    qinv = np.argsort(q)
    assert np.array_equal(bv, Bd[np.ix_(q, q)][np.repeat(np.arange(n), np.diff(rp)), ci])
    assert np.array_equal(np.sort(qinv[A.col]), np.sort(ci))
    o.numeric(TAU64, piv=piv)
    f.numeric(TAU64, piv=piv)
    for a, c in zip(o.factors(), f.factors()):
        assert np.array_equal(a, c)
    o.numeric(TAU64)
    f.numeric(TAU64)
    for a, c in zip(o.factors(), f.factors()):
        assert np.array_equal(a, c)
    b = rng.uniform(-1, 1, n)
    assert np.array_equal(o.solve(b), f.solve(b))
    np.testing.assert_allclose(o.solve(b), np.linalg.solve(_dense(A1), b), rtol=1e-11, atol=1e-12)


def _dense(A):
    D = np.zeros((A.n, A.n))
    D[A.rows(), A.col] = A.val
    return D


def test_pivot_tau_from_own_B():
    """tau = sqrt(eps) max|B| with B = R A C formed here; exactly sqrt(eps)
    when the scaling leaves a unit maximum; the rel argument scales it."""
    n = 40
    A, D, q, dr, dc = _perm_case(n, 91)
    o = oracle_of(A, perm_r=q, perm_c=q, dr=dr, dc=dc)
    bmax = np.abs((dr[:, None] * D) * dc[None, :]).max()
    assert o.pivot_tau() == TAU64 * bmax
    assert o.pivot_tau(1e-3) == 1e-3 * bmax
    Dn = D / np.abs(D).max()
    assert oracle_of(synth.csr_from_dense(Dn)).pivot_tau() == TAU64
