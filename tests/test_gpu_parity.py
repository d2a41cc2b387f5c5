"""HIP path against the CPU oracle, through the C ABI (needs an MI355X).

Tolerances: FP64 factors within 1e-11 of the oracle (normwise, relative to the
largest entry); solutions within 1e-10 normwise relative difference; backward
error at most 1e-12 (FP64 and FP32 with refinement); integer factors bit-exact.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2509_07690_amd import synth  # noqa: E402
from parity import oracle_for, compare_factors, compare_backward_stability, rel_diff  # noqa: E402

TAU64 = np.sqrt(np.finfo(np.float64).eps)

@pytest.fixture(scope="module")
def hylu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_07690_amd import hylu as H
    return H


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def run_case(hylu, A, b, opts=None, sn=(2, 1 << 30), exact=False, tol=1e-11):
    opts = dict(opts or {})
    print(f"[case] n={A.n} nnz={A.nnz} opts={opts}", flush=True)
    h = hylu.Handle(A.row_ptr, A.col, A.val, **opts)
    o, sym = oracle_for(h, A, *sn)
    vals = dev(A.val)
    h.factorize(vals)
    torch.cuda.synchronize()
    o.numeric(o.tau)
    assert h.info()["n_perturbed"] == o.sizes()["n_perturbed"]
    compare_factors(h, o, tol=tol, exact=exact)
    x = h.solve(dev(b)).cpu().numpy()
    xo = o.solve(b)
    eta, _ = o.backward_error(b, x)
    return h, o, x, xo, eta


@pytest.mark.parametrize("pipe", [0, 1024])
@pytest.mark.parametrize("tail", [0.0, 0.5])
def test_random_small(hylu, tail, pipe):
    for seed in range(4):
        rng = np.random.default_rng(seed)
        n = 300
        M = rng.random((n, n)) < 0.015
        np.fill_diagonal(M, True)
        D = np.where(M, rng.standard_normal((n, n)), 0.0)
        A = synth.csr_from_dense(D)
        b = rng.standard_normal(n)
        h, o, x, xo, eta = run_case(hylu, A, b, opts=dict(dense_tail=tail, pipeline_rows=pipe))
        assert rel_diff(x, xo) <= 1e-10 and eta <= 1e-12
        if tail == 0:
            assert (h.info()["pipe_tasks"] > 0) == (pipe > 0)
        assert (h.info()["tail_rows"] > 0) == (tail > 0)


@pytest.mark.parametrize("n,opts", [(70, {}), (70, dict(dense_tail=0.0, sn_dense=32)),
                                    (70, dict(dense_tail=0.0, sn_dense=0)), (300, dict(dense_tail=0.0, sn_dense=32))])
def test_dense_block_pivoting(hylu, n, opts):
    """One dense supernode with column pivoting: through the dense tail, the
    blocked supernode path (16-row panels, wide pivot window) and the
    one-workgroup kernel."""
    rng = np.random.default_rng(11)
    D = rng.standard_normal((n, n))
    A = synth.csr_from_dense(D)
    b = rng.standard_normal(n)
    h, o, x, xo, eta = run_case(hylu, A, b, opts=dict(static_pivot=0, ordering="natural", **opts))
    assert h.info()["max_supernode"] == n
    assert not np.array_equal(h.symbolic()["perm_r"], None)
    assert rel_diff(x, xo) <= 1e-10 and eta <= 1e-12


def _integer_case(n, density, seed):
    rng = np.random.default_rng(seed)
    M = rng.random((n, n)) < density
    np.fill_diagonal(M, True)
    # close the structure (dense boolean elimination)
    for k in range(n):
        rows = np.nonzero(M[k + 1:, k])[0] + k + 1
        if rows.size:
            M[np.ix_(rows, np.arange(k + 1, n))] |= M[k, k + 1:]
    L = np.where(np.tril(M, -1), rng.choice([-2, -1, 1, 2], (n, n)), 0).astype(np.int64) + np.eye(n, dtype=np.int64)
    U = np.where(np.triu(M, 1), rng.integers(-3, 4, (n, n)), 0).astype(np.int64)
    U[np.arange(n), np.arange(n)] = rng.choice([-1, 1], n) * 2 ** rng.integers(2, 5, n)
    Aint = L @ U
    r, c = np.nonzero(M)
    return synth.csr_from_coo(n, r, c, Aint[r, c].astype(np.float64)), L, U


@pytest.mark.parametrize("seed", range(3))
def test_integer_factors_bit_exact(hylu, seed):
    """Integer L and U with power-of-two pivots: every intermediate of the
    substitution is a small dyadic number, so the factors are exact.  The
    block-inverse form of the sup-row update rounds the inverse's entries,
    so it is off here (sn_inverse=0); it is compared at tolerance elsewhere."""
    A, L, U = _integer_case([40, 90, 150][seed], [0.1, 0.04, 0.02][seed], 700 + seed)
    b = np.arange(A.n, dtype=np.float64)
    h, o, x, xo, eta = run_case(hylu, A, b, opts=dict(static_pivot=0, ordering="natural", sn_inverse=0), exact=True)


@pytest.mark.parametrize("ordering,tail,tile", [("amd", 0.5, 16), ("nd", 0.5, 16), ("amd", 0.0, 16), ("amd", 0.05, 16),
                                               ("nd", 0.0, 2), ("nd", 0.0, 0)])
def test_config0_factor_solve(hylu, ordering, tail, tile):
    """tile: supernode targets of at least this many rows take their updates
    by 16-row tiles (2: every supernode; 0: the row kernel only)."""
    w = synth.config(0)
    h, o, x, xo, eta = run_case(hylu, w.A, w.b[:, 0], opts=dict(ordering=ordering, dense_tail=tail, sn_tile=tile))
    print("tail rows", h.info()["tail_rows"], "panels", h.info()["tail_panels"])
    assert rel_diff(x, xo) <= 1e-10 and eta <= 1e-12
    assert np.abs(x - w.x_true[:, 0]).max() < 1e-10


@pytest.mark.parametrize("tail,pipe", [(0.0, 0), (0.3, 0), (0.0, 1024), (0.3, 300)])
def test_config0_refactor_and_transpose(hylu, tail, pipe):
    w = synth.config(0)
    A = w.A
    print(f"[case] config0 refactor tail={tail} pipe={pipe}", flush=True)
    h = hylu.Handle(A.row_ptr, A.col, A.val, dense_tail=tail, pipeline_rows=pipe)
    o, sym = oracle_for(h, A)
    h.factorize(dev(A.val))
    torch.cuda.synchronize()
    piv = hylu.factors_as_rows(h)[2]
    for seed in (5, 6):
        A2 = synth.grid_values(A, seed, 4.0)
        v2 = dev(A2.val)
        h.refactor(v2)
        torch.cuda.synchronize()
        o.set_values(A2.val)
        o.numeric(o.tau, piv=piv)
        compare_factors(h, o)
        b = A2.matvec(w.x_true[:, 0])
        x = h.solve(dev(b)).cpu().numpy()
        assert rel_diff(x, o.solve(b)) <= 1e-10 and o.backward_error(b, x)[0] <= 1e-12
        g = np.random.default_rng(seed).uniform(-1, 1, A.n)
        lam = h.solve(dev(g), transpose=True).cpu().numpy()
        lo = o.solve_transposed(g)
        assert rel_diff(lam, lo) <= 1e-10


def test_multiple_rhs(hylu):
    w = synth.config(0)
    A = w.A
    h = hylu.Handle(A.row_ptr, A.col, A.val)
    o, _ = oracle_for(h, A)
    h.factorize(dev(A.val))
    o.numeric(o.tau)
    B = np.random.default_rng(3).uniform(-1, 1, (A.n, 5))
    X = h.solve_cols(dev(B.T.copy())).cpu().numpy().T
    for k in range(5):
        assert rel_diff(X[:, k], o.solve(B[:, k])) <= 1e-10


def test_fp32_with_refinement(hylu):
    w = synth.config(0)
    A = w.A
    h = hylu.Handle(A.row_ptr, A.col, A.val, precision="fp32")
    o, _ = oracle_for(h, A)
    h.factorize(dev(A.val))
    o.numeric(o.tau)
    b = w.b[:, 0]
    x = h.solve(dev(b)).cpu().numpy()
    eta, _ = o.backward_error(b, x)
    inf = h.info()
    print("fp32+IR iterations", inf["ir_iters"], "eta", eta, "diff", rel_diff(x, o.solve(b)))
    assert eta <= 1e-12 and rel_diff(x, o.solve(b)) <= 1e-10 and inf["ir_iters"] >= 1


def test_perturbation_triggers_refinement(hylu):
    A = synth.csr_from_dense(np.array([[0.0, 1.0], [1.0, 1.0]]))
    h = hylu.Handle(A.row_ptr, A.col, A.val, static_pivot=0, ordering="natural", sn_min=3)
    h.factorize(dev(A.val))
    b = np.array([1.0, 3.0])
    x = h.solve(dev(b)).cpu().numpy()
    inf = h.info()
    assert inf["n_perturbed"] == 1 and inf["ir_iters"] >= 1
    np.testing.assert_allclose(x, [2.0, 1.0], rtol=1e-12)


@pytest.mark.parametrize("m", [0, 1])
def test_batch_members(hylu, m):
    w = synth.batch_member(m)
    h, o, x, xo, eta = run_case(hylu, w.A, w.b[:, 0])
    assert rel_diff(x, xo) <= 1e-10 and eta <= 1e-12


@pytest.mark.parametrize("pipe", [0, 16])
def test_small_circuit(hylu, pipe):
    """Power-law circuit pattern at n = 20000: hub supernodes, a dense tail,
    and (pipe > 0) every narrow level in the pipelined launch."""
    w = synth.circuit_powerlaw(20000)
    h, o, x, xo, eta = run_case(hylu, w.A, w.b[:, 0],
                                opts=dict(amd_dense=0.1, dense_tail=0.15, pipeline_rows=pipe))
    assert rel_diff(x, xo) <= 1e-10 and eta <= 1e-12
    w2 = w.revalue(1)
    piv = hylu.factors_as_rows(h)[2]
    h.refactor(dev(w2.A.val))
    torch.cuda.synchronize()
    o.set_values(w2.A.val)
    o.numeric(o.tau, piv=piv)
    compare_factors(h, o)


@pytest.mark.parametrize("side,sn_dense,tail,tile,inv", [(12, 16, 0.0, 16, 1), (16, 32, 0.15, 16, 1), (16, 2, 0.0, 2, 1),
                                                        (16, 128, 0.0, 0, 1), (16, 128, 0.0, 0, 0), (16, 64, 0.0, 0, 0)])
def test_grid3d_blocked_supernodes(hylu, side, sn_dense, tail, tile, inv):
    """7-point 3D grid (ND): supernodes of at least sn_dense rows go through
    the blocked panel / TRSM / MFMA-GEMM kernels on side streams.  Pivots and
    structure bit-exact; L and U are not diagonally dominant here (growth
    ~1e3 in each), so the entries are compared with a growth-derived tolerance
    and the device factors must reproduce B as closely as the oracle's do;
    refactorisation through the graph; the solve against the oracle.  inv:
    sup-row multipliers from the block inverse (1) or by substitution (0)."""
    w = synth.convdiff3d_7pt(side)
    A = w.A
    h, o, x, xo, eta = run_case(hylu, A, w.b[:, 0], opts=dict(ordering="nd", sn_dense=sn_dense, dense_tail=tail,
                                                              sn_tile=tile, sn_inverse=inv), tol="derived")
    print("residual ratios (device, oracle):", compare_backward_stability(h, o))
    assert rel_diff(x, xo) <= 1e-10 and eta <= 1e-12
    A2 = synth.grid_values(A, 77, 4.0)
    piv = hylu.factors_as_rows(h)[2]
    h.refactor(dev(A2.val))
    torch.cuda.synchronize()
    o.set_values(A2.val)
    o.numeric(o.tau, piv=piv)
    compare_factors(h, o, tol="derived")
    compare_backward_stability(h, o)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_grid27_grouped_panels(hylu, precision):
    """27-point 3D grid 24^3 (ND, the supernode-heavy PDE path) with the
    panel-group thresholds lowered (group_min_rows 128, group_tail_rows 256)
    so the large supernodes' dense views and the dense tail go through the
    grouped panels that the 64^3 grid takes at full size: pivots and structure
    bit-exact, FP64 factors entry by entry (growth-derived tolerance) and by
    their residual, two right-hand sides against the oracle's solutions with
    backward error at most 1e-12 (FP32 factors: after FP64 refinement), then a
    refactorisation with new values through the graph."""
    w = synth.convdiff3d_27pt(24, nrhs=2)
    A = w.A
    opts = dict(ordering="nd_ml", dense_tail=0.5, group_min_rows=128, group_tail_rows=256, precision=precision)
    print(f"[case] 27-point 24^3 grouped {precision}", flush=True)
    h = hylu.Handle(A.row_ptr, A.col, A.val, **opts)
    inf = h.info()
    assert inf["n_dense_sn"] > 0 and inf["sn_groups"] > 0 and inf["tail_groups"] > 0, inf
    o, _ = oracle_for(h, A)
    h.factorize(dev(A.val))
    o.numeric(o.tau)
    if precision == "fp64":
        assert h.info()["n_perturbed"] == o.sizes()["n_perturbed"]
        compare_factors(h, o, tol="derived")
        print("residual ratios (device, oracle):", compare_backward_stability(h, o))
    X = h.solve_cols(dev(w.b.T.copy())).cpu().numpy()
    for k in range(2):
        b = w.b[:, k]
        assert o.backward_error(b, X[k])[0] <= 1e-12, k
        assert rel_diff(X[k], o.solve(b)) <= 1e-10, k
    A2 = synth.grid_values(A, 78, 26.0)
    piv = hylu.factors_as_rows(h)[2]
    h.refactor(dev(A2.val))
    x2 = h.solve(dev(w.b[:, 0])).cpu().numpy()
    o.set_values(A2.val)
    o.numeric(o.tau, piv=piv)
    if precision == "fp64":
        compare_factors(h, o, tol="derived")
        compare_backward_stability(h, o)
    assert rel_diff(x2, o.solve(w.b[:, 0])) <= 1e-10
    ident = np.arange(A.n, dtype=np.int32)
    import oracle
    o2 = oracle.Oracle(A.n, A2.row_ptr, A2.col, A2.val, ident, ident, np.ones(A.n), np.ones(A.n))
    assert o2.backward_error(w.b[:, 0], x2)[0] <= 1e-12


def test_fp32_refactor_fresh_values_full_circuit(hylu):
    """Circuit n = 200000, FP32 factors: refactorisations with fresh value sets
    on the first factorisation's pivot order converge under FP64 refinement
    to a backward error of at most 1e-10 (the FP64 perturbation threshold
    leaves these pivots alone)."""
    base = synth.circuit_powerlaw(200000)
    A = base.A
    h = hylu.Handle(A.row_ptr, A.col, A.val, precision="fp32", amd_dense=0.1, dense_tail=0.15)
    h.factorize(dev(A.val))
    for r in (1, 3):
        w = base.revalue(r)
        h.refactor(dev(w.A.val))
        x = h.solve(dev(w.b[:, 0])).cpu().numpy()
        ok = __import__("oracle").Oracle(A.n, A.row_ptr, A.col, w.A.val, *[np.arange(A.n, dtype=np.int32)] * 2,
                                         np.ones(A.n), np.ones(A.n))
        eta, _ = ok.backward_error(w.b[:, 0], x)
        print(f"refactor {r}: eta {eta:.2e} ir {h.info()['ir_iters']} perturbed {h.info()['n_perturbed']}")
        assert eta <= 1e-10 and np.abs(x - w.x_true[:, 0]).max() <= 1e-9


@pytest.mark.parametrize("case", ["config0_amd", "config0_nd", "circuit", "grid3d", "circuit_fp32"])
def test_sparse_tail_bit_identical(hylu, case):
    """The block-sparse dense tail skips only 64 x 64 products and triangular
    solves that are exactly zero by structure, and sums the rest in the dense
    order: its factors, pivots and solution equal the dense tail's to the bit,
    on a first factorisation (pivot search) and a refactorisation."""
    if case.startswith("config0"):
        w = synth.config(0)
        A, b, A2 = w.A, w.b[:, 0], synth.config(0).A
        A2 = type(A2)(A2.n, A2.row_ptr, A2.col, A2.val * (1.0 + 0.1 * np.sin(np.arange(A2.nnz))))
        opts = dict(ordering=case.split("_")[1], dense_tail=0.3)
    elif case.startswith("circuit"):
        w = synth.circuit_powerlaw(20000)
        A, b, A2 = w.A, w.b[:, 0], w.revalue(1).A
        opts = dict(amd_dense=0.1, dense_tail=0.05)
        if case.endswith("fp32"):
            opts["precision"] = "fp32"
    else:
        w = synth.convdiff3d_7pt(16)
        A, b, A2 = w.A, w.b[:, 0], synth.grid_values(w.A, 5, 4.0)
        opts = dict(ordering="nd", dense_tail=0.05, sn_dense=32)
    out = []
    for sparse in (0, 1):
        print(f"[case] {case} tail_sparse={sparse} n={A.n}", flush=True)
        h = hylu.Handle(A.row_ptr, A.col, A.val, tail_sparse=sparse, **opts)
        assert h.info()["tail_rows"] > 0
        h.factorize(dev(A.val))
        x = h.solve(dev(b)).cpu().numpy()
        f1 = h.factors_raw()
        h.refactor(dev(A2.val))
        torch.cuda.synchronize()
        f2 = h.factors_raw()
        out.append((h.info()["flops_issued"], f1, f2, x))
    assert out[1][0] < out[0][0]
    for k in ("vals", "piv"):
        assert np.array_equal(out[0][1][k], out[1][1][k]), k
        assert np.array_equal(out[0][2][k], out[1][2][k]), k
    assert np.array_equal(out[0][3], out[1][3])


def test_deferred_row_placement_bit_identical(hylu):
    """Deferred rows placed into the narrow levels, long tail rows split into
    pieces over several launches (side_rows=1), or all run in the final level
    (side_rows=0): every row still applies its sources in the same order with
    the same operations, so factors and solution agree to the bit, on a first
    factorisation and a refactorisation."""
    w = synth.circuit_powerlaw(20000)
    A, b, A2 = w.A, w.b[:, 0], w.revalue(1).A
    out = []
    for side in (0, 1):
        print(f"[case] circuit 20000 side_rows={side}", flush=True)
        h = hylu.Handle(A.row_ptr, A.col, A.val, amd_dense=0.1, dense_tail=0.05, side_rows=side)
        h.factorize(dev(A.val))
        x = h.solve(dev(b)).cpu().numpy()
        f1 = h.factors_raw()
        h.refactor(dev(A2.val))
        torch.cuda.synchronize()
        out.append((f1, h.factors_raw(), x))
    for k in ("vals", "piv"):
        assert np.array_equal(out[0][0][k], out[1][0][k]), k
        assert np.array_equal(out[0][1][k], out[1][1][k]), k
    assert np.array_equal(out[0][2], out[1][2])


@pytest.mark.parametrize("case", ["circuit", "grid3d"])
def test_solve_chains(hylu, case):
    """Runs of narrow solve levels solved by one workgroup per run (Sec. 2.3):
    in FP64 the solution agrees with the per-level launches' (the backward
    solve sums each row in another order; the 7-point grid's condition number,
    ~2e4 at 16^3, turns rounding-level differences into ~1e-13), and both
    agree with the oracle's to 1e-10 with backward error at most 1e-12, in
    FP64 and with FP32 factors and refinement."""
    if case == "circuit":
        w = synth.circuit_powerlaw(20000)
        opts = dict(amd_dense=0.1, dense_tail=0.15)
    else:
        w = synth.convdiff3d_7pt(16)
        opts = dict(ordering="nd", dense_tail=0.15, sn_dense=32)
    A, b = w.A, w.b[:, 0]
    print(f"[case] solve chains {case} n={A.n}", flush=True)
    for precision in ("fp64", "fp32"):
        h1 = hylu.Handle(A.row_ptr, A.col, A.val, precision=precision, **opts)
        h0 = hylu.Handle(A.row_ptr, A.col, A.val, precision=precision, solve_chain=0, **opts)
        assert h1.info()["chain_levels"] > 0 and h0.info()["chain_levels"] == 0
        xs = []
        for h in (h1, h0):
            h.factorize(dev(A.val))
            xs.append(h.solve(dev(b)).cpu().numpy())
        if precision == "fp64":          # FP32 + refinement: two converged iterates, compared via the oracle
            assert rel_diff(xs[0], xs[1]) <= 1e-11
        o, _ = oracle_for(h1, A)
        o.numeric(o.tau)
        for x in xs:
            assert rel_diff(x, o.solve(b)) <= 1e-10
            assert o.backward_error(b, x)[0] <= 1e-12


@pytest.mark.parametrize("member", [0, 2])
def test_solve_split_bit_identical(hylu, member):
    """Forward solve of supernodes with a long L region (Sec. 2.3): the sums
    over that region spread over workgroups of eight rows, then the diagonal
    block, give the solution of one workgroup per supernode to the bit (the
    same per-row order), in FP64 and FP32; with nrhs 3 as well; and the FP64
    solution agrees with the oracle's."""
    w = synth.batch_member(member)
    A = w.A
    rng = np.random.default_rng(7)
    B = rng.standard_normal((A.n, 3))
    print(f"[case] solve split, batch member {member} n={A.n}", flush=True)
    for precision in ("fp64", "fp32"):
        h1 = hylu.Handle(A.row_ptr, A.col, A.val, precision=precision)
        h0 = hylu.Handle(A.row_ptr, A.col, A.val, precision=precision, solve_split=0)
        assert h1.info()["split_sn"] > 0 and h0.info()["split_sn"] == 0
        xs = []
        for h in (h1, h0):
            h.factorize(dev(A.val))
            xs.append((h.solve(dev(B[:, 0])).cpu().numpy(), h.solve(dev(B)).cpu().numpy()))
        assert np.array_equal(h1.factors_raw()["vals"], h0.factors_raw()["vals"])
        assert np.array_equal(xs[0][0], xs[1][0]) and np.array_equal(xs[0][1], xs[1][1])
        if precision == "fp64":
            o, _ = oracle_for(h1, A)
            o.numeric(o.tau)
            assert rel_diff(xs[0][0], o.solve(B[:, 0])) <= 1e-10
            assert o.backward_error(B[:, 0], xs[0][0])[0] <= 1e-12


def test_transposed_split(hylu):
    """Transposed solves (the adjoint's A^T lambda = g) with the nodes of 8
    rows or more split (their outside sums by groups of columns, then their
    block 64 columns at a time; nodes of up to 437 rows here) agree with the
    column-by-column solve and with the oracle's, for one and three
    right-hand sides, in FP64 and with FP32 factors and refinement."""
    w = synth.convdiff3d_7pt(32)
    A = w.A
    rng = np.random.default_rng(11)
    G = rng.standard_normal((A.n, 3))
    print(f"[case] transposed split, 7-point 32^3 n={A.n}", flush=True)
    for precision in ("fp64", "fp32"):
        h1 = hylu.Handle(A.row_ptr, A.col, A.val, ordering="nd", precision=precision)
        h0 = hylu.Handle(A.row_ptr, A.col, A.val, ordering="nd", precision=precision, solve_split=0)
        assert h1.info()["split_sn"] > 0 and h0.info()["split_sn"] == 0
        out = []
        for h in (h1, h0):
            h.factorize(dev(A.val))
            out.append((h.solve(dev(G[:, 0]), transpose=True).cpu().numpy(),
                        h.solve(dev(G), transpose=True).cpu().numpy()))
        if precision == "fp64":
            assert rel_diff(out[0][0], out[1][0]) <= 1e-12
            assert rel_diff(out[0][1], out[1][1]) <= 1e-12
        o, _ = oracle_for(h1, A)
        o.numeric(o.tau)
        for k in range(3):
            lo = o.solve_transposed(G[:, k])
            for x1, xk in out:
                assert rel_diff(xk[:, k], lo) <= 1e-10
                if k == 0:
                    assert rel_diff(x1, lo) <= 1e-10


@pytest.mark.parametrize("case", ["config0", "circuit", "circuit_fp32", "grid3d"])
def test_pipelined_bit_identical(hylu, case):
    """Pipeline mode (Sec. 2.2.1): the runs of narrow levels in chain launches,
    one wavefront per node waiting per source on the nodes of its launch.
    Every row applies its sources in the same order with the same operations
    as the bulk row kernel, and supernodes take the same block LU and inverse:
    factors, pivots and solution equal bulk mode's to the bit, on a first
    factorisation (pivot search) and a refactorisation with new values."""
    if case == "config0":
        w = synth.config(0)
        A, b = w.A, w.b[:, 0]
        A2 = type(A)(A.n, A.row_ptr, A.col, A.val * (1.0 + 0.1 * np.sin(np.arange(A.nnz))))
        opts, rows = dict(dense_tail=0.0), 64
    elif case.startswith("circuit"):
        w = synth.circuit_powerlaw(20000)
        A, b, A2 = w.A, w.b[:, 0], w.revalue(1).A
        opts, rows = dict(amd_dense=0.1, dense_tail=0.15), 16
        if case.endswith("fp32"):
            opts["precision"] = "fp32"
    else:
        w = synth.convdiff3d_7pt(16)
        A, b, A2 = w.A, w.b[:, 0], synth.grid_values(w.A, 5, 4.0)
        opts, rows = dict(ordering="nd", dense_tail=0.05, sn_dense=32), 64
    out = []
    for pipe in (0, rows):
        print(f"[case] {case} pipeline_rows={pipe} n={A.n}", flush=True)
        h = hylu.Handle(A.row_ptr, A.col, A.val, pipeline_rows=pipe, **opts)
        assert (h.info()["pipe_tasks"] > 0) == (pipe > 0)
        h.factorize(dev(A.val))
        x = h.solve(dev(b)).cpu().numpy()
        f1 = h.factors_raw()
        n1 = h.info()["n_perturbed"]
        h.refactor(dev(A2.val))
        torch.cuda.synchronize()
        out.append((f1, h.factors_raw(), x, n1))
    for k in ("vals", "piv"):
        assert np.array_equal(out[0][0][k], out[1][0][k]), k
        assert np.array_equal(out[0][1][k], out[1][1][k]), k
    assert np.array_equal(out[0][2], out[1][2])
    assert out[0][3] == out[1][3]


def test_pipelined_wait_gives_up_cleanly(hylu):
    """The waits of a chain launch are bounded: with the poll limit forced to
    one from the host, a wait gives up at once, every other wait of the launch
    stops, the launch ends, and the factorisation reports a device error (its
    factors void) instead of hanging.  A handle with the default limit then
    factorises the same matrix and matches the oracle."""
    w = synth.circuit_powerlaw(20000)
    A = w.A
    opts = dict(amd_dense=0.1, dense_tail=0.15, pipeline_rows=16)
    print("[case] circuit 20000 pipeline_spin=1", flush=True)
    h = hylu.Handle(A.row_ptr, A.col, A.val, pipeline_spin=1, **opts)
    assert h.info()["pipe_tasks"] > 0
    h.factorize(dev(A.val))
    torch.cuda.synchronize()
    with pytest.raises(hylu.HyluError) as e:
        h.info()
    assert e.value.code == -7                # HYLU_ERR_DEVICE
    h2, o, x, xo, eta = run_case(hylu, A, w.b[:, 0], opts=opts)
    assert rel_diff(x, xo) <= 1e-10 and eta <= 1e-12
