"""Full-size cases in the launch configuration bench.py times (needs an
MI355X).  Where the oracle finishes in seconds (the circuit) the factors and
the solution are compared element by element; elsewhere properties that hold
at any size are checked: the normwise backward error of every solution from
the oracle's FP64 residual (compensated sums), the error against x_true, and
the adjoint's gradient against central differences on sampled entries.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2509_07690_amd import synth  # noqa: E402
from parity import oracle_for, compare_factors, rel_diff  # noqa: E402
import oracle  # noqa: E402


@pytest.fixture(scope="module")
def hylu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_07690_amd import hylu as H
    return H


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def eta_of(A, b, x):
    """Normwise backward error by the oracle's residual (no factorisation)."""
    ident = np.arange(A.n, dtype=np.int32)
    o = oracle.Oracle(A.n, A.row_ptr, A.col, A.val, ident, ident, np.ones(A.n), np.ones(A.n))
    return o.backward_error(b, x)[0]


def test_circuit_full_factors_and_solution(hylu):
    """Circuit n = 200000 with the bench's options: refactorisation with a
    fresh value set, factors entry by entry and the solution against the
    oracle on the same pivot order."""
    base = synth.circuit_powerlaw(200000)
    A = base.A
    print("[case] circuit n=200000 full", flush=True)
    h = hylu.Handle(A.row_ptr, A.col, A.val, amd_dense=0.1, dense_tail=0.15)
    h.factorize(dev(A.val))
    piv = hylu.factors_as_rows(h)[2]
    w = base.revalue(5)
    h.refactor(dev(w.A.val))
    x = h.solve(dev(w.b[:, 0])).cpu().numpy()
    o, _ = oracle_for(h, A)
    o.set_values(w.A.val)
    o.numeric(o.tau, piv=piv)
    compare_factors(h, o)
    xo = o.solve(w.b[:, 0])
    assert rel_diff(x, xo) <= 1e-10
    assert eta_of(w.A, w.b[:, 0], x) <= 1e-12
    assert np.abs(x - w.x_true[:, 0]).max() <= 1e-9


def test_grid7_full_solution_and_sampled_gradient(hylu):
    """7-point grid 48^3 (n = 110592): backward error of the solution and of
    the transposed solve, the gradient as the pattern-restricted outer
    product, 64 sampled entries against forward-mode directional derivatives
    (a plain solve each), and 16 against central differences (h = 1e-6)."""
    w = synth.convdiff3d_7pt(48)
    A, b, xt = w.A, w.b[:, 0], w.extra["x_target"]
    print("[case] 7-point 48^3 full", flush=True)
    h = hylu.Handle(A.row_ptr, A.col, A.val, ordering="nd", dense_tail=0.15)
    val = dev(A.val).requires_grad_()
    bb = dev(b).requires_grad_()
    x = hylu.sparse_solve(h, val, bb)
    (0.5 * ((x - dev(xt)) ** 2).sum()).backward()
    xh = x.detach().cpu().numpy()
    assert eta_of(A, b, xh) <= 1e-12
    assert np.abs(xh - w.x_true[:, 0]).max() <= 1e-8
    g = val.grad.cpu().numpy()
    # the transposed solve: A^T lambda = x - x_target, checked by its residual
    lam = bb.grad.cpu().numpy()
    At = synth.csr_from_coo(A.n, A.col, np.repeat(np.arange(A.n), np.diff(A.row_ptr)), A.val)
    assert eta_of(At, xh - xt, lam) <= 1e-12
    rows = A.rows()
    np.testing.assert_allclose(g, -lam[rows] * xh[A.col], rtol=1e-12, atol=1e-300)
    rng = np.random.default_rng(w.extra["fd_seed"])
    picks = rng.choice(A.nnz, 64, replace=False)
    # forward-mode check on 64 entries: dx = A^{-1} (-x[col] e_row) by a plain
    # solve, dL = (x - x_target) . dx must equal the adjoint's entry
    for p in picks:
        e = np.zeros(A.n)
        e[rows[p]] = -xh[A.col[p]]
        dx = h.solve(dev(e)).cpu().numpy()
        dl = float(np.dot(xh - xt, dx))
        assert abs(dl - g[p]) <= 1e-9 * max(1.0, abs(g[p])), (p, dl, g[p])
    # central differences (h = 1e-6) on the first 16 of them, in the product
    # form; the allowance is the solver's measured error amplified by
    # ||x - x_target||_1 / h on top of the O(h^2) truncation
    hstep = 1e-6
    e_x = np.abs(xh - w.x_true[:, 0]).max() + 1e-15
    noise = 2.0 * np.abs(xh - xt).sum() * e_x / (2 * hstep)
    vb = dev(b)
    worst = 0.0
    with torch.no_grad():
        for p in picks[:16]:
            vp = A.val.copy(); vp[p] += hstep
            vm = A.val.copy(); vm[p] -= hstep
            xp = hylu.sparse_solve(h, dev(vp), vb).cpu().numpy()
            xm = hylu.sparse_solve(h, dev(vm), vb).cpu().numpy()
            fd = 0.5 * np.dot(xp - xm, xp + xm - 2 * xt) / (2 * hstep)
            worst = max(worst, abs(fd - g[p]) / max(1.0, abs(g[p])))
            assert abs(fd - g[p]) <= 1e-6 * max(1.0, abs(g[p])) + noise, (p, fd, g[p], noise)
    print(f"finite differences: worst relative difference {worst:.2e} (allowance {noise:.2e})")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_grid27_full_backward_error(hylu, precision):
    """27-point grid 64^3 (n = 262144), 8 right-hand sides, nested dissection
    with multilevel separators (as bench.py runs it): the normwise
    backward error of every right-hand side, at most 1e-12 for FP64 factors
    and for FP32 factors with FP64 refinement."""
    w = synth.convdiff3d_27pt(64)
    A = w.A
    print(f"[case] 27-point 64^3 full {precision}", flush=True)
    h = hylu.Handle(A.row_ptr, A.col, A.val, ordering="nd_ml", precision=precision, dense_tail=0.5)
    h.factorize(dev(A.val))
    X = h.solve_cols(dev(w.b.T.copy())).cpu().numpy().T
    for k in range(w.b.shape[1]):
        assert eta_of(A, w.b[:, k], X[:, k]) <= 1e-12, k
    print("ir iterations", h.info()["ir_iters"])


def test_batch_full_backward_error(hylu):
    """The 256-member uneven batch, refactorised with every member's fresh
    values: every member's backward error at most 1e-12 and its error against
    x_true at most 1e-9."""
    ws = [synth.batch_member(m) for m in range(256)]
    a0 = [w.extra["analyze_values"] for w in ws]
    print("[case] batch of 256 full", flush=True)
    hb = hylu.Handle.batch([(a.row_ptr, a.col, a.val) for a in a0])
    roff, _ = hb.offsets()
    hb.factorize(dev(np.concatenate([a.val for a in a0])))
    hb.refactor(dev(np.concatenate([w.A.val for w in ws])))
    x = hb.solve(dev(np.concatenate([w.b[:, 0] for w in ws]))).cpu().numpy()
    for k, w in enumerate(ws):
        xk = x[roff[k]:roff[k + 1]]
        assert eta_of(w.A, w.b[:, 0], xk) <= 1e-12, k
        assert np.abs(xk - w.x_true[:, 0]).max() <= 1e-9, k
