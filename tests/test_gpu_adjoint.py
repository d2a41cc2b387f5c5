"""Adjoint of x = A^{-1} b through the autograd Function (needs an MI355X).

Loss L = 0.5 ||x - x_target||^2 on a 3D 7-point nonsymmetric grid (the values
recipe of the 2D grid).  Checks: dL/dval and dL/db against the oracle's
gradient (oracle transposed solve + the pattern-restricted outer product), to
1e-10 normwise relative; dL/dval against central finite differences with
h = 1e-6 on random entries, each difference taken with the GPU solver itself;
a multi-RHS loss; and that a refactorisation with other values between
forward and backward does not change the gradient.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2509_07690_amd import synth  # noqa: E402
from parity import oracle_for, rel_diff  # noqa: E402


@pytest.fixture(scope="module")
def hylu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_07690_amd import hylu as H
    return H


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _loss_grad(hylu, h, A, b, xt):
    val = dev(A.val).requires_grad_()
    bb = dev(b).requires_grad_()
    x = hylu.sparse_solve(h, val, bb)
    loss = 0.5 * ((x - dev(xt)) ** 2).sum()
    loss.backward()
    return float(loss), x.detach().cpu().numpy(), val.grad.cpu().numpy(), bb.grad.cpu().numpy()


@pytest.mark.parametrize("side", [10, 16, 32])
def test_gradient_against_oracle_and_fd(hylu, side):
    w = synth.convdiff3d_7pt(side)
    A, b, xt = w.A, w.b[:, 0], w.extra["x_target"]
    print(f"[case] adjoint 7pt side={side} n={A.n}", flush=True)
    h = hylu.Handle(A.row_ptr, A.col, A.val, ordering="nd")
    loss, x, gval, gb = _loss_grad(hylu, h, A, b, xt)
    o, _ = oracle_for(h, A)
    o.numeric(o.tau)
    xo = o.solve(b)
    lam = o.solve_transposed(xo - xt)
    go = o.gradient_values(lam, xo)
    assert rel_diff(x, xo) <= 1e-10
    assert rel_diff(gb, lam) <= 1e-10
    assert rel_diff(gval, go) <= 1e-10
    # central differences with the GPU solver on 64 random entries.  The loss
    # difference is formed as 0.5 (x+ - x-).(x+ + x- - 2 x_target), which avoids
    # cancelling two losses of size ~n; what remains is the solver's own error
    # e_x (estimated by the distance to the oracle), amplified by
    # ||x - x_target||_1 / h, on top of the O(h^2) truncation.
    rng = np.random.default_rng(w.extra["fd_seed"])
    hstep = 1e-6
    e_x = np.abs(x - xo).max() + 1e-15 * np.abs(xo).max()
    noise = 2.0 * np.abs(x - xt).sum() * e_x / (2 * hstep)
    picks = rng.choice(A.nnz, 64, replace=False)
    vb = dev(b)
    worst = 0.0
    with torch.no_grad():
        for p in picks:
            vp = A.val.copy(); vp[p] += hstep
            vm = A.val.copy(); vm[p] -= hstep
            xp = hylu.sparse_solve(h, dev(vp), vb).cpu().numpy()
            xm = hylu.sparse_solve(h, dev(vm), vb).cpu().numpy()
            fd = 0.5 * np.dot(xp - xm, xp + xm - 2 * xt) / (2 * hstep)
            err = abs(fd - gval[p])
            worst = max(worst, err / max(1.0, abs(gval[p])))
            assert err <= 1e-6 * max(1.0, abs(gval[p])) + noise, (p, fd, gval[p], noise)
    print(f"fd: worst relative difference {worst:.2e}, solver-noise allowance {noise:.2e}")


def test_gradient_multi_rhs_and_refactor_between(hylu):
    w = synth.convdiff3d_7pt(10)
    A = w.A
    h = hylu.Handle(A.row_ptr, A.col, A.val, ordering="nd")
    rng = np.random.default_rng(7)
    B = rng.uniform(-1, 1, (A.n, 3))
    T = rng.uniform(-1, 1, (A.n, 3))
    val = dev(A.val).requires_grad_()
    bb = dev(B).requires_grad_()
    X = hylu.sparse_solve(h, val, bb)
    # another value set factorised before backward
    other = synth.grid_values(A, 99, 4.0)
    h.refactor(dev(other.val))
    loss = 0.5 * ((X - dev(T)) ** 2).sum()
    loss.backward()
    o, _ = oracle_for(h, A)
    o.numeric(o.tau, piv=hylu.factors_as_rows(h)[2])   # pivots of the first factorisation
    g = np.zeros(A.nnz)
    for k in range(3):
        xk = o.solve(B[:, k])
        lk = o.solve_transposed(xk - T[:, k])
        g += o.gradient_values(lk, xk)
        assert rel_diff(bb.grad[:, k].cpu().numpy(), lk) <= 1e-10
    assert rel_diff(val.grad.cpu().numpy(), g) <= 1e-10
