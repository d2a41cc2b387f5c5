"""Boundary behaviour of the C ABI that the parity tests do not cover (needs
an MI355X): the accuracy measures of hylu_residual against the oracle's own
evaluation, refinement that stops above its target returning its best
iterate, and device memory taken from PyTorch's caching allocator."""
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


def test_residual_measures_match_the_oracle(hylu):
    """Backward error and ||Ax-b||_1/||b||_1 (Sec. 3.3) of a perturbed
    solution, by the library (FP64 residual on the device) and by the oracle
    (compensated sums on the host), for A and for A^T."""
    w = synth.convdiff2d(side=32)
    A = w.A
    print(f"[case] residual measures n={A.n}", flush=True)
    h = hylu.Handle(A.row_ptr, A.col, A.val)
    h.factorize(dev(A.val))
    o, _ = oracle_for(h, A)
    rng = np.random.default_rng(5)
    B = rng.uniform(-1, 1, (2, A.n))
    for transpose in (False, True):
        X = h.solve_cols(dev(B), transpose=transpose).cpu().numpy()
        X += 1e-4 * rng.standard_normal(X.shape)          # a residual far above the rounding of its sums
        eta, r1 = h.residual(dev(B), dev(X), transpose=transpose)
        At = None
        if transpose:
            import scipy.sparse as sp
            At = sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n)).T.tocsr()
            At.sort_indices()
        worst_eta, worst_r1 = 0.0, 0.0
        for k in range(2):
            if not transpose:
                e, q = o.backward_error(B[k], X[k])
            else:
                ot = _oracle_of(At)
                e, q = ot.backward_error(B[k], X[k])
            worst_eta, worst_r1 = max(worst_eta, e), max(worst_r1, q)
        assert abs(eta - worst_eta) <= 1e-8 * worst_eta, (eta, worst_eta)
        assert abs(r1 - worst_r1) <= 1e-8 * worst_r1, (r1, worst_r1)
        inf = h.info()
        assert inf["berr"] == eta and inf["resid_1"] == r1


def _oracle_of(M):
    """An oracle holding M itself (identity permutations and scalings): its
    backward_error evaluates M's residual measures."""
    import oracle
    n = M.shape[0]
    ident = np.arange(n, dtype=np.int32)
    return oracle.Oracle(n, M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data, ident, ident,
                         np.ones(n), np.ones(n))


def test_refinement_keeps_its_best_iterate(hylu):
    """FP32 factors with an unreachable refinement target: refinement stops
    on stagnation and warns; the returned x is the iterate whose backward
    error the library reports (the library's own residual of the returned x
    gives that value to the bit), that value is at the rounding level, the
    oracle's compensated evaluation agrees to within the rounding of the
    residual sums, and x matches the oracle's solution."""
    w = synth.convdiff2d(side=48)
    A = w.A
    print(f"[case] refinement stagnation n={A.n}", flush=True)
    h = hylu.Handle(A.row_ptr, A.col, A.val, precision="fp32", ir_tol=1e-300, ir_maxit=30)
    h.factorize(dev(A.val))
    b = w.b[:, 0]
    bd = dev(b)
    with pytest.warns(hylu.RefinementWarning):
        xd = h.solve(bd)
    inf = h.info()
    assert h.last_status == hylu.WARN_IR_NOT_CONVERGED
    assert 1 <= inf["ir_iters"] < 30
    eta_again, _ = h.residual(bd, xd)
    assert eta_again == inf["berr"], (eta_again, inf["berr"])
    x = xd.cpu().numpy()
    o, _ = oracle_for(h, A)
    e, q = o.backward_error(b, x)
    assert e <= 1e-15 and inf["berr"] <= 1e-15, (e, inf["berr"])
    assert abs(inf["berr"] - e) <= 0.5 * e, (inf["berr"], e)
    o.numeric(o.tau)
    assert rel_diff(x, o.solve(b)) <= 1e-10


def test_device_memory_comes_from_torch(hylu):
    """The handle's device buffers are allocations of PyTorch's caching
    allocator: they show in torch.cuda.memory_allocated while the handle
    lives and are returned when it is closed."""
    w = synth.convdiff2d(side=64)
    A = w.A
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    h = hylu.Handle(A.row_ptr, A.col, A.val)
    v = dev(A.val)
    h.factorize(v)
    x = h.solve(dev(w.b[:, 0]))
    torch.cuda.synchronize()
    held = torch.cuda.memory_allocated() - before
    assert held >= 8 * h.info()["factor_entries"], (held, h.info()["factor_entries"])
    assert rel_diff(x.cpu().numpy(), w.x_true[:, 0]) <= 1e-10
    h.close()
    del v, x
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() <= before
