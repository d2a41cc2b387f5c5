"""Batched refactorisation of uneven matrices on one handle (needs an MI355X).

Eight members of the uneven batch (four local circuits, four 9-point grids)
analysed together; the factors of the whole block-diagonal union are compared
entry by entry with the oracle on the same permutations and scalings; every
member's solution is compared with the oracle's and its own backward error is
checked (FP64: 1e-12; FP32 factors + FP64 refinement: 1e-10 and at most one
order of magnitude from FP64).  The autotuner must leave bit-identical
factors, and a fresh value set refactorised through the tuned graph matches
the oracle.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2509_07690_amd import synth  # noqa: E402
from parity import checked_tau, compare_factors, rel_diff  # noqa: E402
import oracle  # noqa: E402

MEMBERS = range(8)


@pytest.fixture(scope="module")
def hylu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_07690_amd import hylu as H
    return H


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


@pytest.fixture(scope="module")
def batch():
    ws = [synth.batch_member(m) for m in MEMBERS]
    a0 = [w.extra["analyze_values"] for w in ws]
    return ws, a0


def _union(hb, vals):
    return synth.Csr(hb.n, hb.row_ptr, hb.col, np.concatenate(vals))


def _oracle(hb, U):
    """The oracle on the union with the analysed values U; o.tau from its own
    B, checked against the library's threshold."""
    sym = hb.symbolic()
    o = oracle.Oracle(U.n, U.row_ptr, U.col, U.val, sym["perm_r"], sym["perm_c"], sym["dr"], sym["dc"])
    o.analyse()
    o.tau = checked_tau(hb, o)
    return o


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_factor_and_solve(hylu, batch, precision):
    ws, a0 = batch
    print(f"[case] batch of {len(ws)} precision={precision}", flush=True)
    hb = hylu.Handle.batch([(a.row_ptr, a.col, a.val) for a in a0], precision=precision)
    roff, qoff = hb.offsets()
    U0 = _union(hb, [a.val for a in a0])
    hb.factorize(dev(U0.val))
    torch.cuda.synchronize()
    o = _oracle(hb, U0)
    tau = o.tau
    o.numeric(tau)
    if precision == "fp64":
        compare_factors(hb, o)
    # the fresh value set of every member, refactorised, then one RHS each
    U1 = _union(hb, [w.A.val for w in ws])
    piv = hylu.factors_as_rows(hb)[2]
    hb.refactor(dev(U1.val))
    torch.cuda.synchronize()
    o.set_values(U1.val)
    o.numeric(tau, piv=piv)
    if precision == "fp64":
        compare_factors(hb, o)
    b = np.concatenate([w.b[:, 0] for w in ws])
    x = hb.solve(dev(b)).cpu().numpy()
    xo = o.solve(b)
    for k, w in enumerate(ws):
        sl = slice(roff[k], roff[k + 1])
        ok = oracle.Oracle(w.A.n, w.A.row_ptr, w.A.col, w.A.val, *[np.arange(w.A.n, dtype=np.int32)] * 2,
                           np.ones(w.A.n), np.ones(w.A.n))
        eta, _ = ok.backward_error(w.b[:, 0], x[sl])
        assert eta <= (1e-12 if precision == "fp64" else 1e-10), (k, eta)
        assert rel_diff(x[sl], xo[sl]) <= (1e-10 if precision == "fp64" else 1e-9), k
    print("ir iterations", hb.info()["ir_iters"], "berr", hb.info()["berr"])


def test_autotune_keeps_factors(hylu, batch):
    ws, a0 = batch
    hb = hylu.Handle.batch([(a.row_ptr, a.col, a.val) for a in a0])
    U0 = _union(hb, [a.val for a in a0])
    v0 = dev(U0.val)
    hb.factorize(v0)
    hb.refactor(v0)
    torch.cuda.synchronize()
    before = hb.factors_raw()["vals"]
    t_def, t_tuned = hb.autotune(v0, reps=2)
    print(f"autotune: built-in shapes {t_def:.3f} ms, tuned {t_tuned:.3f} ms")
    assert t_tuned <= t_def + 1e-9
    after = hb.factors_raw()["vals"]
    assert np.array_equal(before, after)
    hb.refactor(v0)                    # through a graph captured with the tuned shapes
    torch.cuda.synchronize()
    assert np.array_equal(before, hb.factors_raw()["vals"])
    U1 = _union(hb, [w.A.val for w in ws])
    piv = hylu.factors_as_rows(hb)[2]
    hb.refactor(dev(U1.val))
    torch.cuda.synchronize()
    o = _oracle(hb, U0)
    o.set_values(U1.val)
    o.numeric(o.tau, piv=piv)
    compare_factors(hb, o)


def test_batch_pipelined(hylu, batch):
    """Pipeline mode on the batch (Sec. 2.2.1): every level from the first one
    after which all levels have at most 1024 rows runs in chain launches, the
    members' nodes waiting per source: factors of the union entry by entry
    against the oracle after factorisation and after a refactorisation with
    every member's fresh values, and every member's solution and backward
    error."""
    ws, a0 = batch
    print(f"[case] batch of {len(ws)} pipelined", flush=True)
    hb = hylu.Handle.batch([(a.row_ptr, a.col, a.val) for a in a0], pipeline_rows=1 << 30)
    assert hb.info()["pipe_tasks"] > 0
    roff, _ = hb.offsets()
    U0 = _union(hb, [a.val for a in a0])
    hb.factorize(dev(U0.val))
    torch.cuda.synchronize()
    o = _oracle(hb, U0)
    o.numeric(o.tau)
    compare_factors(hb, o)
    U1 = _union(hb, [w.A.val for w in ws])
    piv = hylu.factors_as_rows(hb)[2]
    hb.refactor(dev(U1.val))
    torch.cuda.synchronize()
    o.set_values(U1.val)
    o.numeric(o.tau, piv=piv)
    compare_factors(hb, o)
    x = hb.solve(dev(np.concatenate([w.b[:, 0] for w in ws]))).cpu().numpy()
    for k, w in enumerate(ws):
        xk = x[roff[k]:roff[k + 1]]
        e, _ = o.backward_error(np.concatenate([v.b[:, 0] for v in ws]), x) if k == 0 else (0.0, 0.0)
        assert e <= 1e-12
        assert np.abs(xk - w.x_true[:, 0]).max() <= 1e-9, k


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_batch_solve_launch_packing(hylu, batch, precision):
    """The batch's solves with the large supernodes of a level launched
    together (their gathers in one launch, then each panel step of all of
    them in one launch) and the long supernodes split over workgroups
    (solve_split, default) against one launch sequence per supernode and one
    workgroup per supernode: the same factors and, for one and for three
    right-hand sides, the same solutions to the bit."""
    ws, a0 = batch
    print(f"[case] batch of {len(ws)} solve launch packing, {precision}", flush=True)
    U1 = None
    out = []
    for split in (1, 0):
        hb = hylu.Handle.batch([(a.row_ptr, a.col, a.val) for a in a0], precision=precision, solve_split=split)
        assert (hb.info()["split_sn"] > 0) == (split == 1)
        U1 = _union(hb, [w.A.val for w in ws])
        hb.factorize(dev(U1.val))
        b = np.concatenate([w.b[:, 0] for w in ws])
        B = np.stack([b, 2.0 * b - 1.0, np.sin(np.arange(hb.n))], axis=1)
        x1 = hb.solve(dev(b)).cpu().numpy()
        x3 = hb.solve(dev(B)).cpu().numpy()
        out.append((hb.factors_raw()["vals"], x1, x3))
        hb.close()
    assert np.array_equal(out[0][0], out[1][0])
    assert np.array_equal(out[0][1], out[1][1]) and np.array_equal(out[0][2], out[1][2])
