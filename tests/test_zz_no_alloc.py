"""hylu_solve_noalloc, the solve for callers that cannot allocate, against
hylu_solve (needs an MI355X).  Both run the same kernels in the same order on
the same factors, so the solutions must agree to the bit: two calls in a row
on one GPU's shared scratch, the second with a smaller problem (FP32 factors
with FP64 refinement), a transposed solve, and a problem beyond the scratch
rejected on the host."""
import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2509_07690_amd import synth  # noqa: E402


@pytest.fixture(scope="module")
def hylu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2509_07690_amd import hylu as H
    return H


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def noalloc(hylu, h, bt, xt, transpose=0):
    """hylu_solve_noalloc through the C ABI: bt, xt (k, n) column-major RHS."""
    k = 1 if bt.dim() == 1 else bt.shape[0]
    s = torch.cuda.current_stream().cuda_stream
    return hylu._lib.hylu_solve_noalloc(h.h, C.c_void_p(bt.data_ptr()), C.c_void_p(xt.data_ptr()), k, h.n,
                                        transpose, C.c_void_p(s))


def test_noalloc_matches_solve(hylu):
    rng = np.random.default_rng(21)
    # call 1: 2D grid n = 4096, four right-hand sides, FP64 factors
    w1 = synth.convdiff2d(side=64)
    A1 = w1.A
    print(f"[case] noalloc n={A1.n} nrhs=4 fp64", flush=True)
    h1 = hylu.Handle(A1.row_ptr, A1.col, A1.val)
    h1.factorize(dev(A1.val))
    B1 = dev(rng.uniform(-1, 1, (4, A1.n)))
    ref1 = h1.solve_cols(B1)
    X1 = torch.full_like(B1, np.nan)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    assert noalloc(hylu, h1, B1, X1) == 0
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    assert torch.equal(X1, ref1)
    # call 2 right after, smaller: a 32 x 32 grid with FP32 factors (refinement runs)
    w2 = synth.convdiff2d(side=32)
    A2 = w2.A
    print(f"[case] noalloc n={A2.n} nrhs=1 fp32", flush=True)
    h2 = hylu.Handle(A2.row_ptr, A2.col, A2.val, precision="fp32")
    h2.factorize(dev(A2.val))
    b2 = dev(w2.b[:, 0])
    ref2 = h2.solve(b2)
    it_ref = h2.info()["ir_iters"]
    x2 = torch.full_like(b2, np.nan)
    assert noalloc(hylu, h2, b2, x2) == 0
    torch.cuda.synchronize()
    assert h2.info()["ir_iters"] == it_ref >= 1
    assert torch.equal(x2, ref2)
    assert float((x2.cpu() - torch.from_numpy(w2.x_true[:, 0])).abs().max()) <= 1e-10
    # in place (x = b) with refinement
    x3 = b2.clone()
    assert noalloc(hylu, h2, x3, x3) == 0
    assert torch.equal(x3, ref2)
    # transposed, once the handle has its transposed tables
    rt = h1.solve_cols(B1[:2].contiguous(), transpose=True)
    Xt = torch.empty_like(rt)
    assert noalloc(hylu, h1, B1[:2].contiguous(), Xt, transpose=1) == 0
    assert torch.equal(Xt, rt)
    # beyond the scratch: rejected before any launch
    big = torch.zeros((65, A2.n), dtype=torch.float64, device="cuda")
    assert noalloc(hylu, h2, big, big.clone()) == -10
    torch.cuda.synchronize()
    h1.close()
    h2.close()
