"""Symbolic factorisation and level sets on the GPU (option gpu_symbolic).

The analysis with the structure, supernodes and the four level sets computed
by the kernels must equal the host analysis to the bit: the hash of the
compressed structure and level sets, every exported array and every count.
The host analysis is itself checked against the oracle bit-exactly in the CPU
tests; one case here also goes to the oracle directly.
"""
import numpy as np
import pytest

import oracle
from paper_2509_07690_amd import synth

hylu = pytest.importorskip("paper_2509_07690_amd.hylu")
pytestmark = pytest.mark.gpu

KEYS = ("sym_hash", "flops", "flops_padded", "nnz_l", "nnz_u", "n_nodes", "n_supernodes", "n_levels",
        "factor_entries", "tail_rows")


def _same(hh, hg, label):
    a, b = hh.info(), hg.info()
    for k in KEYS:
        assert a[k] == b[k], (label, k, a[k], b[k])
    sa, sb = hh.symbolic(), hg.symbolic()
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), (label, k)
    print(f"{label}: host {a['sym_ms']:.1f} ms, GPU {b['sym_ms']:.1f} ms "
          f"(kernels {b['sym_kernel_ms']:.1f} ms), levels {b['n_levels']}", flush=True)
    return b


def _both(A, label, **opts):
    hh = hylu.Handle(A.row_ptr, A.col, A.val, **opts)
    hg = hylu.Handle(A.row_ptr, A.col, A.val, gpu_symbolic=1, **opts)
    _same(hh, hg, label)
    return hg


@pytest.mark.parametrize("seed", range(4))
def test_random_patterns(seed):
    rng = np.random.default_rng(seed)
    n = 300
    M = rng.random((n, n)) < 0.012
    np.fill_diagonal(M, True)
    A = synth.csr_from_dense(np.where(M, rng.standard_normal((n, n)), 0.0))
    _both(A, f"random {seed}")
    _both(A, f"random {seed} sn 3..8", sn_min=3, sn_max=8, ordering="nd")


def test_against_the_oracle():
    A = synth.config(0).A
    h = _both(A, "5-point 64^2")
    inf, sym = h.info(), h.symbolic()
    o = oracle.Oracle(A.n, A.row_ptr, A.col, A.val, sym["perm_r"], sym["perm_c"], sym["dr"], sym["dc"])
    o.analyse(2, 1 << 30)
    s = o.sizes()
    assert inf["flops"] == s["flops"] and inf["nnz_l"] == s["nnz_l"] and inf["nnz_u"] == s["nnz_u"]
    ptr, isn = o.partition_arrays()
    assert np.array_equal(ptr, sym["node_ptr"]) and np.array_equal(isn, sym["is_sn"])
    assert np.array_equal(o.level_arrays(), sym["levels"])


def test_row_kernel_only_and_small_supernodes():
    A = synth.config(0).A
    _both(A, "5-point rows only", kernel_mode=1)
    _both(A, "5-point sn 2..4", sn_max=4)


def test_circuits():
    _both(synth.circuit_powerlaw(20000).A, "circuit 20k")
    _both(synth.circuit_powerlaw(200000).A, "circuit 200k", dense_tail=0.15)


def test_grids():
    _both(synth.convdiff3d_27pt(24).A, "27-point 24^3", ordering="nd_ml")
    _both(synth.convdiff3d_7pt(32).A, "7-point 32^3", ordering="nd")


def test_batch_union():
    members = []
    for m in range(8):
        A = synth.batch_member(m).A
        members.append((A.row_ptr, A.col, A.val))
    hh = hylu.Handle.batch(members)
    hg = hylu.Handle.batch(members, gpu_symbolic=1)
    _same(hh, hg, "batch of 8")


def test_refactor_and_solve_after_gpu_analysis():
    w = synth.config(0)
    A = w.A
    import torch
    h = hylu.Handle(A.row_ptr, A.col, A.val, gpu_symbolic=1)
    dev = torch.device("cuda:0")
    bh = w.b[:, 0]
    h.factorize(torch.tensor(A.val, dtype=torch.float64, device=dev))
    x = h.solve(torch.tensor(bh, dtype=torch.float64, device=dev)).cpu().numpy()
    r = A.matvec(x) - bh
    norm_a = np.add.reduceat(np.abs(A.val), A.row_ptr[:-1]).max()
    eta = np.abs(r).max() / (norm_a * np.abs(x).max() + np.abs(bh).max())
    assert eta < 1e-15
