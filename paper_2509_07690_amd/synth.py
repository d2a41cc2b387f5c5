"""Seeded synthetic inputs shaped like the workloads HYLU targets.

The paper evaluates on SuiteSparse matrices from circuit simulation, power
networks and PDE discretisations (Sec. 1, Sec. 3, Table I).  None of those
matrices is available here, so every workload is generated from a seed:

* 2D / 3D stencil grids (5-, 9-, 7- and 27-point), nonsymmetric values;
* circuit-like patterns: a power-law column degree with local (Cauchy
  distributed) placement plus uniformly placed hub columns, made diagonally
  dominant, and a local per-row variant for the batched workload.

This module holds no arithmetic of the factorisation method; it only draws
patterns and values and forms right-hand sides b = A x_true.  Both the HIP
path and the CPU oracle are fed from here.

All matrices are returned as CSR with int64 row pointers, int32 column
indices (sorted, unique within a row) and float64 values.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np


@dataclass
class Csr:
    n: int
    row_ptr: np.ndarray  # int64 [n+1]
    col: np.ndarray      # int32 [nnz]
    val: np.ndarray      # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def rows(self) -> np.ndarray:
        """Row index of every stored entry (int64 [nnz])."""
        return np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.row_ptr))

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """y = A x in float64 (x may be [n] or [n, k])."""
        x = np.asarray(x, dtype=np.float64)
        r = self.rows()
        if x.ndim == 1:
            return np.bincount(r, weights=self.val * x[self.col], minlength=self.n)
        out = np.empty((self.n, x.shape[1]), dtype=np.float64)
        for c in range(x.shape[1]):
            out[:, c] = np.bincount(r, weights=self.val * x[self.col, c], minlength=self.n)
        return out

    def diag_positions(self) -> np.ndarray:
        """CSR position of the diagonal entry of every row (-1 if absent)."""
        r = self.rows()
        pos = np.full(self.n, -1, dtype=np.int64)
        hit = np.nonzero(self.col.astype(np.int64) == r)[0]
        pos[r[hit]] = hit
        return pos

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        d[self.rows(), self.col] = self.val
        return d


def csr_from_coo(n: int, rows: np.ndarray, cols: np.ndarray,
                 vals: Optional[np.ndarray] = None) -> Csr:
    """Sort (row, col) pairs, merge duplicates (values summed) and build CSR."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    key = rows * n + cols
    order = np.argsort(key, kind="stable")
    key = key[order]
    uniq, start = np.unique(key, return_index=True)
    if vals is None:
        v = np.zeros(uniq.size)
    else:
        v = np.add.reduceat(np.asarray(vals, dtype=np.float64)[order], start) if uniq.size else np.zeros(0)
    r = uniq // n
    c = uniq % n
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return Csr(n, row_ptr, c.astype(np.int32), v)


def csr_from_dense(d: np.ndarray) -> Csr:
    """CSR of the nonzero entries of a dense square matrix (diagonal always kept)."""
    d = np.asarray(d, dtype=np.float64)
    n = d.shape[0]
    mask = d != 0
    mask[np.arange(n), np.arange(n)] = True
    r, c = np.nonzero(mask)
    return csr_from_coo(n, r, c, d[r, c])


# ----------------------------------------------------------------------------
# stencil grids
# ----------------------------------------------------------------------------

def _stencil_pattern(dims: tuple, offsets: list) -> Csr:
    """Pattern of a stencil on a box grid; node id = x + dims[0]*(y + dims[1]*z)."""
    dims = tuple(int(d) for d in dims)
    nd = len(dims)
    n = int(np.prod(dims))
    strides = [1]
    for d in dims[:-1]:
        strides.append(strides[-1] * d)
    # sort offsets by linear offset so columns come out sorted per row
    offs = sorted(offsets, key=lambda o: sum(o[a] * strides[a] for a in range(nd)))
    idx = np.arange(n, dtype=np.int64)
    coord = []
    rem = idx.copy()
    for a in range(nd):
        coord.append(rem % dims[a])
        rem //= dims[a]
    cols = np.empty((n, len(offs)), dtype=np.int64)
    for t, o in enumerate(offs):
        ok = np.ones(n, dtype=bool)
        lin = np.zeros(n, dtype=np.int64)
        for a in range(nd):
            c = coord[a] + o[a]
            ok &= (c >= 0) & (c < dims[a])
            lin += o[a] * strides[a]
        cols[:, t] = np.where(ok, idx + lin, -1)
    valid = cols >= 0
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    row_ptr[1:] = np.cumsum(counts)
    col = cols[valid].astype(np.int32)  # row-major flatten keeps per-row order
    return Csr(n, row_ptr, col, np.zeros(col.size))


def _offsets(nd: int, kind: str) -> list:
    if kind == "star":  # 5-pt (2D) / 7-pt (3D)
        offs = [tuple([0] * nd)]
        for a in range(nd):
            for s in (-1, 1):
                o = [0] * nd
                o[a] = s
                offs.append(tuple(o))
        return offs
    if kind == "box":  # 9-pt (2D) / 27-pt (3D)
        import itertools
        return [tuple(o) for o in itertools.product((-1, 0, 1), repeat=nd)]
    raise ValueError(kind)


def grid_values(pat: Csr, seed: int, diag_base: float) -> Csr:
    """Nonsymmetric grid values: off-diagonals -1+U[-0.3,0.3] drawn independently
    per entry, diagonal diag_base+U[0,1] (the convection-diffusion recipe)."""
    rng = np.random.default_rng(seed)
    v = rng.uniform(-1.3, -0.7, pat.nnz)
    dpos = pat.diag_positions()
    v[dpos] = diag_base + rng.uniform(0.0, 1.0, pat.n)
    return Csr(pat.n, pat.row_ptr, pat.col, v)


def grid2d(side: int, points: int) -> Csr:
    return _stencil_pattern((side, side), _offsets(2, "star" if points == 5 else "box"))


def grid3d(side: int, points: int) -> Csr:
    return _stencil_pattern((side, side, side), _offsets(3, "star" if points == 7 else "box"))


def grid_nnz_closed_form(dim: int, points: int, side: int) -> int:
    """Stored entries of the stencil matrix (diagonal included)."""
    k = side
    if dim == 2 and points == 5:
        return 5 * k * k - 4 * k
    if dim == 2 and points == 9:
        return (3 * k - 2) ** 2
    if dim == 3 and points == 7:
        return 7 * k ** 3 - 6 * k ** 2
    if dim == 3 and points == 27:
        return (3 * k - 2) ** 3
    raise ValueError((dim, points))


# ----------------------------------------------------------------------------
# circuit-like patterns
# ----------------------------------------------------------------------------

def dominant_values(pat: Csr, seed: int, factor: float = 1.5) -> Csr:
    """Off-diagonals ~ N(0,1); a_ii = factor * sum_{j != i} |a_ij| (factor if the
    row has no off-diagonal).  Every row is strictly diagonally dominant."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(pat.nnz)
    dpos = pat.diag_positions()
    r = pat.rows()
    off = np.abs(v)
    off[dpos] = 0.0
    s = np.bincount(r, weights=off, minlength=pat.n)
    v[dpos] = np.where(s > 0, factor * s, factor)
    return Csr(pat.n, pat.row_ptr, pat.col, v)


# Rescale of the power-law degree draw that brings the mean to 5.0 stored
# entries per row (diagonal included) after self-loops and duplicates are
# removed, for n = 200000 and seed 100 (found by bisection on that seed).
POWERLAW_RESCALE = 1.2421


def circuit_powerlaw_pattern(n: int, seed: int, exponent: float = 2.1, kmax: int = 2000,
                             rescale: float = POWERLAW_RESCALE, hub_min: int = 51,
                             cauchy_scale: float = 3.0) -> Csr:
    """Circuit-like nonsymmetric pattern with power-law column degree.

    Column j draws a degree k_j from P(k) ~ k^-exponent on [1, kmax], rescaled
    by `rescale` with stochastic rounding.  A column of degree < hub_min puts
    its entries near the diagonal (row j + round(cauchy_scale * Cauchy),
    clipped); a hub column (a supply or ground net) puts them uniformly.
    Self-loops and duplicates are dropped and the diagonal is always present.
    """
    rng = np.random.default_rng(seed)
    ks = np.arange(1, kmax + 1, dtype=np.float64)
    p = ks ** (-exponent)
    p /= p.sum()
    k = rng.choice(np.arange(1, kmax + 1), size=n, p=p).astype(np.float64)
    d = np.floor(rescale * k + rng.uniform(0.0, 1.0, n)).astype(np.int64)
    d = np.clip(d, 0, kmax)
    colj = np.repeat(np.arange(n, dtype=np.int64), d)
    hub = np.repeat(d >= hub_min, d)
    local = colj + np.rint(cauchy_scale * rng.standard_cauchy(colj.size)).astype(np.int64)
    local = np.clip(local, 0, n - 1)
    uni = rng.integers(0, n, colj.size)
    rowi = np.where(hub, uni, local)
    keep = rowi != colj
    rows = np.concatenate([rowi[keep], np.arange(n)])
    cols = np.concatenate([colj[keep], np.arange(n)])
    return csr_from_coo(n, rows, cols)


def circuit_local_pattern(n: int, seed: int, lo: int = 3, hi: int = 7,
                          cauchy_scale: float = 3.0) -> Csr:
    """Per row U{lo..hi} off-diagonals at column i + round(cauchy_scale*Cauchy)."""
    rng = np.random.default_rng(seed)
    d = rng.integers(lo, hi + 1, n)
    rowi = np.repeat(np.arange(n, dtype=np.int64), d)
    colj = rowi + np.rint(cauchy_scale * rng.standard_cauchy(rowi.size)).astype(np.int64)
    colj = np.clip(colj, 0, n - 1)
    keep = rowi != colj
    rows = np.concatenate([rowi[keep], np.arange(n)])
    cols = np.concatenate([colj[keep], np.arange(n)])
    return csr_from_coo(n, rows, cols)


def uniform_random_pattern(n: int, seed: int, per_row: int) -> Csr:
    rng = np.random.default_rng(seed)
    rowi = np.repeat(np.arange(n, dtype=np.int64), per_row)
    colj = rng.integers(0, n, rowi.size)
    rows = np.concatenate([rowi, np.arange(n)])
    cols = np.concatenate([colj, np.arange(n)])
    return csr_from_coo(n, rows, cols)


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    A: Csr
    b: np.ndarray              # [n, nrhs] float64, column-major when flattened with order="F"
    x_true: Optional[np.ndarray]
    ordering: str              # "amd" | "nd" | "natural"
    revalue: Optional[Callable[[int], "Workload"]] = None
    extra: dict = field(default_factory=dict)


def _rhs_from_x(A: Csr, seed: int, nrhs: int = 1):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, (A.n, nrhs))
    return A.matvec(x), x


def convdiff2d(side: int = 64, seed: int = 0, rhs_seed: int = 1) -> Workload:
    """5-point nonsymmetric convection-diffusion on a side x side grid,
    diagonal 4+U[0,1], off-diagonals -1+U[-0.3,0.3]; b = A x_true."""
    A = grid_values(grid2d(side, 5), seed, 4.0)
    b, x = _rhs_from_x(A, rhs_seed)
    return Workload(f"convdiff2d_5pt_{side}x{side}", A, b, x, "amd")


def circuit_powerlaw(n: int = 200000, seed: int = 100, refactor: int = 0) -> Workload:
    """Circuit-like matrix: power-law column degree, |a_ii| = 1.5 sum |a_ij|,
    N(0,1) off-diagonals.  Refactor r redraws values with seed 1100+r and
    x_true with seed 2100+r on the same pattern."""
    pat = circuit_powerlaw_pattern(n, seed)
    return _circuit_values(pat, refactor, f"circuit_powerlaw_n{n}")


def _circuit_values(pat: Csr, r: int, name: str) -> Workload:
    A = dominant_values(pat, 1100 + r)
    b, x = _rhs_from_x(A, 2100 + r)
    w = Workload(name, A, b, x, "amd")
    w.revalue = lambda rr: _circuit_values(pat, rr, name)
    w.extra["refactor"] = r
    return w


def convdiff3d_27pt(side: int = 64, seed: int = 200, rhs_seed: int = 201, nrhs: int = 8,
                    diag_base: float = 26.0) -> Workload:
    """27-point nonsymmetric convection-diffusion on side^3, diagonal
    diag_base+U[0,1]; nrhs right-hand sides with entries U[-1,1]."""
    A = grid_values(grid3d(side, 27), seed, diag_base)
    rng = np.random.default_rng(rhs_seed)
    b = rng.uniform(-1.0, 1.0, (A.n, nrhs))
    return Workload(f"convdiff3d_27pt_{side}^3", A, b, None, "nd")


def convdiff3d_7pt(side: int = 48, seed: int = 400, rhs_seed: int = 401,
                   diag_base: float = 4.0) -> Workload:
    """7-point nonsymmetric grid on side^3 with the 2D recipe's values
    (diagonal diag_base+U[0,1]); b = A x_true; x_target ~ U[-1,1] (seed+2)."""
    A = grid_values(grid3d(side, 7), seed, diag_base)
    b, x = _rhs_from_x(A, rhs_seed)
    w = Workload(f"grid3d_7pt_{side}^3", A, b, x, "nd")
    w.extra["x_target"] = np.random.default_rng(seed + 2).uniform(-1.0, 1.0, A.n)
    w.extra["fd_seed"] = seed + 3
    return w


def batch_member(m: int, refactor_values: bool = True) -> Workload:
    """Member m of the 256-matrix uneven batch.  Even m: local circuit with
    n ~ U{2000..50000}; odd m: 9-point grid with side ~ U{32..160}.  The pattern
    and analysis values use seed 3000+m, the fresh value set seed 3500+m."""
    rng = np.random.default_rng(3000 + m)
    if m % 2 == 0:
        n = int(rng.integers(2000, 50001))
        pat = circuit_local_pattern(n, 3000 + m)
        A0 = dominant_values(pat, 3000 + m)
        A1 = dominant_values(pat, 3500 + m)
        name = f"batch{m}_circuit_n{n}"
    else:
        s = int(rng.integers(32, 161))
        pat = grid2d(s, 9)
        A0 = grid_values(pat, 3000 + m, 8.0)
        A1 = grid_values(pat, 3500 + m, 8.0)
        name = f"batch{m}_grid9_{s}x{s}"
    A = A1 if refactor_values else A0
    b, x = _rhs_from_x(A, 3500 + m + 100000)
    w = Workload(name, A, b, x, "amd")
    w.extra["analyze_values"] = A0
    return w


def config(k: int, scale: Optional[int] = None) -> Workload:
    """The five workloads: 0 small 2D grid, 1 circuit, 2 27-pt 3D grid,
    3 batch member 0, 4 7-pt 3D grid (adjoint).  `scale` shrinks the grid
    side or n for quick runs."""
    if k == 0:
        return convdiff2d(scale or 64)
    if k == 1:
        return circuit_powerlaw(scale or 200000)
    if k == 2:
        return convdiff3d_27pt(scale or 64)
    if k == 3:
        return batch_member(scale or 0)
    if k == 4:
        return convdiff3d_7pt(scale or 48)
    raise ValueError(k)
