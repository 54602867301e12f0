"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only *builds inputs*: it holds none of the arithmetic of the
sparse products, indexing or assignment that the library and the oracle
compute.  Every matrix comes out in canonical 0-based CSC on the host:

* ``cp``  int64[n+1]  column pointers,
* ``ir``  int32[nnz]  row indices, strictly increasing inside each column,
* ``num`` values (float64 / float32 / int64) or ``None`` for a pattern.

Generators (all seeded, all deterministic):

* :func:`erdos_renyi` -- exactly ``d`` distinct uniform rows per column
  (the flat random matrix of the paper's experimental section).
* :func:`rmat` -- the recursive-matrix generator with quadrant
  probabilities (a, b, c, d), duplicates merged, vertices relabelled by a
  random symmetric permutation, values drawn after de-duplication in
  sorted (column, row) order (experimental section of the paper: R-MAT
  inputs with a random symmetric permutation applied to them).
* :func:`laplacian7` / :func:`aggregation` -- 7-point Dirichlet Laplacian on
  an n^3 grid and the 2x2x2 piecewise-constant aggregation operator.
* :func:`index_vector` -- an unsorted index vector with a fraction of
  repeated entries.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

# R-MAT quadrant probabilities used by the workloads (a, b, c; d = 1-a-b-c).
RMAT_GRAPH500 = (0.57, 0.19, 0.19)
# The probabilities the paper itself used for its R-MAT inputs.
RMAT_PAPER = (0.6, 0.4 / 3, 0.4 / 3)


@dataclasses.dataclass
class HostCsc:
    """Canonical 0-based CSC matrix on the host."""

    m: int
    n: int
    cp: np.ndarray  # int64[n+1]
    ir: np.ndarray  # int32[nnz]
    num: Optional[np.ndarray]  # [nnz] or None (pattern only)

    @property
    def nnz(self) -> int:
        return int(self.cp[-1])

    def with_values(self, num: Optional[np.ndarray]) -> "HostCsc":
        return HostCsc(self.m, self.n, self.cp, self.ir, num)

    def col(self, j: int):
        s, e = int(self.cp[j]), int(self.cp[j + 1])
        return self.ir[s:e], (None if self.num is None else self.num[s:e])

    def to_dense(self, fill=0):
        """Dense copy (tiny inputs only)."""
        dt = np.float64 if self.num is None else self.num.dtype
        out = np.full((self.m, self.n), fill, dtype=dt)
        for j in range(self.n):
            r, v = self.col(j)
            out[r, j] = 1 if v is None else v
        return out


def csc_from_sorted_keys(keys: np.ndarray, m: int, n: int, num=None) -> HostCsc:
    """Build CSC from unique keys ``col * m + row`` already sorted ascending."""
    cols = keys // m
    rows = (keys - cols * m).astype(np.int32)
    counts = np.bincount(cols, minlength=n).astype(np.int64)
    cp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=cp[1:])
    return HostCsc(m, n, cp, rows, num)


def from_triples(rows, cols, vals, m: int, n: int) -> HostCsc:
    """Canonical CSC from coordinate lists with *distinct* (row, col) pairs.

    Raises ``ValueError`` on a repeated coordinate: callers that want
    duplicates merged must do so explicitly before calling.
    """
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    if rows.size and (rows.min() < 0 or rows.max() >= m or cols.min() < 0 or cols.max() >= n):
        raise ValueError("coordinate out of range")
    keys = cols * m + rows
    order = np.argsort(keys, kind="stable")
    keys = keys[order]
    if keys.size > 1 and np.any(keys[1:] == keys[:-1]):
        raise ValueError("repeated coordinate")
    num = None if vals is None else np.asarray(vals)[order]
    return csc_from_sorted_keys(keys, m, n, num)


def _distinct_rows_per_column(rng, m: int, n: int, d: int) -> np.ndarray:
    if d > m:
        raise ValueError("d exceeds the number of rows")
    if d * d > 2 * m:  # a column of d uniform draws would most likely repeat a row
        return np.stack([np.sort(rng.choice(m, size=d, replace=False)) for _ in range(n)]) if n else \
            np.zeros((0, d), dtype=np.int64)
    rows = rng.integers(0, m, size=(n, d), dtype=np.int64)
    rows.sort(axis=1)
    tries = 0
    while d > 1:
        bad = np.nonzero(np.any(rows[:, 1:] == rows[:, :-1], axis=1))[0]
        if bad.size == 0:
            break
        tries += 1
        if tries > 50:  # dense columns (d close to m): draw those without replacement
            for j in bad:
                rows[j] = np.sort(rng.choice(m, size=d, replace=False))
            break
        fresh = rng.integers(0, m, size=(bad.size, d), dtype=np.int64)
        fresh.sort(axis=1)
        rows[bad] = fresh
    return rows


def erdos_renyi(m: int, n: int, d: int, seed: int, values: str = "f64") -> HostCsc:
    """m x n matrix with exactly ``d`` distinct uniformly random rows per column.

    ``values``: ``"f64"`` / ``"f32"`` uniform [0,1), ``"none"`` (pattern),
    or ``"id40"`` -- int64 ``2**40 + position`` in canonical order.
    """
    rng = np.random.default_rng(seed)
    rows = _distinct_rows_per_column(rng, m, n, d)
    cp = np.arange(n + 1, dtype=np.int64) * d
    ir = rows.reshape(-1).astype(np.int32)
    return HostCsc(m, n, cp, ir, _draw_values(rng, ir.size, values))


def _draw_values(rng, nnz: int, values: str):
    if values == "f64":
        return rng.random(nnz, dtype=np.float64)
    if values == "f32":
        return rng.random(nnz, dtype=np.float32)
    if values == "none":
        return None
    if values == "edge_id":
        return np.arange(nnz, dtype=np.int64)
    if values == "id40":
        return (np.int64(1) << np.int64(40)) + np.arange(nnz, dtype=np.int64)
    if values == "small_int":
        return rng.integers(1, 10, size=nnz, dtype=np.int64)
    raise ValueError(f"unknown value kind {values!r}")


def rmat_keys(scale: int, edge_factor: int, probs, seed: int, chunk: int = 1 << 22):
    """Return (sorted unique keys col*n+row, rng) for a permuted R-MAT graph.

    For every edge and every one of ``scale`` levels a quadrant is drawn with
    probabilities (a, b, c, 1-a-b-c) for (top-left, top-right, bottom-left,
    bottom-right).  Self loops are kept, duplicates merged, and every vertex
    is relabelled by one random permutation (rows and columns alike).
    """
    a, b, c = probs
    n = 1 << scale
    nedges = edge_factor * n
    rng = np.random.default_rng(seed)
    keys = np.empty(nedges, dtype=np.int64)
    ab, abc = np.float32(a + b), np.float32(a + b + c)
    fa = np.float32(a)
    for start in range(0, nedges, chunk):
        cnt = min(chunk, nedges - start)
        r = np.zeros(cnt, dtype=np.int64)
        q = np.zeros(cnt, dtype=np.int64)
        for _ in range(scale):
            u = rng.random(cnt, dtype=np.float32)
            rbit = u >= ab
            cbit = ((u >= fa) & (u < ab)) | (u >= abc)
            r <<= 1
            r |= rbit
            q <<= 1
            q |= cbit
        keys[start:start + cnt] = q * n + r  # temporarily (col, row) unpermuted
    perm = rng.permutation(n).astype(np.int64)
    cols = perm[keys // n]
    rows = perm[keys % n]
    keys = np.unique(cols * n + rows)
    return keys, rng


def rmat(scale: int, edge_factor: int, seed: int, probs=RMAT_GRAPH500, values: str = "f64") -> HostCsc:
    """Permuted R-MAT matrix of dimension 2**scale (see :func:`rmat_keys`).

    ``values``: ``"f64"``/``"f32"`` uniform [0,1) drawn after de-duplication
    in canonical order, ``"edge_id"`` = int64 position in canonical order,
    ``"none"`` = pattern only.
    """
    n = 1 << scale
    keys, rng = rmat_keys(scale, edge_factor, probs, seed)
    A = csc_from_sorted_keys(keys, n, n)
    A.num = _draw_values(rng, A.nnz, values)
    return A


def column_block(A: HostCsc, r0: int, r1: int, c0: int, c1: int) -> HostCsc:
    """Contiguous block A[r0:r1, c0:c1] (input preparation for stage blocks)."""
    s, e = int(A.cp[c0]), int(A.cp[c1])
    rows = A.ir[s:e].astype(np.int64)
    cols = np.repeat(np.arange(c0, c1, dtype=np.int64), np.diff(A.cp[c0:c1 + 1]))
    keep = (rows >= r0) & (rows < r1)
    vals = None if A.num is None else A.num[s:e][keep]
    return from_triples(rows[keep] - r0, cols[keep] - c0, vals, r1 - r0, c1 - c0)


def index_vector(length: int, n: int, seed: int, repeat_frac: float = 0.1) -> np.ndarray:
    """Unsorted int32 index vector over [0, n) with ``repeat_frac`` repeats.

    ``int((1-repeat_frac)*length)`` distinct indices are drawn without
    replacement, the rest uniformly from that set; the concatenation is
    shuffled.
    """
    rng = np.random.default_rng(seed)
    ndist = int((1.0 - repeat_frac) * length)
    if length and ndist == 0:
        ndist = 1
    distinct = rng.choice(n, size=ndist, replace=False).astype(np.int64)
    extra = rng.choice(distinct, size=length - ndist, replace=True) if length > ndist else np.empty(0, np.int64)
    v = np.concatenate([distinct, extra])
    rng.shuffle(v)
    return v.astype(np.int32)


def grid_index(x, y, z, n):
    """Lexicographic index of grid point (x, y, z) on an n^3 grid (x fastest)."""
    return x + n * (y + n * z)


def laplacian7(n: int, dtype=np.float64) -> HostCsc:
    """7-point Dirichlet Laplacian on an n^3 grid: diagonal 6, neighbours -1.

    Neighbours outside the grid are dropped; rows and columns are in
    lexicographic order (x fastest).
    """
    N = n ** 3
    idx = np.arange(N, dtype=np.int64)
    x, y, z = idx % n, (idx // n) % n, idx // (n * n)
    rows, cols, vals = [idx], [idx], [np.full(N, 6, dtype=dtype)]
    for (dx, dy, dz) in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
        ok = (x + dx >= 0) & (x + dx < n) & (y + dy >= 0) & (y + dy < n) & (z + dz >= 0) & (z + dz < n)
        src = idx[ok]
        rows.append(grid_index(x[ok] + dx, y[ok] + dy, z[ok] + dz, n))
        cols.append(src)
        vals.append(np.full(src.size, -1, dtype=dtype))
    return from_triples(np.concatenate(rows), np.concatenate(cols), np.concatenate(vals), N, N)


def aggregation(n: int, dtype=np.float64, transpose: bool = False) -> HostCsc:
    """2x2x2 piecewise-constant aggregation P (n^3 x (n/2)^3), values 1.

    Fine point (x, y, z) belongs to coarse point (x//2, y//2, z//2).  With
    ``transpose`` the (n/2)^3 x n^3 restriction P^T is returned.
    """
    if n % 2:
        raise ValueError("n must be even")
    N, h = n ** 3, n // 2
    idx = np.arange(N, dtype=np.int64)
    x, y, z = idx % n, (idx // n) % n, idx // (n * n)
    coarse = grid_index(x // 2, y // 2, z // 2, h)
    vals = np.ones(N, dtype=dtype)
    if transpose:
        return from_triples(coarse, idx, vals, h ** 3, N)
    return from_triples(idx, coarse, vals, N, h ** 3)


def galerkin_sizes(count: int, seed: int, lo: int = 16, hi: int = 96) -> np.ndarray:
    """Even grid sizes n = 2*round(exp(U)/2), U ~ Uniform[ln lo, ln hi]."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(np.log(lo), np.log(hi), size=count)
    n = 2 * np.round(np.exp(u) / 2).astype(np.int64)
    return np.clip(n, lo, hi)


def random_permutation(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).permutation(n).astype(np.int32)
