"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only *generates inputs*: sparse matrices of the shapes and
coefficient distributions the method is exercised on, exact solutions and
right-hand sides.  It holds none of the solver's arithmetic (no smoothing,
matching, Galerkin products or Krylov steps).  Both the CPU oracle and the
GPU library receive the very same arrays (same bits) from here.

Random numbers come from one counter-based generator, SplitMix64
(Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014): the k-th draw of stream ``seed`` is the first SplitMix64 output
for the state ``seed * 2**32 + k``; uniforms in [0, 1) keep its top 53 bits.

Matrices are CSR with int32 row pointers / column indices (columns strictly
ascending per row, diagonal present) and float64 values.  Grid points are
numbered ``id = x + N*y + N*N*z``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(counter: np.ndarray) -> np.ndarray:
    """First SplitMix64 output for each state in ``counter`` (uint64 array)."""
    z = np.asarray(counter, dtype=np.uint64) + _GOLDEN
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """``count`` uniforms in [0, 1) from stream ``seed`` starting at draw ``offset``."""
    k = np.arange(offset, offset + count, dtype=np.uint64)
    base = np.uint64((int(seed) << 32) & 0xFFFFFFFFFFFFFFFF)
    with np.errstate(over="ignore"):
        bits = splitmix64(base + k)
    return (bits >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_pm1(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """``count`` values uniform in [-1, 1): 2u - 1."""
    return 2.0 * uniform(seed, count, offset) - 1.0


def normal(seed: int, count: int) -> np.ndarray:
    """Standard normals by the Box-Muller transform on pairs of uniforms."""
    m = (count + 1) // 2
    u = uniform(seed, 2 * m)
    u1 = 1.0 - u[0::2]          # (0, 1]: keeps log finite
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * m)
    z[0::2] = r * np.cos(2.0 * math.pi * u2)
    z[1::2] = r * np.sin(2.0 * math.pi * u2)
    return z[:count]


@dataclass
class CSR:
    """Square sparse matrix in CSR form (int32 indices, float64 values)."""
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.row_ptr), shape=(self.n, self.n))


def _assemble(n: int, cols: np.ndarray, vals: np.ndarray, valid: np.ndarray) -> CSR:
    """Pack per-row candidate slots (n, S), already in ascending column order."""
    counts = valid.sum(axis=1).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2 ** 31:
        raise ValueError("nnz does not fit int32 indices")
    col = cols[valid].astype(np.int32)
    val = vals[valid].astype(np.float64)
    return CSR(n, row_ptr.astype(np.int32), col, val)


def _grid(N: int):
    idx = np.arange(N ** 3, dtype=np.int64)
    return idx, idx % N, (idx // N) % N, idx // (N * N)


def _offsets_3d(radius_set):
    """Neighbour offsets (dx, dy, dz) sorted so that ids ascend within a row."""
    offs = sorted(radius_set, key=lambda d: (d[2], d[1], d[0]))
    return offs


def poisson7(N: int) -> CSR:
    """7-point finite-difference Laplacian on an N^3 grid, Dirichlet boundary.

    Unscaled integer stencil: 6 on the diagonal, -1 for each in-domain face
    neighbour (the 1/h^2 factor is dropped: CG iterates do not change under
    A -> cA).  nnz = 7N^3 - 6N^2.
    """
    return poisson7_box(N, N, N)


def poisson7_box(Nx: int, Ny: int, Nz: int) -> CSR:
    """The same stencil on an Nx x Ny x Nz box, id = x + Nx y + Nx Ny z.  With
    Nz = P * Nx the consecutive row blocks of P tasks are Nx x Ny x Nx cubes
    (the per-task share of a weak-scaling run)."""
    n = Nx * Ny * Nz
    idx = np.arange(n, dtype=np.int64)
    x, y, z = idx % Nx, (idx // Nx) % Ny, idx // (Nx * Ny)
    offs = _offsets_3d([(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0),
                        (1, 0, 0), (0, 1, 0), (0, 0, 1)])
    cols = np.empty((n, 7), dtype=np.int64)
    vals = np.empty((n, 7))
    valid = np.empty((n, 7), dtype=bool)
    for s, (dx, dy, dz) in enumerate(offs):
        xx, yy, zz = x + dx, y + dy, z + dz
        valid[:, s] = (xx >= 0) & (xx < Nx) & (yy >= 0) & (yy < Ny) & (zz >= 0) & (zz < Nz)
        cols[:, s] = idx + dx + Nx * dy + Nx * Ny * dz
        vals[:, s] = 6.0 if (dx, dy, dz) == (0, 0, 0) else -1.0
    return _assemble(n, cols, vals, valid)


def _face_operator(N: int, kappa: np.ndarray, offs, boundary_adds_cell: bool) -> CSR:
    """Cell-centred diffusion operator with harmonic-mean couplings.

    For every neighbour offset d: a_ij = -2 k_i k_j / (k_i + k_j) when j is in
    the domain; the diagonal gathers the matching positive couplings and, for
    an out-of-domain neighbour, k_i (Dirichlet wall).  The product and sum are
    commutative so a_ij and a_ji are bitwise equal.
    """
    n = N ** 3
    idx, x, y, z = _grid(N)
    k = kappa.reshape(-1)
    S = len(offs)
    cols = np.empty((n, S), dtype=np.int64)
    vals = np.zeros((n, S))
    valid = np.empty((n, S), dtype=bool)
    diag_slot = offs.index((0, 0, 0))
    diag = np.zeros(n)
    for s, (dx, dy, dz) in enumerate(offs):
        if s == diag_slot:
            cols[:, s] = idx
            valid[:, s] = True
            continue
        xx, yy, zz = x + dx, y + dy, z + dz
        inside = (xx >= 0) & (xx < N) & (yy >= 0) & (yy < N) & (zz >= 0) & (zz < N)
        j = np.where(inside, idx + dx + N * dy + N * N * dz, idx)
        kj = k[j]
        h = 2.0 * (k * kj) / (k + kj)
        valid[:, s] = inside
        cols[:, s] = j
        vals[:, s] = -h
        diag = diag + np.where(inside, h, k if boundary_adds_cell else 0.0)
    vals[:, diag_slot] = diag
    return _assemble(n, cols, vals, valid)


def diffusion27(N: int, seed: int) -> CSR:
    """27-point variable-coefficient diffusion on N^3, kappa log-uniform in [1e-3, 1e3].

    kappa_c = 10**(6u - 3) per cell; all 26 neighbours couple with the
    harmonic-mean coefficient; an out-of-domain slot adds kappa_i to the
    diagonal.  Symmetric, irreducibly diagonally dominant M-matrix (SPD).
    """
    kappa = 10.0 ** (6.0 * uniform(seed, N ** 3) - 3.0)
    offs = _offsets_3d([(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1)
                        for dx in (-1, 0, 1)])
    return _face_operator(N, kappa, offs, boundary_adds_cell=True)


def gaussian_field(N: int, seed: int, ell: float = 8.0) -> np.ndarray:
    """Unit-variance Gaussian random field on N^3 with Gaussian covariance.

    White noise on a padded, non-periodic grid is smoothed separably by a 1-D
    Gaussian of std ell/sqrt(2), truncated at 4 std and normalised so that
    the squared 3-D kernel sums to one; the centre N^3 block is kept.
    Returns an array of shape (N, N, N) indexed [z, y, x].
    """
    from scipy.ndimage import correlate1d
    s = ell / math.sqrt(2.0)
    half = int(math.ceil(4.0 * s))
    t = np.arange(-half, half + 1, dtype=np.float64)
    ker = np.exp(-0.5 * (t / s) ** 2)
    ker /= math.sqrt(float(np.sum(ker ** 2)))
    M = N + 2 * half
    g = normal(seed, M ** 3).reshape(M, M, M)
    for ax in range(3):
        g = correlate1d(g, ker, axis=ax, mode="constant")
    return np.ascontiguousarray(g[half:half + N, half:half + N, half:half + N])


def lognormal7(N: int, seed: int, sigma2: float = 2.0, ell: float = 8.0) -> CSR:
    """7-point diffusion on N^3 with log-normal coefficients.

    log kappa = sqrt(sigma2) * g with g a unit-variance Gaussian random field
    of correlation length ell cells; face coefficient = harmonic mean of the
    two cells, a boundary face uses the cell's own kappa.
    """
    g = gaussian_field(N, seed, ell)
    kappa = np.exp(math.sqrt(sigma2) * g)
    offs = _offsets_3d([(0, 0, -1), (0, -1, 0), (-1, 0, 0), (0, 0, 0),
                        (1, 0, 0), (0, 1, 0), (0, 0, 1)])
    return _face_operator(N, kappa, offs, boundary_adds_cell=True)


def permute_tail(A: CSR, seed: int, start: int) -> CSR:
    """Symmetric relabelling of A: indices below `start` keep their place,
    the others are shuffled by a seeded permutation (P A P^T).  Rows of the
    kept part stay banded; rows of the shuffled part couple to columns spread
    over [start, n).  Column order within each row is ascending again."""
    n = A.n
    perm = np.arange(n, dtype=np.int64)
    tail = n - start
    if tail > 0:
        perm[start:] = start + np.argsort(uniform(seed, tail), kind="stable")
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(A.row_ptr))
    r2, c2 = perm[rows], perm[A.col.astype(np.int64)]
    order = np.lexsort((c2, r2))
    r2, c2, v2 = r2[order], c2[order], A.val[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r2, minlength=n), out=row_ptr[1:])
    return CSR(n, row_ptr.astype(np.int32), c2.astype(np.int32), v2.astype(np.float64))


def with_hubs(A: CSR, hubs, eps: float = 0.05) -> CSR:
    """A plus dense couplings: for each (h, stride) in `hubs`, vertex h gets
    the entry -eps to every stride-th vertex j != h (both triangles), and the
    diagonals of h and j grow by the same amount, so a diagonally dominant A
    stays symmetric and diagonally dominant.  Rows of the hubs are long."""
    n = A.n
    rows = [np.repeat(np.arange(n, dtype=np.int64), np.diff(A.row_ptr))]
    cols = [A.col.astype(np.int64)]
    vals = [A.val.astype(np.float64)]
    for h, stride in hubs:
        js = np.arange(0, n, stride, dtype=np.int64)
        js = js[js != h]
        rows += [np.full(js.size, h), js, np.array([h]), js]
        cols += [js, np.full(js.size, h), np.array([h]), js]
        vals += [np.full(js.size, -eps), np.full(js.size, -eps), np.array([eps * js.size]),
                 np.full(js.size, eps)]
    r, c, v = np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)
    order = np.lexsort((c, r))
    r, c, v = r[order], c[order], v[order]
    first = np.ones(r.size, dtype=bool)
    first[1:] = (r[1:] != r[:-1]) | (c[1:] != c[:-1])
    grp = np.cumsum(first) - 1
    val = np.zeros(int(first.sum()))
    np.add.at(val, grp, v)
    r, c = r[first], c[first]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(r, minlength=n), out=row_ptr[1:])
    return CSR(n, row_ptr.astype(np.int32), c.astype(np.int32), val)


def spmv_input(A: CSR, x: np.ndarray) -> np.ndarray:
    """b = A x for building right-hand sides (scipy's CSR product)."""
    return A.scipy() @ x


def manufactured_rhs(A: CSR, seed: int):
    """Exact solution x* ~ U[-1, 1) from ``seed`` and b = A x*."""
    xs = uniform_pm1(seed, A.n)
    return xs, spmv_input(A, xs)


def batched_edges(nsys: int = 64, seed: int = 5, lo: float = 16.0, ratio: float = 6.0):
    """Grid edges N_s = round(exp(ln lo + u_s ln ratio)): log-uniform in [lo, lo*ratio]."""
    u = uniform(seed, nsys)
    return [int(round(math.exp(math.log(lo) + ui * math.log(ratio)))) for ui in u]


def batched_rhs(sys_index: int, n: int, nrhs: int, seed: int = 6) -> np.ndarray:
    """Exact solutions for system ``sys_index``: array (nrhs, n), stream seed+sys_index."""
    return uniform_pm1(seed + 1000 * (sys_index + 1), nrhs * n).reshape(nrhs, n)


WORKLOADS = {
    # name: (description, builder)
    "poisson7_32": "3D Poisson 7-point, 32^3, x* ~ U[-1,1) seed 1",
    "poisson7_160": "3D Poisson 7-point, 160^3, x* ~ U[-1,1) seed 2",
    "diffusion27_128": "27-point log-uniform diffusion, 128^3, kappa seed 3, x* seed 4",
    "batched_64x16": "64 Poisson systems, edges log-uniform [16,96] seed 5, 16 RHS",
    "lognormal7_128": "7-point log-normal GRF diffusion, 128^3, sigma^2=2, ell=8, seed 7",
}
