"""Seeded synthetic inputs: finite-difference diffusion matrices in CSR form.

This module builds the linear systems the solver is exercised on and nothing
else: it holds none of the solver's arithmetic (no products with the matrix,
no inner products, no preconditioner).  Both the HIP path and the CPU oracle
consume the arrays it returns.

The paper's benchmark problem is the constant-coefficient Laplace equation,
discretised with 5-/7-point stencils in two/three dimensions and solved with
Jacobi-preconditioned CG (Section 4.1, "Methodology").  The variable-coefficient
generalisation below reduces to exactly that matrix when every cell
coefficient is 1.

Discretisation (one unknown per cell, x index fastest):
  * interior face between cells i and j: 2 k_i k_j / (k_i + k_j)
    (harmonic average), multiplied by the anisotropy factor ``a`` on x-faces;
  * Dirichlet boundary face of cell i: k_i (times ``a`` on x-faces), so that
    k == 1 gives diagonal 4 (2D) or 6 (3D) on every row;
  * diagonal = sum of the cell's face coefficients; off-diagonal = -face.
No h^2 scaling is applied (CG iterates are invariant to scaling A and b).

Column indices inside each row are sorted ascending.  Values are float64,
row pointers and column indices int32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class CSR:
    """A square sparse matrix in CSR form (int32 indices, float64 values)."""

    n: int
    rowptr: np.ndarray  # int32[n + 1]
    col: np.ndarray  # int32[nnz]
    val: np.ndarray  # float64[nnz]
    shape: tuple = ()  # grid shape (z, y, x) or (y, x) when built from a grid
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp

        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))


@dataclass
class System:
    """A linear system A x = b with an optional known exact solution."""

    A: CSR
    b: np.ndarray
    x_exact: np.ndarray | None = None
    meta: dict = field(default_factory=dict)


def _harmonic(k1: np.ndarray, k2: np.ndarray) -> np.ndarray:
    return 2.0 * k1 * k2 / (k1 + k2)


def diffusion_csr(k: np.ndarray, aniso: float = 1.0) -> CSR:
    """Assemble the cell-centred diffusion matrix for cell coefficients ``k``.

    ``k`` has shape (ny, nx) for 2D or (nz, ny, nx) for 3D.  ``aniso``
    multiplies every x-direction face coefficient (boundary faces included).
    """
    k = np.asarray(k, dtype=np.float64)
    dim = k.ndim
    if dim not in (2, 3):
        raise ValueError("k must be 2-D or 3-D")
    shape = k.shape
    n = int(np.prod(shape))
    idx = np.arange(n, dtype=np.int64).reshape(shape)
    # axis order in the array: (z, y, x) / (y, x); the x axis is the last one.
    axes = list(range(dim))
    stride = [int(np.prod(shape[ax + 1:])) for ax in axes]
    # entries per row in ascending column order:
    #   -z, -y, -x, centre, +x, +y, +z   (3D)
    #   -y, -x, centre, +x, +y            (2D)
    order = [(ax, -1) for ax in axes] + [None] + [(ax, +1) for ax in reversed(axes)]
    S = len(order)
    vals = np.zeros((n, S), dtype=np.float64)
    cols = np.zeros((n, S), dtype=np.int64)
    mask = np.zeros((n, S), dtype=bool)
    diag = np.zeros(shape, dtype=np.float64)
    centre_slot = order.index(None)
    for slot, item in enumerate(order):
        if item is None:
            continue
        ax, d = item
        factor = aniso if ax == dim - 1 else 1.0
        # neighbour coefficients via a shifted view; boundary face = own k
        face = np.empty(shape, dtype=np.float64)
        inner = [slice(None)] * dim
        nbr = [slice(None)] * dim
        edge = [slice(None)] * dim
        if d < 0:
            inner[ax] = slice(1, None)
            nbr[ax] = slice(0, -1)
            edge[ax] = slice(0, 1)
        else:
            inner[ax] = slice(0, -1)
            nbr[ax] = slice(1, None)
            edge[ax] = slice(-1, None)
        inner, nbr, edge = tuple(inner), tuple(nbr), tuple(edge)
        face[inner] = factor * _harmonic(k[inner], k[nbr])
        face[edge] = factor * k[edge]
        diag += face
        has = np.zeros(shape, dtype=bool)
        has[inner] = True
        v = np.zeros(shape, dtype=np.float64)
        v[inner] = -face[inner]
        c = idx + d * stride[ax]
        vals[:, slot] = v.reshape(-1)
        cols[:, slot] = c.reshape(-1)
        mask[:, slot] = has.reshape(-1)
    vals[:, centre_slot] = diag.reshape(-1)
    cols[:, centre_slot] = idx.reshape(-1)
    mask[:, centre_slot] = True
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    if rowptr[-1] > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds the int32 index range")
    return CSR(
        n=n,
        rowptr=rowptr.astype(np.int32),
        col=cols[mask].astype(np.int32),
        val=np.ascontiguousarray(vals[mask]),
        shape=tuple(shape),
        meta={"dim": dim, "aniso": float(aniso)},
    )


def laplace_2d(n: int) -> CSR:
    """Constant-coefficient 5-point Laplacian on an n x n interior grid."""
    return diffusion_csr(np.ones((n, n)))


def laplace_3d(n: int) -> CSR:
    """Constant-coefficient 7-point Laplacian on an n^3 interior grid."""
    return diffusion_csr(np.ones((n, n, n)))


def stencil_laplacian(shape: tuple, points: int) -> CSR:
    """Constant-coefficient Laplace operator on an interior grid of ``shape``
    ((y, x) or (z, y, x), x fastest) with Dirichlet boundaries, for the four
    stencils of the paper's CG benchmark (Section 4.1):

      * star (5 points in 2D, 7 in 3D): -1 to each face neighbour, 2 d on
        the diagonal (the same matrix as laplace_2d / laplace_3d);
      * box (9 points in 2D, 27 in 3D): -1 to each of the 3^d - 1 neighbours
        sharing a face, edge or corner, 3^d - 1 on the diagonal; this is
        3^d I - S (x) ... (x) S with S = tridiag(1, 1, 1) per axis, SPD
        because every eigenvalue of S lies in (-1, 3).

    Neighbours outside the grid are dropped (their rows keep the full
    diagonal).  Built directly in CSR order: the neighbour offsets are taken
    in lexicographic order of (dz, dy, dx), which is increasing column order,
    so no sort is needed even for 10^8 nonzeros."""
    dim = len(shape)
    if (dim, points) not in ((2, 5), (2, 9), (3, 7), (3, 27)):
        raise ValueError("stencils: 5 or 9 points in 2D, 7 or 27 in 3D")
    box = points in (9, 27)
    deltas = [d for d in np.ndindex(*([3] * dim))]
    deltas = [tuple(c - 1 for c in d) for d in deltas]
    if not box:
        deltas = [d for d in deltas if sum(abs(c) for c in d) <= 1]
    n = int(np.prod(shape))
    strides = [int(np.prod(shape[a + 1:])) for a in range(dim)]
    coords = np.indices(shape, dtype=np.int32).reshape(dim, -1)
    cols = np.empty((n, len(deltas)), dtype=np.int32)
    vals = np.empty((n, len(deltas)), dtype=np.float64)
    center = float(len(deltas) - 1) if box else float(2 * dim)
    for q, d in enumerate(deltas):
        ok = np.ones(n, dtype=bool)
        off = 0
        for a in range(dim):
            c = coords[a] + d[a]
            ok &= (c >= 0) & (c < shape[a])
            off += d[a] * strides[a]
        cols[:, q] = np.where(ok, np.arange(n, dtype=np.int32) + off, -1)
        vals[:, q] = center if not any(d) else -1.0
    keep = cols >= 0
    rowptr = np.zeros(n + 1, dtype=np.int32)
    np.cumsum(keep.sum(axis=1), out=rowptr[1:])
    A = CSR(n=n, rowptr=rowptr, col=np.ascontiguousarray(cols[keep]), val=np.ascontiguousarray(vals[keep]),
            shape=tuple(shape))
    A.meta["stencil"] = f"{points}-point"
    return A


def convection_diffusion(shape: tuple, conv: tuple) -> CSR:
    """Nonsymmetric test operator for TFQMR: the star Laplacian of
    stencil_laplacian plus centred first differences along each axis,
    -1 + c_a/2 to the +1 neighbour and -1 - c_a/2 to the -1 neighbour of
    axis a (c_a = velocity x cell width along a; |c_a| < 2 keeps every
    off-diagonal negative, so the matrix is a nonsingular M-matrix)."""
    dim = len(shape)
    if len(conv) != dim:
        raise ValueError("one convection coefficient per axis")
    A = stencil_laplacian(shape, 5 if dim == 2 else 7)
    strides = [int(np.prod(shape[a + 1:])) for a in range(dim)]
    rows = np.repeat(np.arange(A.n, dtype=np.int64), np.diff(A.rowptr))
    off = A.col.astype(np.int64) - rows
    val = A.val.copy()
    for a in range(dim):
        val[off == strides[a]] += conv[a] / 2.0
        val[off == -strides[a]] -= conv[a] / 2.0
    A.val = val
    A.meta["stencil"] = f"convection-diffusion {conv}"
    return A


def stencil_eigval(shape: tuple, points: int, modes: tuple) -> float:
    """Eigenvalue of stencil_laplacian(shape, points) for the Dirichlet sine
    mode ``modes`` (one 1-based mode number per axis; the eigenvector is
    laplace_eigvec(shape, modes)): star: sum of 2 - 2 cos(m pi / (n + 1));
    box: 3^d - prod of (1 + 2 cos(m pi / (n + 1)))."""
    cs = [math.cos(m * math.pi / (n_ax + 1)) for n_ax, m in zip(shape, modes)]
    if points in (5, 7):
        return float(sum(2.0 - 2.0 * c for c in cs))
    return float(3 ** len(shape) - math.prod(1.0 + 2.0 * c for c in cs))


def laplace_eigvec(shape: tuple, modes: tuple) -> np.ndarray:
    """Dirichlet sine eigenvector with mode numbers ``modes`` (one per axis,
    1-based, axis order matching ``shape``), flattened in row order."""
    vecs = []
    for n_ax, m in zip(shape, modes):
        t = np.arange(1, n_ax + 1, dtype=np.float64)
        vecs.append(np.sin(m * math.pi * t / (n_ax + 1)))
    out = vecs[0]
    for v in vecs[1:]:
        out = np.multiply.outer(out, v)
    return np.ascontiguousarray(out.reshape(-1))


def laplace_eigval(shape: tuple, modes: tuple) -> float:
    """Eigenvalue of the constant-coefficient stencil for ``modes``:
    sum over axes of 2 - 2 cos(m pi / (n + 1))."""
    return float(sum(2.0 - 2.0 * math.cos(m * math.pi / (n_ax + 1)) for n_ax, m in zip(shape, modes)))


def diffusion_csr_torch(k, aniso: float = 1.0):
    """The matrix of :func:`diffusion_csr` assembled with torch tensor
    operations on ``k``'s device (the bulk workloads are assembled on the GPU
    from host-drawn coefficients).  Returns (rowptr int32[n+1], col
    int32[nnz], val float64[nnz]) on that device.  The face values are the
    same IEEE operations in the same order as the numpy assembly (one
    elementwise operation per step, no contraction), so both give the same
    bits from the same ``k``."""
    import torch

    k = k.to(torch.float64)
    dim = k.dim()
    if dim not in (2, 3):
        raise ValueError("k must be 2-D or 3-D")
    shape = tuple(k.shape)
    dev = k.device
    n = int(np.prod(shape))
    idx = torch.arange(n, dtype=torch.int64, device=dev).reshape(shape)
    axes = list(range(dim))
    stride = [int(np.prod(shape[ax + 1:])) for ax in axes]
    order = [(ax, -1) for ax in axes] + [None] + [(ax, +1) for ax in reversed(axes)]
    S = len(order)
    vals = torch.zeros((n, S), dtype=torch.float64, device=dev)
    cols = torch.zeros((n, S), dtype=torch.int64, device=dev)
    mask = torch.zeros((n, S), dtype=torch.bool, device=dev)
    diag = torch.zeros(shape, dtype=torch.float64, device=dev)
    centre_slot = order.index(None)
    for slot, item in enumerate(order):
        if item is None:
            continue
        ax, d = item
        factor = aniso if ax == dim - 1 else 1.0
        face = torch.empty(shape, dtype=torch.float64, device=dev)
        inner = [slice(None)] * dim
        nbr = [slice(None)] * dim
        edge = [slice(None)] * dim
        if d < 0:
            inner[ax], nbr[ax], edge[ax] = slice(1, None), slice(0, shape[ax] - 1), slice(0, 1)
        else:
            inner[ax], nbr[ax], edge[ax] = slice(0, shape[ax] - 1), slice(1, None), slice(shape[ax] - 1, None)
        inner, nbr, edge = tuple(inner), tuple(nbr), tuple(edge)
        k1, k2 = k[inner], k[nbr]
        face[inner] = factor * (2.0 * k1 * k2 / (k1 + k2))
        face[edge] = factor * k[edge]
        diag += face
        has = torch.zeros(shape, dtype=torch.bool, device=dev)
        has[inner] = True
        v = torch.zeros(shape, dtype=torch.float64, device=dev)
        v[inner] = -face[inner]
        vals[:, slot] = v.reshape(-1)
        cols[:, slot] = (idx + d * stride[ax]).reshape(-1)
        mask[:, slot] = has.reshape(-1)
    vals[:, centre_slot] = diag.reshape(-1)
    cols[:, centre_slot] = idx.reshape(-1)
    mask[:, centre_slot] = True
    counts = mask.sum(dim=1)
    rowptr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    torch.cumsum(counts, 0, out=rowptr[1:])
    if int(rowptr[-1]) > np.iinfo(np.int32).max:
        raise ValueError("nnz exceeds the int32 index range")
    return rowptr.to(torch.int32), cols[mask].to(torch.int32), vals[mask].contiguous()


def box_smooth_3(g: np.ndarray) -> np.ndarray:
    """Mean over every valid 3^d window of ``g`` (shape shrinks by 2 per axis)."""
    d = g.ndim
    out_shape = tuple(s - 2 for s in g.shape)
    acc = np.zeros(out_shape, dtype=np.float64)
    for offs in np.ndindex(*(3,) * d):
        sl = tuple(slice(o, o + s) for o, s in zip(offs, out_shape))
        acc += g[sl]
    return acc / float(3 ** d)


# --------------------------------------------------------------------------
# Workload recipes
# --------------------------------------------------------------------------

def poisson2d_manufactured(n: int = 64, seed: int = 0) -> System:
    """2D 5-point Poisson on an n x n grid, x* ~ U[-1, 1], b = A x*.

    The product A x* is taken with scipy.sparse (a library routine) while
    building the input, not with the solver's own kernels."""
    A = laplace_2d(n)
    rng = np.random.default_rng(seed)
    xs = rng.uniform(-1.0, 1.0, A.n)
    b = np.asarray(A.to_scipy() @ xs, dtype=np.float64)
    return System(A=A, b=b, x_exact=xs, meta={"workload": f"poisson2d_{n}x{n}", "seed": seed})


def diffusion3d_smoothed(n: int = 128, seed: int = 2) -> System:
    """3D 7-point variable-coefficient diffusion on n^3 cells.

    k = exp(g_s), g_s = 3^3 box mean of g ~ N(0,1) drawn on an (n+2)^3 grid;
    harmonic face averaging; b ~ U[-1, 1]."""
    rng = np.random.default_rng(seed)
    g = rng.standard_normal((n + 2, n + 2, n + 2))
    k = np.exp(box_smooth_3(g))
    A = diffusion_csr(k)
    b = rng.uniform(-1.0, 1.0, A.n)
    return System(A=A, b=b, meta={"workload": f"diffusion3d_{n}^3_box3", "seed": seed})


@dataclass
class Fields:
    """The host-drawn part of a log-normal diffusion system: cell
    coefficients k (grid-shaped), right-hand side b and the anisotropy; the
    matrix is assembled from them by :func:`diffusion_csr` (host) or
    :func:`diffusion_csr_torch` (any torch device)."""

    k: np.ndarray
    b: np.ndarray
    aniso: float
    meta: dict = field(default_factory=dict)

    def system(self) -> System:
        return System(A=diffusion_csr(self.k, aniso=self.aniso), b=self.b, meta=dict(self.meta))


def _lognormal_fields(rng: np.random.Generator, dim: int, side: int, sigma: float, aniso: float) -> Fields:
    shape = (side,) * dim
    g = rng.standard_normal(shape)
    k = np.exp(sigma * g)
    b = rng.uniform(-1.0, 1.0, int(np.prod(shape)))
    return Fields(k=k, b=b, aniso=aniso, meta={"dim": dim, "side": side, "sigma": sigma, "aniso": aniso})


def _lognormal_system(rng: np.random.Generator, dim: int, side: int, sigma: float, aniso: float) -> System:
    return _lognormal_fields(rng, dim, side, sigma, aniso).system()


def batch2d_lognormal(count: int = 256, seed: int = 3, side_lo: int = 32, side_hi: int = 256,
                      sigma: float = 1.0) -> list[System]:
    """``count`` independent 2D 5-point systems, side ~ U{side_lo..side_hi},
    k = exp(sigma g), g ~ N(0,1) per cell, b ~ U[-1, 1]."""
    out = []
    for i, child in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.default_rng(child)
        side = int(rng.integers(side_lo, side_hi + 1))
        s = _lognormal_system(rng, 2, side, sigma, 1.0)
        s.meta["index"] = i
        out.append(s)
    return out


def _learned_pc_fields_from(child, index: int, side_lo: int, side_hi: int) -> Fields:
    rng = np.random.default_rng(child)
    side = int(rng.integers(side_lo, side_hi + 1))
    sigma = float(rng.uniform(0.5, 2.0))
    aniso = float(math.exp(rng.uniform(0.0, math.log(100.0))))
    f = _lognormal_fields(rng, 3, side, sigma, aniso)
    f.meta["index"] = index
    return f


def _learned_pc_from(child, index: int, side_lo: int, side_hi: int) -> System:
    return _learned_pc_fields_from(child, index, side_lo, side_hi).system()


def learned_pc_set(count: int, seed: int, side_lo: int = 32, side_hi: int = 96) -> list[System]:
    """3D 7-point systems for the learned preconditioner: side ~ U{32..96},
    sigma ~ U[0.5, 2], anisotropy ~ log-U[1, 100]; system i draws from child
    i of SeedSequence(seed)."""
    return [_learned_pc_from(child, i, side_lo, side_hi)
            for i, child in enumerate(np.random.SeedSequence(seed).spawn(count))]


def learned_pc_system(args) -> System:
    """System ``index`` of ``learned_pc_set(count, seed, side_lo, side_hi)``
    alone (args = (seed, index, count, side_lo, side_hi)), for generating a
    set in several processes."""
    seed, index, count, side_lo, side_hi = args
    # child i of SeedSequence(seed).spawn(...) is SeedSequence(seed, spawn_key=(i,))
    return _learned_pc_from(np.random.SeedSequence(seed, spawn_key=(index,)), index, side_lo, side_hi)


def learned_pc_fields(args) -> Fields:
    """The fields of :func:`learned_pc_system` (same args, same draws)."""
    seed, index, count, side_lo, side_hi = args
    return _learned_pc_fields_from(np.random.SeedSequence(seed, spawn_key=(index,)), index, side_lo, side_hi)


def mixed_batch_params(count: int = 1024, seed: int = 5, n_lo: float = 1e3, n_hi: float = 1e6):
    """Per-system parameters of the mixed 2D/3D batch (drawn before the
    fields so a caller can size the batch without assembling it)."""
    params = []
    for i, child in enumerate(np.random.SeedSequence(seed).spawn(count)):
        rng = np.random.default_rng(child)
        dim = 2 + int(rng.integers(0, 2))
        nt = math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))
        side = max(2, int(round(nt ** (1.0 / dim))))
        sigma = float(rng.uniform(0.5, 2.0))
        aniso = float(math.exp(rng.uniform(0.0, math.log(1000.0))))
        params.append({"index": i, "dim": dim, "side": side, "sigma": sigma, "aniso": aniso, "rng": rng})
    return params


def mixed_batch(count: int = 1024, seed: int = 5, limit: int | None = None) -> list[System]:
    """Mixed batch: dim ~ {2,3}, N ~ log-U[1e3, 1e6], sigma ~ U[0.5, 2],
    anisotropy ~ log-U[1, 1000]; ``limit`` assembles only the first systems."""
    out = []
    for p in mixed_batch_params(count, seed)[: (limit or count)]:
        s = _lognormal_system(p["rng"], p["dim"], p["side"], p["sigma"], p["aniso"])
        s.meta["index"] = p["index"]
        out.append(s)
    return out


def mixed_fields(args) -> Fields:
    """The fields of system ``index`` of ``mixed_batch(count, seed)`` alone
    (args = (seed, index, n_lo, n_hi)): child i of SeedSequence(seed).spawn(...)
    is SeedSequence(seed, spawn_key=(i,)), drawn in the same order."""
    seed, index, n_lo, n_hi = args
    rng = np.random.default_rng(np.random.SeedSequence(seed, spawn_key=(index,)))
    dim = 2 + int(rng.integers(0, 2))
    nt = math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))
    side = max(2, int(round(nt ** (1.0 / dim))))
    sigma = float(rng.uniform(0.5, 2.0))
    aniso = float(math.exp(rng.uniform(0.0, math.log(1000.0))))
    f = _lognormal_fields(rng, dim, side, sigma, aniso)
    f.meta["index"] = index
    return f


def mixed_system(args) -> System:
    """System ``index`` of ``mixed_batch(count, seed)`` alone (args as for
    :func:`mixed_fields`)."""
    return mixed_fields(args).system()


def fields_threaded(fn, args, threads: int = 8) -> list:
    """fn over args in a thread pool (numpy's generators and elementwise
    functions release the GIL on large arrays), results in args order."""
    if threads <= 1 or len(args) < 4:
        return [fn(a) for a in args]
    from concurrent.futures import ThreadPoolExecutor

    with ThreadPoolExecutor(threads) as ex:
        return list(ex.map(fn, args))


def random_csr(n: int, max_per_row: int, seed: int, empty_rows: bool = True) -> CSR:
    """Random square CSR with sorted columns (for SpMV/reduction edge cases):
    row lengths ~ U{0..max_per_row} (or U{1..} without empty rows)."""
    rng = np.random.default_rng(seed)
    lo = 0 if empty_rows else 1
    counts = rng.integers(lo, max_per_row + 1, size=n)
    counts = np.minimum(counts, n)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    cols = np.empty(int(rowptr[-1]), dtype=np.int32)
    for i in range(n):
        c = np.sort(rng.choice(n, size=int(counts[i]), replace=False))
        cols[rowptr[i]:rowptr[i + 1]] = c
    vals = rng.uniform(-1.0, 1.0, int(rowptr[-1]))
    return CSR(n=n, rowptr=rowptr.astype(np.int32), col=cols, val=vals)


# --------------------------------------------------------------------------
# Seeded initial parameters of the 16 -> 64 -> 64 -> 9 MLP
# --------------------------------------------------------------------------
MLP_SHAPES = [("W1", (64, 16)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (9, 64)), ("b3", (9,))]


def mlp_initial_params(seed: int = 7) -> dict:
    """Glorot-uniform weights, zero biases, drawn in the order of MLP_SHAPES
    (float64; the GPU side takes float32 copies of the same numbers)."""
    rng = np.random.default_rng(seed)
    out = {}
    for name, shape in MLP_SHAPES:
        if name.startswith("W"):
            lim = math.sqrt(6.0 / (shape[0] + shape[1]))
            out[name] = rng.uniform(-lim, lim, shape)
        else:
            out[name] = np.zeros(shape)
    return out
