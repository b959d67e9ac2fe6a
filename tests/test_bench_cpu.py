"""Host logic of bench.py that the roofline depends on: the byte model of
the marching product with symmetric reads, the symmetry test that selects
it, and the source hash that ties the committed counters to the kernel's
code."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2306_17801_amd import problems as P  # noqa: E402


def test_upper_slots_of_a_7_point_grid():
    """16^3 grid: 64 slices of 64 rows, planes of 4 slices.  Every slice
    holds the offsets 0, +1, +16 and +256 on or right of the diagonal (a
    slice spans 4 grid rows, so the last grid row of a plane, which lacks
    +16, shares its slice with rows that have it), except the top plane's 4
    slices, which have no +256."""
    A = P.stencil_laplacian((16, 16, 16), 7)
    assert bench.sdia_shape(A) == (7, 8)
    assert bench.sdia_upper_slots(A) == 64 * 4 - 4


def test_upper_slots_count_brute_force():
    """Distinct (slice, offset >= 0) pairs, counted with a Python set."""
    rng = np.random.default_rng(3)
    A = P.diffusion_csr(np.exp(rng.standard_normal((5, 9, 13))), aniso=2.0)
    pairs = set()
    for i in range(A.n):
        for e in range(A.rowptr[i], A.rowptr[i + 1]):
            o = int(A.col[e]) - i
            if o >= 0:
                pairs.add((i // 64, o))
    assert bench.sdia_upper_slots(A) == len(pairs)


def test_is_symmetric():
    A = P.stencil_laplacian((6, 7, 5), 7)
    assert bench.is_symmetric(A)
    B = P.CSR(n=A.n, rowptr=A.rowptr, col=A.col, val=A.val.copy())
    row = A.n // 2
    k = int(A.rowptr[row])  # the row's first entry, left of the diagonal
    assert A.col[k] < row
    B.val[k] = np.nextafter(B.val[k], 0.0)  # one ulp: no longer symmetric bit for bit
    assert not bench.is_symmetric(B)


def test_source_hash_ignores_comments_and_whitespace(tmp_path):
    a = tmp_path / "a.hip"
    b = tmp_path / "b.hip"
    c = tmp_path / "c.hip"
    a.write_text("int f(int x) {\n    return x + 1;  // one more\n}\n")
    b.write_text("/* header */\nint f(int x) {\n  return x + 1;\n}\n")
    c.write_text("int f(int x) {\n    return x + 2;\n}\n")
    assert bench.source_hash(str(a)) == bench.source_hash(str(b))
    assert bench.source_hash(str(a)) != bench.source_hash(str(c))
    # several files (a kernel and the helpers it inlines): a code change in
    # either changes the hash, a comment change in either does not
    assert bench.source_hash(str(a)) == bench.source_hash([str(a)])
    assert bench.source_hash([str(a), str(c)]) == bench.source_hash([str(b), str(c)])
    assert bench.source_hash([str(a), str(c)]) != bench.source_hash([str(a), str(a)])
    assert bench.source_hash([str(a), str(c)]) != bench.source_hash([str(c), str(a)])


def test_dia_offsets_of_stencils():
    """Distinct column offsets: the 3D 7-point grid (nz, ny, nx) has
    0, +-1, +-nx, +-nx ny; the 2D 9-point box stencil has the 9 offsets
    of its 3 x 3 neighbourhood."""
    A = P.stencil_laplacian((4, 5, 6), 7)
    assert bench.dia_offsets(A) == [-30, -6, -1, 0, 1, 6, 30]
    B = P.stencil_laplacian((7, 8), 9)
    assert bench.dia_offsets(B) == [-9, -8, -7, -1, 0, 1, 7, 8, 9]


class _StubApcg:
    """The few binding calls batch_roofline makes, answered from a table."""
    APCG_SPMV_SDIA = 3

    def __init__(self, layouts):
        self.layouts = layouts  # handle -> (schedule, value slots)

    def apcg_mat_get_spmv_config(self, h):
        return {"schedule": self.layouts[h][0]}

    def apcg_mat_get_sdia_info(self, h):
        return {"state": 1, "offset_slots": 8, "value_slots": self.layouts[h][1]}


class _H:
    def __init__(self, h):
        self.h = h


class _Opts:
    def __init__(self, schedule):
        self.batch_schedule = schedule


def test_batch_roofline_byte_model():
    """Two systems, one on a 5-slot sliced-diagonal copy and one on CSR:
    each system's iterations times its tile product bytes (512 U + 96 per
    slice + 32 n, or 12 nnz + 4 (n + 1) + 32 n) plus 64 n of update,
    written out by hand; the persistent schedule has no such count."""
    A1 = P.laplace_2d(10)  # n = 100, 2 slices
    A2 = P.laplace_2d(7)  # n = 49, nnz = 217
    systems = [P.System(A=A1, b=np.zeros(A1.n)), P.System(A=A2, b=np.zeros(A2.n))]
    apcg = _StubApcg({0: (3, 5), 1: (0, 0)})
    res = [{"iterations": 30}, {"iterations": 11}]
    r = bench.batch_roofline(apcg, systems, [_H(0), _H(1)], res, 0.5, _Opts(2))
    b1 = 30 * (2 * (512 * 5 + 96) + 32 * 100 + 64 * 100)
    b2 = 11 * (12 * 217 + 4 * 50 + 32 * 49 + 64 * 49)
    assert A2.nnz == 217
    assert r["algorithmic_bytes"] == b1 + b2
    assert r["row_iterations"] == 30 * 100 + 11 * 49
    assert abs(r["achieved"] - (b1 + b2) / 0.5 / 1e9) < 0.06
    assert bench.batch_roofline(apcg, systems, [_H(0), _H(1)], res, 0.5, _Opts(1)) is None


class _M:
    def __init__(self, h, A):
        self.h, self.n, self.nnz = h, A.n, A.nnz


def test_learned_batch_roofline_byte_model():
    """A system on a 7-slot sliced-diagonal copy (30 flexible iterations, no
    fallback) and one on CSR (5 flexible and 20 Jacobi-mode iterations):
    9 V + 392 n per flexible iteration, V + 112 n per Jacobi-mode iteration
    (the feature run's 12 steps included) and two CSR row passes, by hand."""
    A1 = P.stencil_laplacian((6, 6, 6), 7)  # n = 216, 4 slices
    A2 = P.laplace_2d(7)
    apcg = _StubApcg({0: (3, 7), 1: (0, 0)})
    res = [{"iterations": 30, "fcg_iterations": 30}, {"iterations": 25, "fcg_iterations": 5}]
    r = bench.learned_batch_roofline(apcg, [_M(0, A1), _M(1, A2)], res, 0.25)
    csr1 = 12 * A1.nnz + 4 * (A1.n + 1)
    V1 = 4 * (512 * 7 + 96)
    csr2 = 12 * A2.nnz + 4 * (A2.n + 1)
    b1 = 30 * (9 * V1 + 392 * 216) + 12 * (V1 + 112 * 216) + 2 * csr1
    b2 = 5 * (9 * csr2 + 392 * 49) + 32 * (csr2 + 112 * 49) + 2 * csr2
    assert r["algorithmic_bytes"] == b1 + b2
    assert abs(r["achieved"] - (b1 + b2) / 0.25 / 1e9) < 0.06
