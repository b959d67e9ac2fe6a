"""The tuning table's keys and its file round trip, on the CPU (no device
calls): keys of patterns worked out by hand, the size bucket edges, and
insert / lookup / save / load / clear."""
import os

import numpy as np
import pytest

from paper_2306_17801_amd import problems as P

ARCH = "gfx950:sramecc+:xnack-"


@pytest.fixture(scope="module")
def apcg():
    import paper_2306_17801_amd as m

    m.load()
    return m


def test_key_of_the_64x64_poisson_pattern(apcg):
    # 5-point stencil on a 64 x 64 grid: every 64-row slice is one grid row,
    # offsets -64, -1, 0, 1, 64 (5 per slice, 5 overall), +-64 in the 62
    # interior slices (plane marching applies), symmetric, rows of at most 5
    # entries; n = 4096 = 2^12, nnz = 5 * 4096 - 4 * 64 = 20224, 4 nnz / n = 19.75
    A = P.laplace_2d(64)
    assert A.nnz == 20224
    key = apcg.apcg_tune_key_pattern(ARCH, A.rowptr, A.col)
    assert key == f"{ARCH}|u5.d5.p1.s1.m5|n12|r20"


def test_key_of_a_7_point_pattern(apcg):
    # 7-point stencil on 16^3: a plane is 256 rows = 4 slices, so +-256 is
    # 64 * 4 with both signs in the interior slices; n = 4096, nnz = 7 * 16^3
    # - 6 * 16^2 = 27136, 4 nnz / n = 26.5, rounded half away from zero: 27
    A = P.laplace_3d(16)
    assert A.nnz == 27136
    key = apcg.apcg_tune_key_pattern(ARCH, A.rowptr, A.col)
    assert key == f"{ARCH}|u7.d7.p1.s1.m7|n12|r27"


def test_key_of_a_1d_and_a_ragged_pattern(apcg):
    # tridiagonal of 50 rows: offsets -1, 0, 1; no offset that is a multiple of 64
    n = 50
    rows = [[i - 1, i, i + 1] for i in range(n)]
    rows[0] = [0, 1]
    rows[-1] = [n - 2, n - 1]
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.concatenate([np.array(r, np.int32) for r in rows])
    key = apcg.apcg_tune_key_pattern(ARCH, rp, col)
    assert key == f"{ARCH}|u3.d3.p0.s1.m3|n5|r12"  # 4 * 148 / 50 = 11.84
    # a 2D grid of 37 x 29: the +-37 offsets are not multiples of 64
    A = P.diffusion_csr(np.ones((29, 37)))
    key = apcg.apcg_tune_key_pattern(ARCH, A.rowptr, A.col)
    assert key.startswith(f"{ARCH}|u5.d5.p0.s1.m5|n10|")


def test_key_of_an_unsymmetric_pattern_with_many_offsets(apcg):
    # one entry above the diagonal without its transpose; 10 distinct offsets
    n = 128
    rows = [[i] for i in range(n)]
    for d in range(1, 10):
        rows[d * 3].append(min(n - 1, d * 3 + d))
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum([len(r) for r in rows])
    col = np.concatenate([np.array(sorted(r), np.int32) for r in rows])
    key = apcg.apcg_tune_key_pattern(ARCH, rp, col)
    assert key == f"{ARCH}|u10.d0.p0.s0.m2|n7|r4"  # 4 * 137 / 128 = 4.28


def test_size_bucket_edges(apcg):
    for n, lg in ((1, 0), (63, 5), (64, 6), (4095, 11), (4096, 12), (4097, 12)):
        rp = np.arange(n + 1, dtype=np.int32)
        col = np.arange(n, dtype=np.int32)
        key = apcg.apcg_tune_key_pattern(ARCH, rp, col)
        assert key.split("|")[-2] == f"n{lg}", (n, key)
        assert key.split("|")[-1] == "r4"


def test_bad_pattern_is_rejected(apcg):
    with pytest.raises(apcg.ApcgError):
        apcg.apcg_tune_key_pattern(ARCH, np.array([0, 2, 1], np.int32), np.array([0, 1], np.int32))
    with pytest.raises(apcg.ApcgError):
        apcg.apcg_tune_key_pattern("bad\tarch", np.array([0, 1], np.int32), np.array([0], np.int32))


def test_table_round_trip(apcg, tmp_path):
    apcg.apcg_tune_cache_clear()
    assert apcg.apcg_tune_cache_size() == 0
    assert apcg.apcg_tune_cache_lookup("k|a") is None
    apcg.apcg_tune_cache_insert("k|a", (8, 256, 0, apcg.APCG_SPMV_SDIA), 30.25)
    apcg.apcg_tune_cache_insert("batch|k|b", (2, 0, 1024, 1), 1.5e5)
    apcg.apcg_tune_cache_insert("k|a", (6, 512, 0, apcg.APCG_SPMV_SDIA), 29.5)  # replaces
    assert apcg.apcg_tune_cache_size() == 2
    assert apcg.apcg_tune_cache_lookup("k|a") == ((6, 512, 0, apcg.APCG_SPMV_SDIA), 29.5)
    path = str(tmp_path / "tune.tsv")
    assert apcg.apcg_tune_cache_save(path) == 2
    text = open(path).read().splitlines()
    assert text[0].startswith("#") and len(text) == 3
    apcg.apcg_tune_cache_clear()
    assert apcg.apcg_tune_cache_load(path) == 2
    assert apcg.apcg_tune_cache_lookup("batch|k|b") == ((2, 0, 1024, 1), 1.5e5)
    assert apcg.apcg_tune_cache_lookup("k|a") == ((6, 512, 0, apcg.APCG_SPMV_SDIA), 29.5)
    # a malformed file changes nothing and names its line
    bad = str(tmp_path / "bad.tsv")
    with open(bad, "w") as f:
        f.write("# header\nz|q\t1 2 3 4\t5.0\nz|r\t1 2 x 4\t5.0\n")
    with pytest.raises(apcg.ApcgError):
        apcg.apcg_tune_cache_load(bad)
    assert "line 3" in apcg.apcg_last_error()
    assert apcg.apcg_tune_cache_lookup("z|q") is None
    assert apcg.apcg_tune_cache_size() == 2
    with pytest.raises(apcg.ApcgError):
        apcg.apcg_tune_cache_load(str(tmp_path / "missing.tsv"))
    apcg.apcg_tune_cache_clear()
    assert not os.path.exists(path + ".tmp")
