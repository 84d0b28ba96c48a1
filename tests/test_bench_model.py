"""Host logic of bench.py: the algorithmic byte model behind the roofline figures, checked
against counts written out by hand for each storage form (no GPU)."""
import importlib.util
import os

import pytest

_spec = importlib.util.spec_from_file_location(
    "bench", os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "bench.py"))
bench = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(bench)


def test_spmv_bytes_diagonal_form():
    # 14 stored diagonals of n values, x read once, y written once; no indices or offsets
    n = 1081665
    assert bench.spmv_bytes(n, 28607425, 8, 0, 0, 14) == 14 * n * 8 + 2 * n * 8 == 138453120
    assert bench.spmv_bytes(n, 28607425, 4, 0, 0, 14) == 16 * n * 4


@pytest.mark.parametrize("col_bytes,tiles,extra", [(4, 0, 0), (4, 100, 4 * 101), (3, 100, 4 * 101),
                                                   (2, 100, 4 * 101 + 4 * 100), (1, 100, 4 * 101)])
def test_spmv_bytes_csr_forms(col_bytes, tiles, extra):
    # values and column indices per entry (4, 3, 2 or 1 bytes), row offsets, x and y once, the
    # tile table (and the per-tile column bases of the 16-bit form)
    n, nnz = 1000, 27000
    assert bench.spmv_bytes(n, nnz, 8, col_bytes, tiles) == nnz * (8 + col_bytes) + n * (4 + 16) + extra


def test_iteration_bytes_counts_every_level():
    info = {"n": [1000, 100, 10], "nnz": [27000, 2000, 100], "nlevels": 3, "p_nnz": [1000, 100, 0],
            "col_bytes": [0, 2, 4], "tiles": [0, 5, 1], "col_bytes_p": [2, 4, 0], "col_bytes_r": [4, 4, 0],
            "diags": [14, 0, 0]}
    s = 8
    want = bench.spmv_bytes(1000, 27000, 8, 0, 0, 14)                      # outer product
    for k, (n, nnz, nc) in enumerate([(1000, 27000, 100), (100, 2000, 10)]):
        want += 4 * bench.spmv_bytes(n, nnz, s, info["col_bytes"][k], info["tiles"][k], info["diags"][k])
        pn = info["p_nnz"][k]
        want += pn * (s + info["col_bytes_r"][k]) + nc * (4 + s) + n * s
        want += pn * (s + info["col_bytes_p"][k]) + n * (4 + 2 * s) + nc * s
        want += 6 * n * s
    want += 10 * 1000 * 8 + 10 * 10 * 8
    assert bench.iteration_bytes(info, s) == want
