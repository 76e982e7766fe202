"""Host-side checks of bench.py: the one-GPU contract and the algorithmic
bytes that the roofline figure divides by the measured launch time."""
import os
import subprocess
import sys
from types import SimpleNamespace

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr


def _pattern():
    # 3 block rows of 2 x 2 blocks, symmetric pattern:
    # row 0: columns 0 1 / row 1: 0 1 2 / row 2: 1 2
    return SimpleNamespace(n_rows=3, np=2, row_ptr=np.array([0, 2, 5, 7]),
                           col_idx=np.array([0, 1, 0, 1, 2, 1, 2]))


def test_spmv_bytes_general_storage():
    # 7 blocks of 4 doubles, 7 column indices, 4 row pointers (int32),
    # x and y of 3 x 2 doubles
    assert bench.spmv_bytes(_pattern()) == 7 * 32 + 7 * 4 + 4 * 4 + 2 * 6 * 8


def test_spmv_bytes_symmetric_storage():
    # stored blocks (column >= row): (0,0) (0,1) (1,1) (1,2) (2,2) = 5, each
    # read once; upper list: 5 column indices and 4 row pointers; lower list:
    # 4 row pointers and, for the 2 lower blocks, a column and a stored-block
    # index each; x and y
    expect = 5 * 32 + (5 * 4 + 4 * 4) + (4 * 4 + 2 * 8) + 2 * 6 * 8
    assert bench.spmv_bytes(_pattern(), sym=True) == expect
    # FP32 blocks halve the block and vector bytes only
    expect32 = 5 * 16 + (5 * 4 + 4 * 4) + (4 * 4 + 2 * 8) + 2 * 6 * 4
    assert bench.spmv_bytes(_pattern(), word=4, sym=True) == expect32
