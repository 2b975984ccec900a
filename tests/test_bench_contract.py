"""bench.py contract on the host: the one-GPU guard and the algorithmic byte and
flop counts behind its roofline line (values worked out by hand)."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402  (top level imports only the standard library)


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_tridiag_bytes_by_hand():
    # n = 3: one column (c = 0) reads the 2 x 2 trailing block (4 doubles);
    # one panel of one reflector updates the 2 x 2 block below it (read and
    # write, 8 doubles): 12 doubles
    assert bench.tridiag_bytes(np.array([3])) == 12 * 8
    # n = 18: columns 0..15 read (17 - c)^2 doubles, 2^2 + ... + 17^2 = 1784;
    # one panel of 16 reflectors leaves a 2 x 2 trailing block (8 doubles)
    assert bench.tridiag_bytes(np.array([18])) == (1784 + 8) * 8
    # n = 34: columns 0..31, 2^2 + ... + 33^2 = 12528; panels end at 16 and 32,
    # leaving 18 x 18 and 2 x 2 trailing blocks: 2 (324 + 4) = 656
    assert bench.tridiag_bytes(np.array([34])) == (12528 + 656) * 8
    # sums over subgraphs; sizes below 3 have no reflector
    assert bench.tridiag_bytes(np.array([3, 18, 1, 2])) == (12 + 1792) * 8


def test_algorithmic_flops_by_hand():
    w = bench.algorithmic_work(np.array([2, 3]), np.array([1, 2]))
    assert w["k_xy"] == (8 + 4) + (27 + 9)          # n^3 + n^2 per subgraph
    assert w["k_density_rows"] == 4 * 1 * 4 + 4 * 2 * 9  # 4 c n^2
    assert np.isclose(w["k_tridiag"], 4.0 / 3.0 * (8 + 27))


def test_minimum_bytes_by_hand():
    # eigensolve: the matrix in, the vectors out, 16 n^2 bytes
    assert bench.eigensolve_min_bytes(np.array([2, 3])) == 16 * 4 + 16 * 9
    # congruence per perturbation: 16 n^2 + 8 n + 8 c n
    assert bench.congruence_min_bytes(np.array([3]), np.array([2])) == 16 * 9 + 8 * 3 + 8 * 6
