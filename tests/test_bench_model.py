"""Host logic of bench.py: the algorithmic work counted per orbit evaluation and per
deposit sweep, for both particle shapes, against totals counted by hand from the
per-point and per-node terms the docstrings list (2D, one segment per evaluation)."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_quadratic_counts_2d_gl3():
    # per node 1 + 2 + 4 + 21 + 1 = 29; per point 20 + 3 + 9 * 29 = 284;
    # endpoint 9 * 7 + 12 = 75; push and secant 250
    assert bench.flops_per_eval(2, 1.0, 3) == 3 * 284 + 75 + 250
    # deposit: per point 20 + 9 * 2 = 38; per particle 9 * 12
    assert bench.deposit_flops(2, 1.0, 3) == 3 * 38 + 108


def test_linear_counts_2d_gl2():
    # 2 support nodes per axis, 3 flops per axis for the 1D weights
    assert bench.flops_per_eval(2, 1.0, 2, shape=1) == 2 * (6 + 3 + 4 * 29) + (4 * 7 + 12) + 250
    assert bench.deposit_flops(2, 1.0, 2, shape=1) == 2 * (6 + 4 * 2) + 4 * 12


def test_bytes_per_particle_and_node():
    assert bench.bytes_per_particle(2, 8) == 136 and bench.bytes_per_particle(2, 4) == 84
    assert bench.bytes_per_node(2) == 8 * 11 + 48
