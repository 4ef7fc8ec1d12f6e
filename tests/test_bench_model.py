"""Host logic of bench.py: the algorithmic work counted per orbit evaluation, for both
particle shapes, against totals counted by hand from the per-point terms its docstring
lists, and against the per-evaluation work of the five run configurations (1D, 2D at
two segment lengths, 3D) at GL(d+1) and GL8."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_quadratic_counts_2d_gl3():
    # per point: gathers 2 * 9 * 15 = 270, weights 2 * 20 + 27 + 2 * 6 = 79;
    # endpoint 2 * 3 * 9 + 40 + 27 = 121; push and secant 250
    assert bench.flops_per_eval(2, 1.0, 3) == 3 * 349 + 121 + 250


def test_linear_counts_2d_gl2():
    # per point: gathers 2 * 4 * 15 = 120, weights 2 * 6 + 12 + 2 * 6 = 36;
    # endpoint 2 * 3 * 4 + 12 + 12 = 48
    assert bench.flops_per_eval(2, 1.0, 2, shape=1) == 2 * 156 + 48 + 250


@pytest.mark.parametrize("d, seg, gl_d1, gl8", [
    (1, 1.36, 489, 1093),     # 1D two-stream runs
    (2, 1.01, 1428, 3191),    # 2D, short orbits
    (2, 1.18, 1606, 3666),    # 2D mixed beams
    (3, 1.16, 7023, 13454),   # 3D Weibel
])
def test_counts_per_configuration(d, seg, gl_d1, gl8):
    assert abs(bench.flops_per_eval(d, seg, d + 1) - gl_d1) < 1.0
    assert abs(bench.flops_per_eval(d, seg, 8) - gl8) < 1.0


def test_bytes_per_particle_and_node():
    assert bench.bytes_per_particle(2, 8) == 136 and bench.bytes_per_particle(2, 4) == 84
    assert bench.bytes_per_node(2) == 8 * 11 + 48
