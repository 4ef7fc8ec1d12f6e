"""Pins of the oracle's forward-mode derivatives (oracle/gmhc_tangent.cpp), CPU only.

The tangent oracle carries derivatives through a 1D, 2D or 3D run (Algorithm 1 with the orbit
maps, the GM-HC step, the secant velocity and the CN field step) by dual-number
arithmetic.  It is pinned here against what does not depend on it:
  * its values equal the main oracle's run (same step, separately written);
  * its derivatives equal central differences of the main oracle's run;
  * the derivative of the total energy is conserved: the energy theorem of the step
    (section "CN field energy and total energy theorem") holds for every value of the
    inputs, so d(K + W)/d(theta) after the run equals d(K + W)/d(theta) at the start.
    A dropped term, a wrong sign or a wrong index anywhere in the derivative of the
    push, the gathers, the deposit or the field step breaks this identity.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2609_36383_amd import workloads as W

STEPS = 3


def _case(n=16, ppc=8, length=4.0 * math.pi, gl=2):
    w = W.spec("tsi1d_big", n=(n,), ppc=ppc, length=(length,))
    x, u, q = W.particles(w)
    cfg = O.config_from_dict(W.config_dict(w), gl_order=gl)
    return w, cfg, x[0], u, q


def _directions(w, x, u, q, seed=7):
    """Seed directions: a random position field, the beam momentum u0 (u_x = +-u0) and
    the weight perturbation of mode 1 (q_j scaled by cos(k x_j + theta))."""
    rng = np.random.default_rng(seed)
    n = q.size
    L = w["length"][0]
    dx = np.zeros((3, n))
    du = np.zeros((3, 3, n))
    dq = np.zeros((3, n))
    dx[0] = 0.1 * rng.standard_normal(n)
    du[1, 0] = np.sign(u[0])
    dq[2] = 0.5 * q * np.cos(2.0 * math.pi * (x - w["lo"][0]) / L + 0.3)
    return dx, du, dq


def _main_oracle(cfg, x, u, q, steps):
    s = O.OracleSim(cfg)
    s.load_particles(x[None, :], u, q)
    s.initialize()
    d0 = s.diagnostics()
    for _ in range(steps):
        s.step()
    d = s.diagnostics()
    return np.array([d0["field"], d0["kinetic"], d["field"], d["kinetic"]])


def test_tangent_values_equal_main_oracle():
    _, cfg, x, u, q = _case()
    E, _, outer = O.tangent_run(cfg, x, u, q, STEPS)
    ref = _main_oracle(cfg, x, u, q, STEPS)
    assert outer >= STEPS
    np.testing.assert_allclose(E, ref, rtol=1e-11, atol=0)


@pytest.mark.parametrize("gl", [2, 8])
def test_tangent_equals_central_differences(gl):
    w, cfg, x, u, q = _case(gl=gl)
    dx, du, dq = _directions(w, x, u, q)
    E, dE, _ = O.tangent_run(cfg, x, u, q, STEPS, dx=dx, du=du, dq=dq)
    h = 1e-6
    for k in range(3):
        fp = _main_oracle(cfg, x + h * dx[k], u + h * du[k], q + h * dq[k], STEPS)
        fm = _main_oracle(cfg, x - h * dx[k], u - h * du[k], q - h * dq[k], STEPS)
        fd = (fp - fm) / (2.0 * h)
        # W is small against K, so each is compared on its own scale; the difference
        # quotient carries the run's solver tolerance divided by h.
        for a in (0, 2):  # field energy at the start and at the end
            assert abs(dE[a, k] - fd[a]) <= 1e-5 * abs(fd[a]) + 1e-12, (k, a, dE[a, k], fd[a])
        for a in (1, 3):  # kinetic energy
            assert abs(dE[a, k] - fd[a]) <= 1e-5 * (abs(fd[a]) + abs(dE[0, k])) + 1e-9 * E[a], (k, a)


def test_total_energy_derivative_is_conserved():
    """d(K + W) along every direction is the same after the run as at its start."""
    w, cfg, x, u, q = _case(n=32, ppc=8, length=8.0 * math.pi)
    dx, du, dq = _directions(w, x, u, q, seed=11)
    E, dE, _ = O.tangent_run(cfg, x, u, q, 6, dx=dx, du=du, dq=dq)
    start = dE[0] + dE[1]
    end = dE[2] + dE[3]
    scale = np.abs(dE).max(axis=0)
    assert np.all(np.abs(end - start) <= 1e-9 * scale), (start, end)
    # and the values conserve energy at the run's tolerance
    assert abs((E[2] + E[3]) - (E[0] + E[1])) <= 1e-11 * (E[0] + E[1])


def test_single_beam_direction_and_zero_direction():
    """Speeding up the second beam (u_x = -u0 made more negative) raises the initial
    kinetic energy, keeps the energy identity, and a zero seed gives exactly zero."""
    w, cfg, x, u, q = _case()
    n = q.size
    du = np.zeros((2, 3, n))
    du[0, 0, n // 2:] = -1.0
    E, dE, _ = O.tangent_run(cfg, x, u, q, STEPS, du=du)
    assert np.all(dE[:, 1] == 0.0)
    assert abs((dE[2, 0] + dE[3, 0]) - (dE[0, 0] + dE[1, 0])) <= 1e-9 * abs(dE[1, 0])
    assert dE[1, 0] > 0.0


def _case_nd(dim):
    if dim == 2:
        w = W.spec("weibel2d", n=(16, 16), ppc=4)
    else:
        w = W.spec("weibel3d", n=(8, 8, 8), ppc=2)
    x, u, q = W.particles(w)
    cfg = O.config_from_dict(W.config_dict(w), gl_order=dim + 1)
    rng = np.random.default_rng(3)
    n = q.size
    dx = 0.05 * rng.standard_normal((3, dim, n))
    du = 0.1 * rng.standard_normal((3, 3, n))
    dq = q * rng.standard_normal((3, n))
    return cfg, x, u, q, dx, du, dq


@pytest.mark.parametrize("dim", [2, 3])
def test_tangent_multid_values_derivatives_and_energy_identity(dim):
    """2D (16 x 16, 1024 particles) and 3D (8^3, 1024 particles), 3 and 2 steps: values
    equal the main oracle's run, the derivatives along random directions of positions,
    momenta and charges equal central differences of the main oracle, and d(K + W) is
    conserved."""
    cfg, x, u, q, dx, du, dq = _case_nd(dim)
    steps = STEPS if dim == 2 else 2
    E, dE, _ = O.tangent_run(cfg, x, u, q, steps, dx=dx, du=du, dq=dq)

    def run(xx, uu, qq):
        s = O.OracleSim(cfg)
        s.load_particles(xx, uu, qq)
        s.initialize()
        d0 = s.diagnostics()
        for _ in range(steps):
            s.step()
        d = s.diagnostics()
        return np.array([d0["field"], d0["kinetic"], d["field"], d["kinetic"]])

    np.testing.assert_allclose(E, run(x, u, q), rtol=1e-11, atol=0)
    h = 1e-6
    for k in range(3):
        fd = (run(x + h * dx[k], u + h * du[k], q + h * dq[k]) - run(x - h * dx[k], u - h * du[k], q - h * dq[k])) / (2 * h)
        assert abs(dE[2, k] - fd[2]) <= 1e-6 * abs(fd[2]), (k, dE[2, k], fd[2])
    start, end = dE[0] + dE[1], dE[2] + dE[3]
    assert np.all(np.abs(end - start) <= 1e-9 * np.abs(dE).max(axis=0))


def test_tangent_rejects_unsupported_configurations():
    _, cfg, x, u, q = _case()
    cfg.outer_scheme = 1
    with pytest.raises(O.OracleError):
        O.tangent_run(cfg, x, u, q, 1)
