"""Pins of the oracle's spectral Crank-Nicolson field step and Nyquist projection."""
import math

import numpy as np
import pytest

import oracle as O


def _sim(dim, n, length, dt=0.2, project=1):
    cfg = O.make_config(dim, n, (0, 0, 0), length, dt, project=project)
    s = O.OracleSim(cfg)
    s.load_particles(np.zeros((dim, 0)), np.zeros((3, 0)), np.zeros(0))
    return s


def _grid(n, length, dim):
    h = [length[i] / n[i] for i in range(dim)]
    g = np.meshgrid(*[np.arange(n[i]) * h[i] for i in range(dim)], indexing="ij")
    return [np.transpose(gg, tuple(reversed(range(dim)))).ravel() for gg in g]


def test_vacuum_mode_cn_phase():
    """A single vacuum mode has |lambda| = 1 and phase 2 atan(kappa |k| dt / 2) per step."""
    n, length, dt = (16, 8), (4.0, 3.0), 0.37
    s = _sim(2, n, length, dt)
    X, Y = _grid(n, length, 2)
    k = (2 * math.pi * 2 / length[0], 2 * math.pi * 1 / length[1])
    mode = np.cos(k[0] * X + k[1] * Y)
    A0 = np.zeros((3, X.size))
    A0[2] = mode  # A_z: divergence free, no charge coupling
    s.load_potentials(A0, np.zeros_like(A0))
    s.initialize()
    theta = 2 * math.atan(math.hypot(*k) * dt / 2)
    for nstep in range(1, 31):
        s.cn_advance(np.zeros((3, X.size)))
        A = s.read_field("A")
        assert np.allclose(A[2], math.cos(nstep * theta) * mode, atol=1e-12)
    # field energy of the free wave is conserved exactly by CN
    d = s.diagnostics()
    assert d["energy_rel"] < 1e-13


@pytest.mark.parametrize("dim,n,length", [(1, (32,), (5.0,)), (2, (16, 8), (3.0, 2.0)),
                                          (3, (8, 8, 4), (2.0, 2.0, 1.5))])
def test_field_work_balance_and_constraints(dim, n, length):
    """W^{n+1} - W^n = -dt <J, E^{n+1/2}> for any projected current, and the Gauss and
    Lorenz residuals stay at roundoff when they vanish initially."""
    s = _sim(dim, n, length, dt=0.15)
    ng = int(np.prod(n))
    s.load_potentials(np.zeros((3, ng)), np.zeros((3, ng)))
    s.initialize()
    rng = np.random.default_rng(dim)
    for step in range(6):
        j = rng.normal(size=(3, ng))
        # project j so that <j, E> uses the retained space only
        jp = np.stack([np.real(np.fft.ifftn(_proj(np.fft.fftn(c.reshape(tuple(reversed(n)))), n)))
                       .ravel() for c in j])
        E0 = s.read_field("E")
        W0 = s.diagnostics()["field"]
        s.cn_advance(jp)
        E1 = s.read_field("E")
        d = s.diagnostics()
        dV = float(np.prod([length[i] / n[i] for i in range(dim)]))
        rhs = -0.15 * float((jp * 0.5 * (E0 + E1)).sum()) * dV
        assert abs((d["field"] - W0) - rhs) < 1e-12 * max(1.0, abs(d["field"]))
        assert d["gauss_rms"] < 1e-12 and d["lorenz_rms"] < 1e-12


def _proj(F, n):
    F = F.copy()
    dim = len(n)
    for ax in range(dim):
        nn = n[dim - 1 - ax]  # numpy axis order is reversed (x fastest)
        if nn % 2 == 0:
            idx = [slice(None)] * dim
            idx[ax] = nn // 2
            F[tuple(idx)] = 0
    return F


def test_nyquist_counterexample_and_projection():
    """A_x = a (-1)^{j_y}: zero mesh curl, yet the spline interpolant has d_y A_x != 0 and
    generates a nonzero skew matrix; the projector removes the component."""
    n, length = (8, 8), (2.0, 2.0)
    ng = 64
    jy = np.repeat(np.arange(8), 8)  # node g = ix + 8 iy
    a = 0.3
    A = np.zeros((3, ng))
    A[0] = a * (-1.0) ** jy
    s = _sim(2, n, length, project=0)
    s.load_potentials(A, np.zeros_like(A))
    s.initialize()
    B = s.read_field("B")
    assert np.abs(B).max() < 1e-14  # mesh curl vanishes (Nyquist symbol is zero)
    cfg = O.make_config(2, n, (0, 0, 0), length, 0.1)
    z = np.zeros((3, ng))
    o = O.orbit_eval(cfg, np.zeros((2, ng)), A, A, z, [0.61, 0.77], [0, 0, 0], -1.0, 1.0,
                     [0.0, 0.0, 0.0])
    assert abs(o["Beff"][2]) > 1e-3  # the interpolant's derivative rotates particles
    sp = _sim(2, n, length, project=1)
    sp.load_potentials(A, np.zeros_like(A))
    sp.initialize()
    assert np.abs(sp.read_field("A")).max() < 1e-15


def test_projected_work_identity():
    """<P J, E> = <J, P E> = <J, E> when E lies in the retained space."""
    n = (8, 16)
    rng = np.random.default_rng(3)
    J = rng.normal(size=(16, 8))
    E = np.real(np.fft.ifftn(_proj(np.fft.fftn(rng.normal(size=(16, 8))), n)))
    PJ = np.real(np.fft.ifftn(_proj(np.fft.fftn(J), n)))
    assert abs((PJ * E).sum() - (J * E).sum()) < 1e-12


def test_initial_constraints_with_charge_and_potentials():
    """Initialization solves Gauss's law for phi and sets psi from the Lorenz gauge."""
    dim, n, length = 2, (16, 16), (3.2, 3.2)
    cfg = O.make_config(dim, n, (0, 0, 0), length, 0.05)
    s = O.OracleSim(cfg)
    rng = np.random.default_rng(0)
    npart = 500
    x = rng.uniform(0, 3.2, (2, npart))
    u = rng.normal(size=(3, npart)) * 0.3
    q = -np.full(npart, 3.2 * 3.2 / npart)
    s.load_particles(x, u, q)
    A0 = rng.normal(size=(3, 256)) * 0.01
    U0 = rng.normal(size=(3, 256)) * 0.01
    s.load_potentials(A0, U0)
    s.initialize()
    d = s.diagnostics()
    assert d["gauss_rms"] < 1e-12 and d["lorenz_rms"] < 1e-12
    rho = s.read_field("rho")
    assert abs(rho.sum()) < 1e-10  # neutral including the background
