"""The entry point that allocates nothing (gmhc_orbit_pass_static) against the workspace
entry point it varies (gmhc_orbit_pass_frozen), through the C ABI.

Both run the same kernels on the same particle order and inputs, so v_out, P^{n+1} and
the orbit current must agree bit for bit, and the accepted positions must be the orbit
endpoints x + dt v_in.  Two calls in a row, the second on a smaller input (fewer
particles, a smaller mesh), check that the static scratch is cleared between calls; the
limits are enforced with clear errors.
"""
import numpy as np
import pytest

from paper_2609_36383_amd import workloads as W

pytestmark = pytest.mark.gpu


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2609_36383_amd import gmhc as G
    return G, torch


def _case(G, torch, dim, n, length, num, seed, iterate):
    dt = 0.05
    gphi, An, Anp1, _ = W.random_fields(dim, n, length, seed=seed, amp=0.3)
    Uh = (Anp1 - An) / dt
    x, u, q = W.random_particles(dim, n, length, num, seed + 1, umax=0.8)
    P = np.abs(q)[None, :] * u
    vin = u / np.sqrt(1.0 + (u * u).sum(axis=0))[None, :]
    kw = dict(dim=dim, n=n, lo=(0.0,) * dim, length=length, dt=dt)
    cfg = G.make_config(**kw, gl_order=0)
    # the workspace entry point
    sim = G.Simulation(cfg, num)
    sim.load_particles(x, u, q)
    sim.set_particle_state(x, P, vin)
    sim.set_frozen_fields(gphi, An, Anp1, Uh)
    rep_ref = sim.orbit_pass_frozen(iterate=iterate)
    vref, Pref, Jref = sim.read_pass()
    sim.close()
    # the static entry point on device tensors
    dev = torch.device("cuda:0")
    T = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device=dev)  # noqa: E731
    tx, tP, tq, tv = T(x), T(P), T(q), T(vin)
    fields = [T(a) for a in (gphi, An, Anp1, Uh)]
    vout = torch.empty_like(tv)
    Pn1 = torch.empty_like(tP)
    xn1 = torch.empty_like(tx)
    J = torch.empty((3, int(np.prod(n))), dtype=torch.float64, device=dev)
    stream = torch.cuda.Stream(device=dev)
    stream.wait_stream(torch.cuda.current_stream(dev))
    rep = G.orbit_pass_static(cfg, tx, tP, tq, tv, *fields, vout, Pn1, xn1, J, iterate=iterate, stream=stream)
    torch.cuda.synchronize()
    vs, Ps, xs, Js = (t.cpu().numpy() for t in (vout, Pn1, xn1, J))
    assert rep["failed"] == 0 and rep_ref["failed"] == 0
    assert rep["evaluations"] == rep_ref["evaluations"] and rep["segments"] == rep_ref["segments"]
    assert np.array_equal(vs, vref) and np.array_equal(Ps, Pref) and np.array_equal(Js, Jref)
    # accepted positions: the orbit endpoint x + dt v_in, wrapped (v_in = v_out within the
    # inner tolerance when iterating, the given warm start otherwise)
    vacc = vout.cpu().numpy() if iterate else vin
    for l in range(dim):
        d = np.abs((x[l] + dt * vacc[l]) % length[l] - xs[l])
        d = np.minimum(d, length[l] - d)
        assert d.max() <= 1e-12 * length[l] + (dt * 1e-11 if iterate else 0.0)
    return rep


@pytest.mark.parametrize("iterate", [False, True])
def test_static_pass_matches_workspace_pass_twice(iterate):
    G, torch = _gpu()
    big = _case(G, torch, 2, (64, 32), (12.8, 6.4), 70001, seed=3, iterate=iterate)
    small = _case(G, torch, 2, (16, 8), (3.2, 1.6), 1777, seed=9, iterate=iterate)
    assert big["evaluations"] > small["evaluations"]
    small3 = _case(G, torch, 3, (8, 8, 4), (1.6, 1.6, 0.8), 999, seed=21, iterate=iterate)
    assert small3["evaluations"] >= 999


def test_static_pass_limits():
    G, torch = _gpu()
    cfg = G.make_config(2, (1024, 512), (0, 0), (1.0, 1.0), 0.05)  # 2^19 nodes > the limit
    dev = torch.device("cuda:0")
    z = torch.zeros((3, 4), dtype=torch.float64, device=dev)
    f = torch.zeros((3, 1024 * 512), dtype=torch.float64, device=dev)
    with pytest.raises(G.GmhcError, match="GMHC_STATIC_MAX_NODES"):
        G.orbit_pass_static(cfg, z[:2], z, z[0], z, f[:2], f, f, f, z, z, z[:2], f)
    big_q = torch.zeros(G.STATIC_MAX_PARTICLES + 1, dtype=torch.float64, device=dev)
    cfg16 = G.make_config(2, (16, 16), (0, 0), (1.0, 1.0), 0.05)
    f16 = torch.zeros((3, 256), dtype=torch.float64, device=dev)
    with pytest.raises(G.GmhcError, match="GMHC_STATIC_MAX_PARTICLES"):
        G.orbit_pass_static(cfg16, z[:2], z, big_q, z, f16[:2], f16, f16, f16, z, z, z[:2], f16)
    cfg32 = G.make_config(2, (16, 16), (0, 0), (1.0, 1.0), 0.05, precision=G.FP32_BULK)
    with pytest.raises(G.GmhcError, match="FP64"):
        G.orbit_pass_static(cfg32, z[:2], z, z[0], z, f[:2], f, f, f, z, z, z[:2], f)
