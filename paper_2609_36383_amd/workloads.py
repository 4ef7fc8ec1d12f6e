"""Seeded synthetic workloads: run parameters and initial particle arrays.

This module only draws inputs.  It holds none of the method's arithmetic (no
deposit, shape, push or field solve), so both the GPU library and the independent
CPU checker can be fed from it.

Workloads (nondimensional units, kappa = sigma1 = sigma2 = rho0 = 1, q/m = -1,
m = |q|, uniform immobile neutralizing background):

  tsi1d     1D cold relativistic two-stream, 64 cells, L = 4 pi (k = 0.5), beams
            u_x = +-1, 32 particles/cell/beam (4096), quiet start with a seeded 1e-3
            weight perturbation at mode 1, dt = 0.1, 200 steps.
  weibel2d  2D Weibel/filamentation, 128 x 128, dx = 0.2, beams u_z = +-0.5 with
            Gaussian spread 0.01, 64 particles/cell (1,048,576), dt = 0.05, 500 steps.
  mixed2d   2D two-stream/Weibel mixed, 512 x 512, dx = 0.2, beams u_x = +-1 with
            spread 0.02, 256 particles/cell (67,108,864), dt = 0.05, 100 steps.
  tsi1d_big 1D two-stream, 1024 cells, L = 64 pi, beams u_x = +-1, 1024 particles/
            cell (1,048,576), 1e-3 weight perturbation at modes 1-8 with seeded
            phases, dt = 0.1, 50 steps.
  weibel3d  3D Weibel, 128^3, dx = 0.2, beams u_z = +-0.8 with spread 0.01,
            32 particles/cell (67,108,864), dt = 0.05, 50 steps.
  tsi       the paper's cold relativistic two-stream run: [-4 pi, 4 pi]^3 on 32^3
            (dx = pi/4), 10 pairs/cell (655,360), beams v = +-0.9 x, the growing
            eigenmode of k_x = 1/4 with grid charge density 5e-3 cos(k x') (E_x =
            0.02 sin(k x'), x' = x - lo), dt = 0.1 (TSI-0.1; dt = 0.3 is TSI-0.3), 600
            steps, the paper's tolerances.  eig_gamma defaults to the printed growth rate.
  wbi       the paper's cold relativistic Weibel/filamentation run: [-pi, pi]^3 on 32^3
            (dy = pi/16), 25 pairs/cell (1,638,400), beams v = +-0.9 x, the growing
            eigenmode of k_y = 1 with B0 = 1e-4 in the fields and the particles, dt = 0.04
            (WBI-0.04; dt = 0.2 is WBI-0.2), 2500 steps, the paper's tolerances.
            eig_gamma defaults to the printed growth rate; potentials(w) gives A0, U0.

Beam loading: 1D workloads, tsi and wbi use a quiet start (both beams share the positions
x_j = lo + (j + 1/2) L / N_beam, weights carry the density perturbation).  2D and 3D
workloads place ppc/2 symmetry-related pairs per cell at uniform random positions;
the two members of a pair share the position and have opposite momenta
+-(u_d e + du), du ~ N(0, sigma^2 I), so the initial current and net momentum vanish.
tsi and wbi place the pairs of every cell evenly along x, x = lo + (i + (j + 1/2) / npair) dx,
at the cell centre in y and z; the two members of a pair share the position.  This loading
reproduces the growth rates the paper prints for both runs.  Eigenmode perturbations are
applied to the velocities (u = gamma(v) v afterwards) and to the weights.
"""
import math

import numpy as np

COMMON = dict(kappa=1.0, sigma1=1.0, sigma2=1.0)


def _tol(fp32_bulk=False):
    # FP32-bulk: the inner test stops at 1e-6 relative, and the per-node outer residual
    # then carries noise of about 5e-7 of the node current (measured), so the outer
    # tests sit a factor 20 above that floor.
    if fp32_bulk:
        return dict(tol_outer_abs=1e-7, tol_outer_rel=1e-5, tol_inner_abs=1e-10, tol_inner_rel=1e-6)
    return dict(tol_outer_abs=1e-14, tol_outer_rel=1e-12, tol_inner_abs=1e-14, tol_inner_rel=1e-12)


WORKLOADS = {
    "tsi1d": dict(kind="quiet1d", dim=1, n=(64,), dx=None, length=(4.0 * math.pi,), dt=0.1, steps=200,
                  ppc=64, u_drift=1.0, eps=1e-3, modes=(1,), seed=1),
    "weibel2d": dict(kind="pairs", dim=2, n=(128, 128), dx=0.2, dt=0.05, steps=500, ppc=64,
                     drift_axis=2, u_drift=0.5, u_spread=0.01, seed=2),
    "mixed2d": dict(kind="pairs", dim=2, n=(512, 512), dx=0.2, dt=0.05, steps=100, ppc=256,
                    drift_axis=0, u_drift=1.0, u_spread=0.02, seed=3),
    "tsi1d_big": dict(kind="quiet1d", dim=1, n=(1024,), dx=None, length=(64.0 * math.pi,), dt=0.1,
                      steps=50, ppc=1024, u_drift=1.0, eps=1e-3, modes=tuple(range(1, 9)), seed=4),
    "weibel3d": dict(kind="pairs", dim=3, n=(128, 128, 128), dx=0.2, dt=0.05, steps=50, ppc=32,
                     drift_axis=2, u_drift=0.8, u_spread=0.01, seed=5),
    "tsi": dict(kind="tsi", dim=3, n=(32, 32, 32), dx=None, lo=(-4.0 * math.pi,) * 3,
                length=(8.0 * math.pi,) * 3, dt=0.1, steps=600, ppc=20, v0=0.9, alpha=5e-3, kx_mode=1,
                eig_gamma=9.109138040e-2,  # Gamma_TS as the two-stream subsection prints it
                tol=dict(tol_outer_abs=1e-13, tol_outer_rel=1e-11, tol_inner_abs=1e-13, tol_inner_rel=1e-11)),
    "wbi": dict(kind="wbi", dim=3, n=(32, 32, 32), dx=None, lo=(-math.pi,) * 3, length=(2.0 * math.pi,) * 3,
                dt=0.04, steps=2500, ppc=50, v0=0.9, B0=1e-4, ky_mode=1,
                eig_gamma=5.103647904e-1,  # Gamma_W as the Weibel subsection prints it
                tol=dict(tol_outer_abs=1e-13, tol_outer_rel=1e-11, tol_inner_abs=1e-14, tol_inner_rel=1e-12)),
}


def spec(name, **over):
    """Workload description with optional overrides (e.g. a smaller n or ppc for tests)."""
    w = dict(WORKLOADS[name])
    w.update(over)
    w["name"] = name
    d = w["dim"]
    if w["kind"] == "pairs":
        w["length"] = tuple(w["n"][i] * w["dx"] for i in range(d))
    w["lo"] = tuple(w["lo"]) if "lo" in w else (0.0,) * d
    w["n"] = tuple(int(v) for v in w["n"])
    ncell = int(np.prod(w["n"]))
    w["num_particles"] = ncell * int(w["ppc"])
    return w


def config_dict(w, fp32_bulk=False):
    """Mesh, physics and solver settings of a workload as plain keyword values."""
    d = dict(dim=w["dim"], n=tuple(w["n"]), lo=tuple(w["lo"]), length=tuple(w["length"]), dt=w["dt"])
    d.update(COMMON)
    d.update(w["tol"] if "tol" in w and not fp32_bulk else _tol(fp32_bulk))
    d.update(max_outer=80, max_inner=64, beta=1.0)
    return d


def particles(w):
    """Initial arrays (x [d][N], u = p/(m kappa) [3][N], q [N]) of a workload."""
    if w["kind"] == "quiet1d":
        return _quiet1d(w)
    if w["kind"] == "wbi":
        return _wbi(w)
    if w["kind"] == "tsi":
        return _tsi(w)
    return _pairs(w)


def potentials(w):
    """Initial potentials (A0, U0) [3][Ng] of a workload, or None when they start at zero."""
    if w["kind"] != "wbi":
        return None
    n = w["n"]
    ky = 2.0 * math.pi * w["ky_mode"] / w["length"][1]
    y = w["lo"][1] + np.arange(n[1]) * (w["length"][1] / n[1])
    # node g = i0 + n0 (i1 + n1 i2): the y index is (g // n0) % n1
    ng = int(np.prod(n))
    yg = y[(np.arange(ng) // n[0]) % n[1]]
    A0 = np.zeros((3, ng))
    U0 = np.zeros((3, ng))
    A0[0] = w["B0"] / ky * np.cos(ky * yg)
    U0[0] = w["eig_gamma"] * A0[0]
    return A0, U0


def _pairs_along_x(w):
    """Pair positions [d][ncell npair]: npair per cell evenly along x, cell centre in y, z."""
    n, L, lo = w["n"], w["length"], w["lo"]
    d = len(n)
    npair = w["ppc"] // 2
    ncell = int(np.prod(n))
    cells = np.repeat(np.arange(ncell, dtype=np.int64), npair)
    sub = np.tile(np.arange(npair, dtype=np.int64), ncell)
    pos = []
    rem = cells
    for i in range(d):
        ci = rem % n[i]
        rem = rem // n[i]
        frac = (sub + 0.5) / npair if i == 0 else np.full(sub.size, 0.5)
        pos.append(lo[i] + (ci + frac) * (L[i] / n[i]))
    return pos


def _tsi(w):
    """The paper's two-stream eigenmode loading.  For the gathered field chi E (E = E0
    sin(k x'), E0 = sigma1 alpha rho0 / k, chi = sinc(k dx / 2)^3) and stream s = +-1 with
    w_s = i Gamma - k s v0, the linear cold-fluid response is dv_s = i (q/m) chi E_c /
    (g0^3 w_s) (E_c = -i E0 the complex amplitude) and dn_s = k dv_s / w_s: velocity s v0 +
    Re(dv_s e^{i k x'}) along x and relative weight 1 + Re(dn_s e^{i k x'})."""
    if not w.get("eig_gamma"):
        raise ValueError("tsi needs eig_gamma (the two-stream growth rate)")
    n, L, lo = w["n"], w["length"], w["lo"]
    d = len(n)
    pos = _pairs_along_x(w)
    v0, G = w["v0"], w["eig_gamma"]
    g0 = 1.0 / math.sqrt(1.0 - v0 * v0)
    k = 2.0 * math.pi * w["kx_mode"] / L[0]
    dx = L[0] / n[0]
    z = 0.5 * k * dx
    chi = (math.sin(z) / z) ** 3
    Ec = -1j * w["alpha"] / k  # sigma1 = rho0 = 1
    ph = np.exp(1j * k * (pos[0] - lo[0]))
    m = pos[0].size
    xs = np.empty((d, 2 * m))
    u = np.zeros((3, 2 * m))
    q = np.empty(2 * m)
    qc = float(np.prod([L[i] / n[i] for i in range(d)])) / w["ppc"]
    for s, sl in ((1.0, slice(0, None, 2)), (-1.0, slice(1, None, 2))):
        for i in range(d):
            xs[i, sl] = pos[i]
        ws = 1j * G - k * s * v0
        dv = 1j * (-1.0) * chi * Ec / (g0 ** 3 * ws)
        vx = s * v0 + np.real(dv * ph)
        u[0, sl] = vx / np.sqrt(1.0 - vx * vx)
        q[sl] = -qc * (1.0 + np.real(k * dv / ws * ph))
    return xs, u, q


def _wbi(w):
    """The paper's Weibel eigenmode loading: for stream s = +-1 at height y,
      v_x = s v0 + chi B0 cos(k y) / (k g0^3),  v_y = s chi v0 B0 sin(k y) / (g0 Gamma),
      weight 1 - s chi v0 k B0 cos(k y) / (g0 Gamma^2),
    with chi = sinc(k dy / 2)^3 and Gamma = eig_gamma (from the caller)."""
    if not w.get("eig_gamma"):
        raise ValueError("wbi needs eig_gamma (the Weibel growth rate)")
    n, L, lo = w["n"], w["length"], w["lo"]
    dx = [L[i] / n[i] for i in range(3)]
    pos = _pairs_along_x(w)
    v0, B0, G = w["v0"], w["B0"], w["eig_gamma"]
    g0 = 1.0 / math.sqrt(1.0 - v0 * v0)
    k = 2.0 * math.pi * w["ky_mode"] / L[1]
    z = 0.5 * k * dx[1]
    chi = (math.sin(z) / z) ** 3
    cy, sy = np.cos(k * pos[1]), np.sin(k * pos[1])
    xs = np.empty((3, 2 * pos[0].size))
    u = np.zeros((3, 2 * pos[0].size))
    q = np.empty(2 * pos[0].size)
    qc = float(np.prod(dx)) / w["ppc"]
    for s, sl in ((1.0, slice(0, None, 2)), (-1.0, slice(1, None, 2))):
        for i in range(3):
            xs[i, sl] = pos[i]
        vx = s * v0 + chi * B0 * cy / (k * g0 ** 3)
        vy = s * chi * v0 * B0 * sy / (g0 * G)
        gam = 1.0 / np.sqrt(1.0 - vx * vx - vy * vy)
        u[0, sl] = gam * vx
        u[1, sl] = gam * vy
        q[sl] = -qc * (1.0 - s * chi * v0 * k * B0 * cy / (g0 * G * G))
    return xs, u, q


def _quiet1d(w):
    L = w["length"][0]
    lo = w["lo"][0]
    nb = w["n"][0] * w["ppc"] // 2
    rng = np.random.default_rng(w["seed"])
    theta = 2.0 * math.pi * rng.random(len(w["modes"]))
    xj = lo + (np.arange(nb) + 0.5) * (L / nb)
    u = np.zeros((3, 2 * nb))
    u[0, :nb] = w["u_drift"]
    u[0, nb:] = -w["u_drift"]
    x = np.concatenate([xj, xj])[None, :]
    if w.get("eig_gamma"):
        return x, u, _eigen1d(w, xj, u)
    pert = np.zeros(nb)
    for mth, th in zip(w["modes"], theta):
        pert += np.cos(2.0 * math.pi * mth / L * (xj - lo) + th)
    wj = 0.5 * (L / nb) * (1.0 + w["eps"] * pert)
    q = -np.concatenate([wj, wj])
    return np.ascontiguousarray(x), u, q


def quiet1d_parts(w):
    """Pieces of the quiet 1D two-beam start of a "quiet1d" workload, for callers that
    build the particles from parameters: the beam positions xj [nb] (both beams share
    them), and the per-mode weight patterns cos(2 pi m (xj - lo) / L + theta_m)
    [nmodes][nb] with the workload's seeded phases.  The particles are x = (xj, xj),
    u_x = (+u_drift, -u_drift), q = -(w, w) with w = (L / nb) / 2 (1 + sum_m eps_m pattern_m)."""
    L = w["length"][0]
    lo = w["lo"][0]
    nb = w["n"][0] * w["ppc"] // 2
    rng = np.random.default_rng(w["seed"])
    theta = 2.0 * math.pi * rng.random(len(w["modes"]))
    xj = lo + (np.arange(nb) + 0.5) * (L / nb)
    pat = np.stack([np.cos(2.0 * math.pi * m / L * (xj - lo) + th) for m, th in zip(w["modes"], theta)])
    return xj, pat


def _eigen1d(w, xj, u):
    """Cold-fluid growing eigenmode of mode 1 for two equal electron beams (q/m = -1).

    The caller supplies the growth rate ``eig_gamma`` and the field amplitude ``eig_E``
    (E_x = eig_E sin(k x) after the field solve).  For beam s with drift s v0 and
    w' = i Gamma - k s v0, linear cold-fluid theory gives the velocity perturbation
    dv = i (q/m) chi E / (g0^3 w') (chi = sinc(k dx / 2)^3 is the gathered-field factor)
    and the relative density (weight) perturbation k dv / w'.  The perturbation is
    applied to the velocity (u = gamma(v) v), as for the tsi workload.  Modifies ``u``
    in place and returns the charges.
    """
    L = w["length"][0]
    nb = xj.size
    u0 = w["u_drift"]
    g0 = math.sqrt(1.0 + u0 * u0)
    v0 = u0 / g0
    k = 2.0 * math.pi / L
    z = 0.5 * k * L / w["n"][0]
    chi = (math.sin(z) / z) ** 3
    E1 = -1j * w["eig_E"]
    phase = np.exp(1j * k * (xj - w["lo"][0]))
    q = np.empty(2 * nb)
    w0 = 0.5 * (L / nb)
    for s, sl in ((1.0, slice(0, nb)), (-1.0, slice(nb, 2 * nb))):
        wp = 1j * w["eig_gamma"] - k * s * v0
        dv = 1j * (-1.0) * chi * E1 / (g0 ** 3 * wp)
        vx = s * v0 + np.real(dv * phase)
        u[0, sl] = vx / np.sqrt(1.0 - vx * vx)
        q[sl] = -w0 * (1.0 + np.real(k * dv / wp * phase))
    return q


def _pairs(w):
    d = w["dim"]
    n = w["n"]
    ncell = int(np.prod(n))
    npair = w["ppc"] // 2
    dx = [w["length"][i] / n[i] for i in range(d)]
    cellvol = float(np.prod(dx))
    rng = np.random.default_rng(w["seed"])
    cells = np.repeat(np.arange(ncell, dtype=np.int64), npair)
    idx = []
    rem = cells
    for i in range(d):
        idx.append(rem % n[i])
        rem = rem // n[i]
    xs = np.empty((d, 2 * cells.size))
    for i in range(d):
        pos = w["lo"][i] + (idx[i] + rng.random(cells.size)) * dx[i]
        xs[i, 0::2] = pos
        xs[i, 1::2] = pos
    du = rng.normal(0.0, w["u_spread"], size=(3, cells.size))
    du[w["drift_axis"]] += w["u_drift"]
    u = np.empty((3, 2 * cells.size))
    u[:, 0::2] = du
    u[:, 1::2] = -du
    q = np.full(2 * cells.size, -cellvol / w["ppc"])
    return xs, u, q


def random_fields(dim, n, length, seed, amp=1.0, modes=3):
    """Smooth random periodic mesh arrays (sums of a few low Fourier modes), for tests.

    Returns gradphi-like [d][Ng] and three [3][Ng] arrays drawn independently.
    """
    rng = np.random.default_rng(seed)
    shape = tuple(n[i] for i in range(dim))
    grids = np.meshgrid(*[np.arange(n[i]) * (length[i] / n[i]) for i in range(dim)], indexing="ij")

    def one():
        f = np.zeros(shape)
        for _ in range(modes):
            kk = [2.0 * math.pi * rng.integers(-2, 3) / length[i] for i in range(dim)]
            ph = rng.random() * 2.0 * math.pi
            arg = sum(kk[i] * grids[i] for i in range(dim)) + ph
            f += amp * rng.normal() * np.cos(arg)
        # node order: x fastest
        return np.ascontiguousarray(np.transpose(f, axes=tuple(reversed(range(dim)))).ravel())

    gphi = np.stack([one() for _ in range(dim)])
    An = np.stack([one() for _ in range(3)])
    Anp1 = np.stack([one() for _ in range(3)])
    Uh = np.stack([one() for _ in range(3)])
    return gphi, An, Anp1, Uh


def random_particles(dim, n, length, num, seed, umax=1.0):
    """Random positions in the box, momenta u in [-umax, umax]^3 and weights, for tests."""
    rng = np.random.default_rng(seed)
    x = np.stack([rng.random(num) * length[i] for i in range(dim)])
    u = (2.0 * rng.random((3, num)) - 1.0) * umax
    q = -(0.5 + rng.random(num)) * 0.01
    return x, u, q
