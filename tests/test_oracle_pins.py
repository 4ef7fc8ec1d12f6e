"""Pins of the CPU oracle's building blocks against library routines, closed forms,
brute force and the exact identities the paper proves (no GPU involved)."""
import math

import numpy as np
import pytest
from scipy.interpolate import BSpline

import oracle as O
from paper_2609_36383_amd import workloads as W


def cfg_for(dim, n=(8, 8, 8), length=(2.0, 2.5, 3.0), dt=0.3, gl=8):
    return O.make_config(dim, n, (0.0, 0.0, 0.0), length, dt, gl_order=gl)


# ---- Gauss-Legendre rule ------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8])
def test_gl_rule_matches_numpy(n):
    x, w = O.gl_rule(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, 0.5 * (xr + 1.0), atol=1e-15, rtol=0)
    assert np.allclose(w, 0.5 * wr, atol=1e-15, rtol=0)
    for k in range(2 * n):  # exact for degree <= 2n-1
        assert abs(np.dot(w, x ** k) - 1.0 / (k + 1)) < 1e-14


# ---- quadratic B-spline ---------------------------------------------------------------

def test_shape_matches_cox_de_boor():
    ref = BSpline.basis_element([-1.5, -0.5, 0.5, 1.5], extrapolate=False)
    dref = ref.derivative()
    for xi in np.linspace(-1.49, 1.49, 301):
        S, dS = O.shape(xi)
        assert abs(S - ref(xi)) < 1e-15
        assert abs(dS - dref(xi)) < 1e-14
    assert O.shape(1.6)[0] == 0.0 and O.shape(-2.0)[0] == 0.0


def test_shape_special_values_and_partition_of_unity():
    assert O.shape(0.0) == (0.75, 0.0)
    assert O.shape(0.5)[0] == 0.5 and O.shape(-0.5)[0] == 0.5
    assert O.shape(1.0)[0] == 0.125 and O.shape(-1.0)[0] == 0.125
    assert O.shape(1.5) == (0.0, 0.0)
    rng = np.random.default_rng(0)
    for xi in rng.uniform(-5, 5, 200):
        g = np.arange(math.floor(xi) - 2, math.floor(xi) + 3)
        vals = [O.shape(xi - gg) for gg in g]
        assert abs(sum(v[0] for v in vals) - 1.0) < 1e-15
        assert abs(sum(v[1] for v in vals)) < 1e-14


def test_shape_is_c1_at_knots():
    for k in (-1.5, -0.5, 0.5, 1.5):
        e = 1e-12
        Sl, dSl = O.shape(k - e)
        Sr, dSr = O.shape(k + e)
        assert abs(Sl - Sr) < 1e-11 and abs(dSl - dSr) < 1e-11


# ---- FFT ------------------------------------------------------------------------------

@pytest.mark.parametrize("dim,n", [(1, (64,)), (2, (16, 8)), (3, (8, 4, 16))])
def test_fft_matches_numpy(dim, n):
    cfg = O.make_config(dim, n + (1,) * (3 - dim), (0, 0, 0), (1, 1, 1), 0.1)
    rng = np.random.default_rng(1)
    shape = tuple(reversed(n))  # x fastest
    a = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    f = O.fft(cfg, a)
    assert np.allclose(f, np.fft.fftn(a), atol=1e-12 * np.abs(a).sum() / a.size ** 0.5)
    b = O.fft(cfg, f, inverse=True)
    assert np.allclose(b, a, atol=1e-13)


# ---- knot split and orbit quadrature --------------------------------------------------

def test_knot_split_hand_cases():
    cfg = O.make_config(1, (16, 1, 1), (0, 0, 0), (16.0, 1, 1), 0.1)  # h = 1, knots at j + 1/2
    s = O.knot_split(cfg, [2.2], [2.0])  # 2.2 -> 4.2 crosses 2.5, 3.5
    assert np.allclose(s, [0.0, 0.15, 0.65, 1.0])
    s = O.knot_split(cfg, [2.5], [0.5])  # starts on a knot: s = 0 is not a crossing
    assert np.allclose(s, [0.0, 1.0])
    s = O.knot_split(cfg, [15.8], [0.9])  # unwrapped orbit past the periodic end: 16.5
    assert np.allclose(s, [0.0, 0.7 / 0.9, 1.0])
    s = O.knot_split(cfg, [1.2], [-1.0])  # backwards through 0.5
    assert np.allclose(s, [0.0, 0.7, 1.0])
    cfg2 = O.make_config(2, (16, 16, 1), (0, 0, 0), (16.0, 16.0, 1), 0.1)
    s = O.knot_split(cfg2, [0.0, 0.0], [1.0, 1.0])  # both axes cross 0.5 at s = 0.5: merged
    assert np.allclose(s, [0.0, 0.5, 1.0])


def _bspline_mesh_weights(dim, n, length, x, dx, nsub=2000):
    """Brute-force S-bar_g by composite GL5 over nsub equal pieces (B-spline from scipy)."""
    ref = BSpline.basis_element([-1.5, -0.5, 0.5, 1.5], extrapolate=False)
    t, w = np.polynomial.legendre.leggauss(5)
    s = ((np.arange(nsub)[:, None] + 0.5 * (t[None, :] + 1)) / nsub).ravel()
    ws = np.tile(0.5 * w / nsub, nsub)
    h = [length[i] / n[i] for i in range(dim)]
    out = {}
    pts = [(x[i] + s * dx[i]) / h[i] for i in range(dim)]
    lo = [int(math.floor(min(p.min(), p.max()))) - 2 for p in pts]
    hi = [int(math.ceil(max(p.min(), p.max()))) + 2 for p in pts]
    import itertools
    for g in itertools.product(*[range(lo[i], hi[i] + 1) for i in range(dim)]):
        val = np.ones_like(s)
        for i in range(dim):
            val = val * np.nan_to_num(ref(pts[i] - g[i]))
        tot = float(np.dot(ws, val))
        if tot != 0.0:
            key = 0
            mul = 1
            for i in range(dim):
                key += (g[i] % n[i]) * mul
                mul *= n[i]
            out[key] = out.get(key, 0.0) + tot
    return out


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_orbit_weights_brute_force(dim):
    n = (8, 6, 5)[:dim]
    length = (2.0, 1.8, 1.5)[:dim]
    cfg = O.make_config(dim, n + (1,) * (3 - dim), (0, 0, 0), length + (1,) * (3 - dim), 0.1)
    rng = np.random.default_rng(dim)
    for trial in range(3):
        x = rng.uniform(0, 1, dim) * np.array(length)
        dx = rng.uniform(-1.2, 1.2, dim) * np.array([length[i] / n[i] for i in range(dim)]) * (trial + 1)
        nodes, w = O.orbit_weights(cfg, x, dx)
        ref = _bspline_mesh_weights(dim, n, length, x, dx)
        got = dict(zip(nodes.tolist(), w.tolist()))
        assert set(k for k, v in ref.items() if abs(v) > 1e-12) <= set(got)
        for k in set(got) | set(ref):
            assert abs(got.get(k, 0.0) - ref.get(k, 0.0)) < 2e-9
        assert abs(w.sum() - 1.0) < 1e-14  # orbit-averaged partition of unity


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_low_order_gl_is_exact(dim):
    """GL(d+1) integrates the per-segment polynomials exactly: same result as GL8."""
    n = (6, 5, 4)
    length = (2.0, 2.2, 1.9)
    fields = W.random_fields(dim, n, length, seed=11)
    rng = np.random.default_rng(5)
    for _ in range(5):
        x = rng.uniform(0, 1, dim) * np.array(length[:dim])
        P = rng.normal(size=3) * 0.3
        vin = rng.uniform(-0.55, 0.55, 3)
        outs = []
        for gl in (dim + 1, 8):
            cfg = O.make_config(dim, n, (0, 0, 0), length, 0.7, gl_order=gl)
            outs.append(O.orbit_eval(cfg, *fields, x, P, -0.3, 0.3, vin))
        for key in ("vout", "Pnp1", "gradphibar", "Ubar", "D"):
            assert np.allclose(outs[0][key], outs[1][key], atol=2e-14, rtol=0), key
        if dim >= 2:  # one order lower is not exact
            cfg = O.make_config(dim, n, (0, 0, 0), length, 0.7, gl_order=dim)
            lo = O.orbit_eval(cfg, *fields, x, P, -0.3, 0.3, vin)
            assert np.abs(lo["D"] - outs[1]["D"]).max() > 1e-10


def test_orbit_discrete_gradient_brute_force():
    """D_lj = sum_g int A_l,g(s) d_j S_g(x(s)) ds, brute force in 2D with scipy B-splines."""
    dim, n, length = 2, (6, 5), (2.0, 1.5)
    gphi, An, Anp1, Uh = W.random_fields(dim, n, length, seed=3)
    cfg = O.make_config(dim, n + (1,), (0, 0, 0), length + (1,), 0.5)
    x = np.array([0.37, 1.21])
    vin = np.array([0.8, -0.9, 0.1])
    out = O.orbit_eval(cfg, gphi, An, Anp1, Uh, x, [0.1, 0.2, 0.3], -1.0, 1.0, vin)
    dx = 0.5 * vin[:2]
    ref = BSpline.basis_element([-1.5, -0.5, 0.5, 1.5], extrapolate=False)
    dref = ref.derivative()
    t, w = np.polynomial.legendre.leggauss(5)
    nsub = 3000
    s = ((np.arange(nsub)[:, None] + 0.5 * (t[None, :] + 1)) / nsub).ravel()
    ws = np.tile(0.5 * w / nsub, nsub)
    h = [length[i] / n[i] for i in range(dim)]
    D = np.zeros((3, 2))
    for gx in range(-3, 10):
        for gy in range(-3, 10):
            xi = (x[0] + s * dx[0]) / h[0] - gx
            yi = (x[1] + s * dx[1]) / h[1] - gy
            Sx, Sy = np.nan_to_num(ref(xi)), np.nan_to_num(ref(yi))
            dSx, dSy = np.nan_to_num(dref(xi)) / h[0], np.nan_to_num(dref(yi)) / h[1]
            g = (gx % n[0]) + n[0] * (gy % n[1])
            for l in range(3):
                Al = (1 - s) * An[l][g] + s * Anp1[l][g]
                D[l, 0] += np.dot(ws, Al * dSx * Sy)
                D[l, 1] += np.dot(ws, Al * Sx * dSy)
    assert np.allclose(out["D"][:, :2], D, atol=1e-8)
    assert np.all(out["D"][:, 2] == 0.0)


# ---- Higuera-Cary map -----------------------------------------------------------------

def _cross_matrix(B):
    """C(B) with C(B) v = v x B (cross-matrix convention of the paper)."""
    return np.array([[0, B[2], -B[1]], [-B[2], 0, B[0]], [B[1], -B[0], 0]], dtype=float)


def _hc_cases(n=200, seed=7):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        um = rng.normal(size=3) * 10 ** rng.uniform(-3, 1.5)
        tau = rng.normal(size=3) * 10 ** rng.uniform(-4, 1)
        yield um, tau


def test_cross_matrix_convention():
    rng = np.random.default_rng(0)
    for _ in range(10):
        v, B = rng.normal(size=3), rng.normal(size=3)
        assert np.allclose(_cross_matrix(B) @ v, np.cross(v, B), atol=1e-15)


def test_hc_zero_work_and_centered_gamma():
    for um, tau in _hc_cases():
        up, g = O.hc_map(um, tau)
        n2 = np.dot(um, um)
        assert abs(np.dot(up, up) - n2) <= 4e-15 * max(n2, 1e-300) + 1e-300
        ubar = 0.5 * (up + um)
        assert abs(g * g - (1 + np.dot(ubar, ubar))) <= 1e-14 * g * g


def test_hc_equals_cayley_rotation():
    for um, tau in _hc_cases(seed=8):
        up, g = O.hc_map(um, tau)
        Ct = _cross_matrix(tau / g)
        I = np.eye(3)
        ref = np.linalg.solve(I - Ct, (I + Ct) @ um)
        assert np.allclose(up, ref, atol=1e-14 * max(1.0, np.abs(um).max()), rtol=1e-13)


def test_hc_is_rotation_about_b_by_cayley_angle():
    """u+ is u- rotated about tau by -2 atan(|tau|/gamma_HC) (Rodrigues formula)."""
    for um, tau in _hc_cases(50, seed=9):
        up, g = O.hc_map(um, tau)
        nt = np.linalg.norm(tau)
        k = tau / nt
        th = -2.0 * math.atan(nt / g)
        rot = um * math.cos(th) + np.cross(k, um) * math.sin(th) + k * np.dot(k, um) * (1 - math.cos(th))
        assert np.allclose(up, rot, atol=1e-13 * max(1.0, np.abs(um).max()))


def test_hc_identity_without_field():
    up, g = O.hc_map([0.3, -2.0, 1.0], [0.0, 0.0, 0.0])
    assert np.allclose(up, [0.3, -2.0, 1.0], atol=0) and abs(g - math.sqrt(1 + 0.09 + 4 + 1)) < 1e-15


def test_hc_unit_jacobian_fd():
    """The full nonlinear HC map u- -> u+ (gamma_HC depends on u-) has det 1."""
    for um, tau in _hc_cases(60, seed=10):
        h = 1e-6 * max(1.0, np.linalg.norm(um))
        J = np.zeros((3, 3))
        for c in range(3):
            e = np.zeros(3)
            e[c] = h
            J[:, c] = (O.hc_map(um + e, tau)[0] - O.hc_map(um - e, tau)[0]) / (2 * h)
        assert abs(np.linalg.det(J) - 1.0) < 1e-7


# ---- secant velocity ------------------------------------------------------------------

def test_secant_identity():
    rng = np.random.default_rng(3)
    for _ in range(200):
        m = rng.uniform(0.1, 3.0)
        kap = rng.uniform(0.5, 2.0)
        pa, pb = rng.normal(size=3) * 3, rng.normal(size=3) * 3
        K = lambda p: m * kap ** 2 * (math.sqrt(1 + np.dot(p, p) / (m * kap) ** 2) - 1)
        v = O.vdg(pa, pb, m, kap)
        lhs = K(pa) - K(pb)
        assert abs(lhs - np.dot(v, pa - pb)) < 1e-13 * (abs(K(pa)) + abs(K(pb)) + 1)
        assert np.linalg.norm(v) < kap


# ---- one orbit evaluation: the paper's exact identities --------------------------------

def _rand_eval(dim, seed, dt=0.6, vscale=0.7):
    n = (6, 5, 4)
    length = (2.0, 1.7, 1.9)
    gphi, An, Anp1, _ = W.random_fields(dim, n, length, seed=seed)
    # the CN relation (A^{n+1} - A^n)/dt = U^{n+1/2} that the chain-rule lemma uses
    fields = (gphi, An, Anp1, (Anp1 - An) / dt)
    rng = np.random.default_rng(seed + 100)
    x = rng.uniform(0, 1, dim) * np.array(length[:dim])
    P = rng.normal(size=3)
    vin = rng.uniform(-1, 1, 3)
    vin *= vscale / max(1.0, np.linalg.norm(vin))
    q = -rng.uniform(0.5, 2.0)
    m = abs(q)
    cfg = O.make_config(dim, n, (0, 0, 0), length, dt)
    return cfg, fields, x, P, q, m, vin, O.orbit_eval(cfg, *fields, x, P, q, m, vin)


def _kin(p, m, kap=1.0):
    return m * kap ** 2 * (math.sqrt(1 + np.dot(p, p) / (m * kap) ** 2) - 1)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_chain_rule_lemma(dim):
    """A_h^{n+1}(x^{n+1}) - A_h^n(x^n) = dt U-bar + dt D v-bar at roundoff."""
    for seed in range(8):
        cfg, fields, x, P, q, m, vin, o = _rand_eval(dim, seed)
        Dv = o["D"][:, :dim] @ vin[:dim]
        RA = o["Aplus"] - o["Aminus"] - cfg.dt * (o["Ubar"] + Dv)
        scale = np.abs(o["Aplus"]).max() + np.abs(o["Aminus"]).max()
        assert np.abs(RA).max() < 5e-15 * max(scale, 1.0)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_canonical_equals_mechanical_split_and_work(dim):
    """GM-HC half transforms equal electric half kicks with E-bar = -grad-phi-bar - U-bar;
    the rotation does no work; the single-particle work balance holds at any iterate."""
    for seed in range(8):
        cfg, fields, x, P, q, m, vin, o = _rand_eval(dim, seed + 20)
        Ebar = -o["gradphibar"] - o["Ubar"]
        half = 0.5 * q * cfg.dt * Ebar
        sc = 1e-13 * max(1.0, np.abs(o["pn"]).max())
        assert np.allclose(o["pminus"] - o["pn"], half, atol=sc)
        assert np.allclose(o["pnp1"] - o["pplus"], half, atol=sc)
        assert abs(np.dot(o["pplus"], o["pplus"]) - np.dot(o["pminus"], o["pminus"])) < sc
        dK = _kin(o["pnp1"], m) - _kin(o["pn"], m)
        assert abs(dK - q * cfg.dt * np.dot(Ebar, o["vout"])) < 1e-13 * max(1.0, _kin(o["pn"], m))
        # endpoint definitions
        assert np.allclose(o["pn"], P - q * o["Aminus"], atol=1e-15 * max(1, np.abs(P).max()))
        assert np.allclose(o["pnp1"], o["Pnp1"] - q * o["Aplus"], atol=1e-14)
        # orbit velocity from the two secant velocities
        v = 0.5 * (O.vdg(o["pminus"], o["pn"], m) + O.vdg(o["pnp1"], o["pplus"], m))
        assert np.allclose(v, o["vout"], atol=1e-15)


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_beff_is_axial_vector_of_skew_part(dim):
    cfg, fields, x, P, q, m, vin, o = _rand_eval(dim, 40)
    D = o["D"]
    K = D.T - D
    assert np.allclose(_cross_matrix(o["Beff"]), K, atol=1e-15)
    v = np.array([0.3, -0.2, 0.5])
    assert np.allclose(K @ v, np.cross(v, o["Beff"]), atol=1e-15)  # K v = v x B_eff
    assert np.allclose(D.T @ v, D @ v + K @ v, atol=1e-15)  # D-split


def _linear_mesh(n, length, Afun):
    h = [length[i] / n[i] for i in range(3)]
    g = np.stack(np.meshgrid(*[np.arange(n[i]) * h[i] for i in range(3)], indexing="ij"))
    A = Afun(g)  # [3][nx][ny][nz]
    return np.ascontiguousarray(np.stack([np.transpose(A[c], (2, 1, 0)).ravel() for c in range(3)]))


def test_beff_sign_check_landau_gauge():
    """A = (0, B x, 0) gives B_eff = (0, 0, B) (sign check stated after the axial-vector helper)."""
    n, length = (16, 16, 16), (4.0, 4.0, 4.0)
    Bv = 0.37
    A = _linear_mesh(n, length, lambda g: np.stack([0 * g[0], Bv * g[0], 0 * g[0]]))
    cfg = O.make_config(3, n, (0, 0, 0), length, 0.05)
    zero3 = np.zeros_like(A)
    o = O.orbit_eval(cfg, zero3, A, A, zero3, [2.0, 2.1, 1.9], [0.1, 0.2, 0.3], -1.0, 1.0,
                     [0.3, 0.2, -0.1])
    assert np.allclose(o["Beff"], [0, 0, Bv], atol=1e-13)


def test_uniform_b_reduces_to_mechanical_hc():
    """Static A linear in x (uniform B), phi = 0: the GM-HC momentum map equals the
    mechanical HC rotation p^{n+1} = R_HC(p^n; B) (HC leapfrog template with E = 0)."""
    n, length = (16, 16, 16), (4.0, 4.0, 4.0)
    B = np.array([0.4, -0.7, 1.1])
    A = _linear_mesh(n, length, lambda g: 0.5 * np.stack([B[1] * g[2] - B[2] * g[1],
                                                         B[2] * g[0] - B[0] * g[2],
                                                         B[0] * g[1] - B[1] * g[0]]))
    cfg = O.make_config(3, n, (0, 0, 0), length, 0.08)
    zero3 = np.zeros_like(A)
    rng = np.random.default_rng(2)
    for _ in range(10):
        x = 2.0 + rng.uniform(-0.3, 0.3, 3)
        q = -rng.uniform(0.5, 2)
        m = abs(q)
        p = rng.normal(size=3) * 2
        Ah = O.interp(cfg, A, x)
        P = p + q * Ah
        vin = rng.uniform(-0.5, 0.5, 3)
        o = O.orbit_eval(cfg, zero3, A, A, zero3, x, P, q, m, vin)
        assert np.allclose(o["Beff"], B, atol=1e-12)
        up, _ = O.hc_map(p / m, q * cfg.dt / (2 * m) * B)
        assert np.allclose(o["pnp1"], m * up, atol=1e-12 * max(1, np.abs(p).max()))


def test_fixed_field_volume_preservation():
    """Frozen orbit data (v-bar, grad-phi-bar, D, K fixed): det d(x',P')/d(x,P) = 1 in 3D."""
    dim, n, length = 3, (6, 5, 4), (2.0, 1.7, 1.9)
    gphi, An, Anp1, Uh = W.random_fields(dim, n, length, seed=4)
    cfg = O.make_config(dim, n, (0, 0, 0), length, 0.4)
    x0 = np.array([0.7, 0.5, 1.1])
    P0 = np.array([0.4, -0.3, 0.8])
    q, m = -1.3, 1.3
    vbar = np.array([0.5, -0.3, 0.2])
    o = O.orbit_eval(cfg, gphi, An, Anp1, Uh, x0, P0, q, m, vbar)
    F3 = -0.5 * q * cfg.dt * o["gradphibar"] + 0.5 * q * cfg.dt * (o["D"] @ vbar)
    tau = q * cfg.dt / (2 * m) * o["Beff"]

    def fmap(z):
        x, P = z[:3], z[3:]
        Am = O.interp(cfg, An, x)
        Ap = O.interp(cfg, Anp1, x + cfg.dt * vbar)
        Aep = 0.5 * (Am + Ap)
        pm = P - q * Aep + F3
        up, _ = O.hc_map(pm / m, tau)
        return np.concatenate([x + cfg.dt * vbar, m * up + q * Aep + F3])

    z0 = np.concatenate([x0, P0])
    # the map at the base point reproduces the oracle's P^{n+1}
    assert np.allclose(fmap(z0)[3:], o["Pnp1"], atol=1e-13)
    h = 1e-6
    J = np.zeros((6, 6))
    for c in range(6):
        e = np.zeros(6)
        e[c] = h
        J[:, c] = (fmap(z0 + e) - fmap(z0 - e)) / (2 * h)
    assert abs(np.linalg.det(J) - 1.0) < 1e-8


def test_scatter_gather_adjointness():
    """sum_i q_i v_i . G-bar_i = sum_g J_g . G_g dV with the same orbit weights."""
    dim, n, length = 2, (8, 6), (2.0, 1.5)
    cfg = O.make_config(dim, n + (1,), (0, 0, 0), length + (1,), 0.3)
    rng = np.random.default_rng(9)
    G = rng.normal(size=(3, n[0] * n[1]))
    dV = (length[0] / n[0]) * (length[1] / n[1])
    J = np.zeros((3, n[0] * n[1]))
    lhs = 0.0
    for _ in range(40):
        x = rng.uniform(0, 1, 2) * np.array(length)
        v = rng.uniform(-0.9, 0.9, 3)
        q = -rng.uniform(0.1, 1)
        nodes, w = O.orbit_weights(cfg, x, 0.3 * v[:2])
        Gbar = (G[:, nodes] * w).sum(axis=1)
        lhs += q * np.dot(v, Gbar)
        for c in range(3):
            np.add.at(J[c], nodes, q * v[c] * w / dV)
    rhs = float((J * G).sum() * dV)
    assert abs(lhs - rhs) < 1e-13 * max(1.0, abs(lhs))
