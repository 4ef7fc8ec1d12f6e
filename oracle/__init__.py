"""ctypes binding of the plain FP64 CPU oracle (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never does.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmhc_oracle.so")

OK, EINVAL, ESTATE, EINNER, ENOCONV = 0, -1, -2, -5, -6

FIELD = {"phi": 0, "psi": 1, "A": 2, "U": 3, "rho": 4, "J": 5, "E": 6, "B": 7}
FIELD_NCOMP = {"phi": 1, "psi": 1, "A": 3, "U": 3, "rho": 1, "J": 3, "E": 3, "B": 3}


class Config(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("len", C.c_double * 3),
        ("kappa", C.c_double), ("sigma1", C.c_double), ("sigma2", C.c_double), ("dt", C.c_double),
        ("gl_order", C.c_int32), ("project", C.c_int32),
        ("tol_outer_abs", C.c_double), ("tol_outer_rel", C.c_double),
        ("tol_inner_abs", C.c_double), ("tol_inner_rel", C.c_double),
        ("max_outer", C.c_int32), ("max_inner", C.c_int32), ("beta", C.c_double),
        ("threads", C.c_int32), ("outer_scheme", C.c_int32), ("anderson_m", C.c_int32),
        ("anderson_start", C.c_int32), ("ls_halvings", C.c_int32), ("anderson_lambda", C.c_double),
        ("ls_decrease", C.c_double), ("ls_growth", C.c_double), ("shape_order", C.c_int32),
        ("refine_levels", C.c_int32),
    ]


class EvalOut(C.Structure):
    _fields_ = [(name, C.c_double * 3) for name in (
        "vout", "Pnp1", "pminus", "pplus", "pn", "pnp1", "Aminus", "Aplus", "gradphibar", "Ubar")] + [
        ("D", C.c_double * 9), ("Beff", C.c_double * 3), ("gammaHC", C.c_double), ("nseg", C.c_int32)]

    def as_dict(self):
        d = {k: np.array(getattr(self, k)) for k, _ in self._fields_ if k not in ("gammaHC", "nseg", "D")}
        d["D"] = np.array(self.D).reshape(3, 3)
        d["gammaHC"] = self.gammaHC
        d["nseg"] = self.nseg
        return d


class Report(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("inner_max", C.c_int32), ("inner_mean", C.c_double),
                ("evaluations", C.c_int64), ("res_rms_ratio", C.c_double), ("res_max_ratio", C.c_double),
                ("outer_updates", C.c_int32), ("refined", C.c_int32)]


class Diag(C.Structure):
    _fields_ = [("t", C.c_double), ("step", C.c_int64)] + [(k, C.c_double) for k in (
        "kinetic", "field", "total", "energy_rel", "gauss_rms", "lorenz_rms", "chain_rms",
        "work_residual", "vperp_rms", "res_rms_ratio", "res_max_ratio")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        dp = C.POINTER(C.c_double)
        cfgp = C.POINTER(Config)
        L.orc_gl_rule.argtypes = [C.c_int, dp, dp]
        L.orc_shape.argtypes = [C.c_double, dp, dp]
        L.orc_shape.restype = None
        L.orc_shape_r.argtypes = [C.c_int, C.c_double, dp, dp]
        L.orc_shape_r.restype = None
        L.orc_hc_map.argtypes = [dp, dp, dp]
        L.orc_hc_map.restype = C.c_double
        L.orc_vdg.argtypes = [dp, dp, C.c_double, C.c_double, dp]
        L.orc_vdg.restype = None
        L.orc_fft.argtypes = [cfgp, dp, dp, C.c_int]
        L.orc_knot_split.argtypes = [cfgp, dp, dp, dp, C.c_int]
        L.orc_orbit_weights.argtypes = [cfgp, dp, dp, C.POINTER(C.c_int64), dp, C.c_int]
        L.orc_interp.argtypes = [cfgp, dp, dp, dp]
        L.orc_orbit_eval.argtypes = [cfgp, dp, dp, dp, dp, dp, dp, C.c_double, C.c_double, dp,
                                     C.POINTER(EvalOut)]
        L.orc_max_threads.argtypes = []
        L.orc_max_threads.restype = C.c_int
        L.orc_create.argtypes = [cfgp, C.POINTER(C.c_int)]
        L.orc_create.restype = C.c_void_p
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_destroy.restype = None
        L.orc_load_particles.argtypes = [C.c_void_p, C.c_int64, dp, dp, dp]
        L.orc_load_potentials.argtypes = [C.c_void_p, dp, dp]
        L.orc_initialize.argtypes = [C.c_void_p]
        L.orc_set_particle_state.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_read_particles.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_read_field.argtypes = [C.c_void_p, C.c_int, dp]
        L.orc_cn_advance.argtypes = [C.c_void_p, dp]
        L.orc_set_fields.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
        L.orc_step.argtypes = [C.c_void_p, C.POINTER(Report)]
        L.orc_diagnostics.argtypes = [C.c_void_p, C.POINTER(Diag)]
        L.orc_mode_amplitude.argtypes = [C.c_void_p, C.c_int, C.c_int, C.POINTER(C.c_int32), dp]
        ip = C.POINTER(C.c_int32)
        L.orc_orbit_pass.argtypes = [C.c_void_p, dp, dp, dp, dp, dp, C.c_int, dp, dp, dp, ip, ip, ip, dp, dp]
        L.orc_orbit_pass.restype = C.c_int64
        L.orc_trial_fields.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
        L.orc_spd_solve.argtypes = [C.c_int, dp, dp, dp]
        L.orc_num_particles.argtypes = [C.c_void_p]
        L.orc_num_particles.restype = C.c_int64
        L.orc_tangent_run.argtypes = [cfgp, C.c_int64, dp, dp, dp, C.c_int, dp, dp, dp, C.c_int, dp, dp,
                                      C.POINTER(C.c_int64)]
        _lib = L
    return _lib


def _p(a):
    """Pointer to a contiguous float64 numpy array (None passes NULL)."""
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"], "need contiguous float64"
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def make_config(dim, n, lo, length, dt, kappa=1.0, sigma1=1.0, sigma2=1.0, gl_order=8, project=1,
                tol_outer_abs=1e-14, tol_outer_rel=1e-12, tol_inner_abs=1e-14, tol_inner_rel=1e-12,
                max_outer=80, max_inner=64, beta=1.0, threads=0, outer_scheme=0, anderson_m=4,
                anderson_start=2, ls_halvings=6, anderson_lambda=1e-12, ls_decrease=1e-4, ls_growth=1.2,
                shape_order=2, refine_levels=0):
    c = Config()
    c.dim = dim
    for i in range(3):
        c.n[i] = int(n[i]) if i < dim else 1
        c.lo[i] = float(lo[i]) if i < dim else 0.0
        c.len[i] = float(length[i]) if i < dim else 1.0
    c.kappa, c.sigma1, c.sigma2, c.dt = kappa, sigma1, sigma2, dt
    c.gl_order, c.project = gl_order, project
    c.tol_outer_abs, c.tol_outer_rel = tol_outer_abs, tol_outer_rel
    c.tol_inner_abs, c.tol_inner_rel = tol_inner_abs, tol_inner_rel
    c.max_outer, c.max_inner, c.beta, c.threads = max_outer, max_inner, beta, threads
    c.outer_scheme, c.anderson_m, c.anderson_start, c.ls_halvings = outer_scheme, anderson_m, anderson_start, ls_halvings
    c.anderson_lambda, c.ls_decrease, c.ls_growth = anderson_lambda, ls_decrease, ls_growth
    c.shape_order = shape_order
    c.refine_levels = refine_levels
    return c


def config_from_dict(d, **over):
    kw = dict(d)
    kw.update(over)
    return make_config(**kw)


def ng(cfg):
    n = 1
    for i in range(cfg.dim):
        n *= cfg.n[i]
    return n


# ---- small helpers over single formulas -------------------------------------------------

def gl_rule(n):
    x = np.zeros(n)
    w = np.zeros(n)
    assert lib().orc_gl_rule(n, _p(x), _p(w)) == OK
    return x, w


def shape(xi, r=2):
    """Centered B-spline S_r(xi) of degree r (2: the paper's quadratic; 1: linear) and
    its derivative."""
    S = C.c_double()
    dS = C.c_double()
    lib().orc_shape_r(int(r), float(xi), C.byref(S), C.byref(dS))
    return S.value, dS.value


def hc_map(um, tau):
    um = _f64(um)
    tau = _f64(tau)
    up = np.zeros(3)
    g = lib().orc_hc_map(_p(um), _p(tau), _p(up))
    return up, g


def vdg(pa, pb, m, kappa=1.0):
    out = np.zeros(3)
    lib().orc_vdg(_p(_f64(pa)), _p(_f64(pb)), float(m), float(kappa), _p(out))
    return out


def fft(cfg, a, inverse=False):
    a = np.asarray(a, dtype=np.complex128)
    re = np.ascontiguousarray(a.real.ravel())
    im = np.ascontiguousarray(a.imag.ravel())
    assert lib().orc_fft(C.byref(cfg), _p(re), _p(im), int(inverse)) == OK
    return (re + 1j * im).reshape(a.shape)


def knot_split(cfg, x, dx):
    s = np.zeros(256)
    k = lib().orc_knot_split(C.byref(cfg), _p(_f64(x)), _p(_f64(dx)), _p(s), 256)
    assert k > 0
    return s[:k]


def orbit_weights(cfg, x, dx, cap=4096):
    nodes = np.zeros(cap, dtype=np.int64)
    w = np.zeros(cap)
    k = lib().orc_orbit_weights(C.byref(cfg), _p(_f64(x)), _p(_f64(dx)),
                                nodes.ctypes.data_as(C.POINTER(C.c_int64)), _p(w), cap)
    assert k >= 0
    return nodes[:k], w[:k]


def interp(cfg, F, x):
    out = np.zeros(3)
    assert lib().orc_interp(C.byref(cfg), _p(_f64(F)), _p(_f64(x)), _p(out)) == OK
    return out


def spd_solve(G, b):
    """x of G x = b by the oracle's Anderson small solve (Cholesky), or None when G is not
    numerically positive definite."""
    G = _f64(G)
    b = _f64(b)
    n = b.size
    x = np.zeros(n)
    st = lib().orc_spd_solve(n, _p(G.reshape(-1)), _p(b), _p(x))
    return x if st == OK else None


def orbit_eval(cfg, gphi, An, Anp1, Uh, x, P, q, m, vin):
    o = EvalOut()
    st = lib().orc_orbit_eval(C.byref(cfg), _p(_f64(gphi)), _p(_f64(An)), _p(_f64(Anp1)),
                              _p(_f64(Uh)), _p(_f64(x)), _p(_f64(P)), float(q), float(m),
                              _p(_f64(vin)), C.byref(o))
    assert st == OK
    return o.as_dict()


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


class OracleSim:
    """The oracle's whole-step interface: create, load, initialize, step, diagnose."""

    def __init__(self, cfg):
        self.cfg = cfg
        st = C.c_int(0)
        self.h = lib().orc_create(C.byref(cfg), C.byref(st))
        if not self.h:
            raise OracleError(st.value, "orc_create")
        self.d = cfg.dim
        self.ng = ng(cfg)
        self.np = 0

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            lib().orc_destroy(h)
            self.h = None

    def _chk(self, st, what):
        if st != OK:
            raise OracleError(st, what)

    def load_particles(self, x, u, q):
        x = _f64(x).reshape(self.d, -1)
        u = _f64(u).reshape(3, -1)
        q = _f64(q).ravel()
        self.np = q.size
        self._chk(lib().orc_load_particles(self.h, self.np, _p(x), _p(u), _p(q)), "load_particles")

    def load_potentials(self, A0, U0):
        self._chk(lib().orc_load_potentials(self.h, _p(_f64(A0).reshape(3, -1)),
                                            _p(_f64(U0).reshape(3, -1))), "load_potentials")

    def initialize(self):
        self._chk(lib().orc_initialize(self.h), "initialize")

    def set_particle_state(self, x, P, vbar):
        self._chk(lib().orc_set_particle_state(self.h, _p(_f64(x).reshape(self.d, -1)),
                                               _p(_f64(P).reshape(3, -1)),
                                               _p(_f64(vbar).reshape(3, -1))), "set_particle_state")

    def set_fields(self, phi, psi, A, U, rho):
        self._chk(lib().orc_set_fields(self.h, _p(_f64(phi)), _p(_f64(psi)), _p(_f64(A)),
                                       _p(_f64(U)), _p(_f64(rho))), "set_fields")

    def step(self, raise_on_error=True):
        r = Report()
        st = lib().orc_step(self.h, C.byref(r))
        if raise_on_error:
            self._chk(st, "step")
        return st, {k: getattr(r, k) for k, _ in r._fields_}

    def diagnostics(self):
        d = Diag()
        self._chk(lib().orc_diagnostics(self.h, C.byref(d)), "diagnostics")
        return d.as_dict()

    def read_particles(self):
        x = np.zeros((self.d, self.np))
        P = np.zeros((3, self.np))
        v = np.zeros((3, self.np))
        self._chk(lib().orc_read_particles(self.h, _p(x), _p(P), _p(v)), "read_particles")
        return x, P, v

    def read_field(self, which):
        nc = FIELD_NCOMP[which]
        out = np.zeros((nc, self.ng))
        self._chk(lib().orc_read_field(self.h, FIELD[which], _p(out)), "read_field")
        return out if nc > 1 else out[0]

    def cn_advance(self, j):
        self._chk(lib().orc_cn_advance(self.h, _p(_f64(j).reshape(3, -1))), "cn_advance")

    def mode_amplitude(self, which, comp, mode):
        m = (C.c_int32 * 3)(*[int(v) for v in mode])
        a = C.c_double()
        self._chk(lib().orc_mode_amplitude(self.h, FIELD[which], comp, m, C.byref(a)), "mode_amplitude")
        return a.value

    def trial_fields(self, j):
        gphi = np.zeros((self.d, self.ng))
        An = np.zeros((3, self.ng))
        Anp1 = np.zeros((3, self.ng))
        Uh = np.zeros((3, self.ng))
        self._chk(lib().orc_trial_fields(self.h, _p(_f64(j).reshape(3, -1)), _p(gphi), _p(An),
                                         _p(Anp1), _p(Uh)), "trial_fields")
        return gphi, An, Anp1, Uh

    def orbit_pass(self, gphi, An, Anp1, Uh, vin, iterate=False, want_J=True, level_in=None):
        """One frozen-field pass; level_in (iterate only) sets the refinement level each
        particle starts at.  Returns v_out, P^{n+1}, J, per-particle evaluations and levels
        (refine_levels + 1 where every level failed), the converged v_in and the unwrapped
        end positions."""
        ip = C.POINTER(C.c_int32)
        vout = np.zeros((3, self.np))
        Pn1 = np.zeros((3, self.np))
        J = np.zeros((3, self.ng)) if want_J else None
        iters = np.zeros(self.np, dtype=np.int32)
        level = np.zeros(self.np, dtype=np.int32)
        vinc = np.zeros((3, self.np))
        xend = np.zeros((self.d, self.np))
        lin = None
        if level_in is not None:
            lin = np.ascontiguousarray(np.broadcast_to(np.asarray(level_in, dtype=np.int32), (self.np,)))
        nfail = lib().orc_orbit_pass(self.h, _p(_f64(gphi).reshape(self.d, -1)),
                                     _p(_f64(An).reshape(3, -1)), _p(_f64(Anp1).reshape(3, -1)),
                                     _p(_f64(Uh).reshape(3, -1)), _p(_f64(vin).reshape(3, -1)),
                                     int(iterate), _p(vout), _p(Pn1), _p(J), iters.ctypes.data_as(ip),
                                     None if lin is None else lin.ctypes.data_as(ip), level.ctypes.data_as(ip),
                                     _p(vinc), _p(xend))
        if nfail < 0:
            raise OracleError(EINVAL, "orbit_pass: level_in outside 0..refine_levels")
        return {"vout": vout, "Pnp1": Pn1, "J": J, "iters": iters, "nfail": int(nfail), "level": level,
                "vin": vinc, "xend": xend}


def tangent_run(cfg, x, u, q, steps, dx=None, du=None, dq=None):
    """Forward-mode derivatives of a 1D, 2D or 3D run (gmhc_tangent.cpp): from the initial
    particles x [dim][N], u [3][N], q [N] and the seed directions dx [nd][dim][N],
    du [nd][3][N], dq [nd][N] (None: zero; nd <= 16), run ``steps`` steps.  Returns (E, dE, outer): E = (W0, K0, WT,
    KT), the field and kinetic energies at the start and at the end, dE [4][nd] their
    derivatives along each direction, and the outer map evaluations of the run."""
    q = _f64(q).ravel()
    n = q.size
    d = cfg.dim
    x = _f64(x).reshape(d, n)
    u = _f64(u).reshape(3, n)
    nd = max(int(np.shape(a)[0]) for a in (dx, du, dq) if a is not None) if any(
        a is not None for a in (dx, du, dq)) else 0
    dx = _f64(np.zeros((nd, d, n)) if dx is None else dx).reshape(nd, d, n)
    du = _f64(np.zeros((nd, 3, n)) if du is None else du).reshape(nd, 3, n)
    dq = _f64(np.zeros((nd, n)) if dq is None else dq).reshape(nd, n)
    E = np.zeros(4)
    dE = np.zeros((4, max(nd, 1)))
    outer = C.c_int64(0)
    st = lib().orc_tangent_run(C.byref(cfg), n, _p(x), _p(u), _p(q), nd, _p(dx), _p(du), _p(dq), int(steps),
                               _p(E), _p(dE), C.byref(outer))
    if st != OK:
        raise OracleError(st, "tangent_run")
    return E, dE[:, :nd], outer.value
