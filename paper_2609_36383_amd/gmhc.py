"""Thin ctypes binding of libgmhc (include/gmhc.h).

Argument marshalling only: every step of the computation runs in the HIP library.
PyTorch supplies the device workspace (a uint8 tensor) and the stream.  The library
must be built in-tree (``python -m paper_2609_36383_amd.build``); its absence is an
error, there is no fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmhc.so")

OK, EINVAL, ESTATE, ENOMEM, EDEVICE, EINNER, ENOCONV = 0, -1, -2, -3, -4, -5, -6
HOST, DEVICE = 0, 1
ABI_VERSION = 6  # layout of the structures below (include/gmhc.h, GMHC_ABI_VERSION)
FP64, FP32_BULK = 0, 1
PICARD, ANDERSON = 0, 1
FIELD = {"phi": 0, "psi": 1, "A": 2, "U": 3, "rho": 4, "J": 5, "E": 6, "B": 7}
FIELD_NCOMP = {"phi": 1, "psi": 1, "A": 3, "U": 3, "rho": 1, "J": 3, "E": 3, "B": 3}

# Every entry point include/gmhc.h declares.
SYMBOLS = (
    "gmhc_abi_version", "gmhc_status_str", "gmhc_last_error", "gmhc_create", "gmhc_destroy",
    "gmhc_workspace_bytes", "gmhc_bind", "gmhc_load_particles", "gmhc_load_potentials",
    "gmhc_initialize", "gmhc_step", "gmhc_diagnostics", "gmhc_read_particles",
    "gmhc_set_particle_state", "gmhc_read_field", "gmhc_mode_amplitude", "gmhc_set_frozen_fields",
    "gmhc_orbit_pass_frozen", "gmhc_read_pass", "gmhc_state_bytes", "gmhc_save", "gmhc_load",
    "gmhc_orbit_pass_static", "gmhc_adjoint_bytes", "gmhc_energy_grad", "gmhc_adjoint_step",
    "gmhc_adjoint_initialize",
)
STATIC_MAX_PARTICLES = 1 << 22  # GMHC_STATIC_MAX_PARTICLES
STATIC_MAX_NODES = 1 << 18      # GMHC_STATIC_MAX_NODES


class Config(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("n", C.c_int32 * 3), ("lo", C.c_double * 3), ("len", C.c_double * 3),
        ("kappa", C.c_double), ("sigma1", C.c_double), ("sigma2", C.c_double), ("dt", C.c_double),
        ("gl_order", C.c_int32), ("project_nyquist", C.c_int32), ("precision", C.c_int32),
        ("sort_every", C.c_int32),
        ("tol_outer_abs", C.c_double), ("tol_outer_rel", C.c_double),
        ("tol_inner_abs", C.c_double), ("tol_inner_rel", C.c_double),
        ("max_outer", C.c_int32), ("max_inner", C.c_int32), ("beta", C.c_double),
        ("timing", C.c_int32), ("graphs", C.c_int32),
        ("outer_scheme", C.c_int32), ("anderson_m", C.c_int32), ("anderson_start", C.c_int32),
        ("ls_halvings", C.c_int32), ("shape_order", C.c_int32),
        ("deterministic", C.c_int32),
        ("anderson_lambda", C.c_double), ("ls_decrease", C.c_double), ("ls_growth", C.c_double),
        ("refine_levels", C.c_int32),
    ]


class StepReport(C.Structure):
    _fields_ = [("outer_iters", C.c_int32), ("inner_max", C.c_int32), ("inner_mean", C.c_double),
                ("evaluations", C.c_int64), ("res_rms_ratio", C.c_double), ("res_max_ratio", C.c_double),
                ("orbit_ms", C.c_double), ("orbit_launches", C.c_int32), ("graph_replays", C.c_int32),
                ("segments", C.c_int64), ("outer_updates", C.c_int32), ("refined", C.c_int32)]


class Diag(C.Structure):
    _fields_ = [("t", C.c_double), ("step", C.c_int64)] + [(k, C.c_double) for k in (
        "kinetic", "field", "total", "energy_rel", "gauss_rms", "lorenz_rms", "chain_rms",
        "work_residual", "vperp_rms", "res_rms_ratio", "res_max_ratio")]


class PassReport(C.Structure):
    _fields_ = [("failed", C.c_int64), ("inner_max", C.c_int32), ("over_limit", C.c_int32),
                ("inner_mean", C.c_double), ("evaluations", C.c_int64), ("orbit_ms", C.c_double),
                ("segments", C.c_int64), ("refined", C.c_int64)]


class AdjointReport(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("change_ratio", C.c_double)]


def _todict(s):
    return {k: getattr(s, k) for k, _ in s._fields_ if k not in ("pad", "reserved")}


_lib = None


def load_library(path=LIB_PATH):
    """Load libgmhc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libgmhc.so not found at {path}: build it with "
                           "`python -m paper_2609_36383_amd.build`")
    # torch's HIP runtime must be the one the library binds to (one runtime per
    # process: the workspace and stream come from torch)
    import torch  # noqa: F401
    L = C.CDLL(path)
    vp, dp, i32, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64
    sig = {
        "gmhc_abi_version": ([], i32),
        "gmhc_status_str": ([i32], C.c_char_p),
        "gmhc_last_error": ([vp], C.c_char_p),
        "gmhc_create": ([C.POINTER(Config), C.POINTER(vp)], i32),
        "gmhc_destroy": ([vp], None),
        "gmhc_workspace_bytes": ([vp, i64, C.POINTER(C.c_size_t)], i32),
        "gmhc_bind": ([vp, i64, vp, C.c_size_t, vp], i32),
        "gmhc_load_particles": ([vp, vp, vp, vp, i32], i32),
        "gmhc_load_potentials": ([vp, vp, vp, i32], i32),
        "gmhc_initialize": ([vp], i32),
        "gmhc_step": ([vp, C.POINTER(StepReport)], i32),
        "gmhc_diagnostics": ([vp, C.POINTER(Diag)], i32),
        "gmhc_read_particles": ([vp, vp, vp, vp, i32], i32),
        "gmhc_set_particle_state": ([vp, vp, vp, vp, i32], i32),
        "gmhc_read_field": ([vp, i32, vp, i32], i32),
        "gmhc_mode_amplitude": ([vp, i32, i32, C.POINTER(i32), dp], i32),
        "gmhc_set_frozen_fields": ([vp, vp, vp, vp, vp, i32], i32),
        "gmhc_orbit_pass_frozen": ([vp, i32, C.POINTER(PassReport)], i32),
        "gmhc_read_pass": ([vp, vp, vp, vp, vp, vp, i32], i32),
        "gmhc_state_bytes": ([vp, C.POINTER(C.c_size_t)], i32),
        "gmhc_save": ([vp, vp, C.c_size_t, i32], i32),
        "gmhc_load": ([vp, vp, C.c_size_t, i32], i32),
        "gmhc_orbit_pass_static": ([C.POINTER(Config), i64] + [vp] * 8 + [i32] + [vp] * 5 +
                                   [C.POINTER(PassReport)], i32),
        "gmhc_adjoint_bytes": ([vp, C.POINTER(C.c_size_t)], i32),
        "gmhc_energy_grad": ([vp, vp, i32], i32),
        "gmhc_adjoint_step": ([vp, vp, C.c_size_t] + [vp] * 9 + [C.POINTER(AdjointReport)], i32),
        "gmhc_adjoint_initialize": ([vp, vp, C.c_size_t] + [vp] * 6, i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    if L.gmhc_abi_version() != ABI_VERSION:
        raise RuntimeError(f"{path} has ABI version {L.gmhc_abi_version()}, this binding expects "
                           f"{ABI_VERSION}: rebuild with `python -m paper_2609_36383_amd.build`")
    _lib = L
    return L


class GmhcError(RuntimeError):
    def __init__(self, code, where, msg=""):
        lib = load_library()
        super().__init__(f"{where}: {lib.gmhc_status_str(code).decode()} ({code}) {msg}")
        self.code = code


def make_config(dim, n, lo, length, dt, kappa=1.0, sigma1=1.0, sigma2=1.0, gl_order=0,
                project_nyquist=1, precision=FP64, sort_every=0, tol_outer_abs=1e-14,
                tol_outer_rel=1e-12, tol_inner_abs=1e-14, tol_inner_rel=1e-12, max_outer=80,
                max_inner=64, beta=1.0, timing=0, graphs=0, outer_scheme=0, anderson_m=4,
                anderson_start=2, ls_halvings=6, anderson_lambda=1e-12, ls_decrease=1e-4, ls_growth=1.2,
                shape_order=2, deterministic=1, refine_levels=0):
    c = Config()
    c.dim = dim
    for i in range(3):
        c.n[i] = int(n[i]) if i < dim else 1
        c.lo[i] = float(lo[i]) if i < dim else 0.0
        c.len[i] = float(length[i]) if i < dim else 1.0
    c.kappa, c.sigma1, c.sigma2, c.dt = kappa, sigma1, sigma2, dt
    c.gl_order, c.project_nyquist, c.precision, c.sort_every = gl_order, project_nyquist, precision, sort_every
    c.tol_outer_abs, c.tol_outer_rel = tol_outer_abs, tol_outer_rel
    c.tol_inner_abs, c.tol_inner_rel = tol_inner_abs, tol_inner_rel
    c.max_outer, c.max_inner, c.beta, c.timing, c.graphs = max_outer, max_inner, beta, timing, graphs
    c.outer_scheme, c.anderson_m, c.anderson_start, c.ls_halvings = outer_scheme, anderson_m, anderson_start, ls_halvings
    c.anderson_lambda, c.ls_decrease, c.ls_growth = anderson_lambda, ls_decrease, ls_growth
    c.shape_order = shape_order
    c.deterministic = deterministic
    c.refine_levels = refine_levels
    return c


def config_from_dict(d, **over):
    kw = dict(d)
    kw.update(over)
    return make_config(**kw)


def _host(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(C.c_void_p)


class Simulation:
    """One GM-HC-CN simulation on one GPU (the C-ABI context plus its torch workspace)."""

    def __init__(self, cfg, n_particles, device="cuda", stream=None):
        import torch
        self.torch = torch
        self.lib = load_library()
        self.cfg = cfg
        self.d = cfg.dim
        self.ng = int(np.prod([cfg.n[i] for i in range(cfg.dim)]))
        self.np = int(n_particles)
        h = C.c_void_p()
        self._chk(self.lib.gmhc_create(C.byref(cfg), C.byref(h)), "gmhc_create", None)
        self.h = h
        nbytes = C.c_size_t()
        self._chk(self.lib.gmhc_workspace_bytes(self.h, self.np, C.byref(nbytes)), "gmhc_workspace_bytes")
        self.device = torch.device(device)
        # the library's own stream (default priority): a non-null stream, so that the
        # outer iterations can be replayed as HIP graphs
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        # 256-byte aligned device workspace owned by torch
        self.ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=self.device)
        self.stream.wait_stream(torch.cuda.current_stream(self.device))
        base = self.ws.data_ptr()
        self.ws_ptr = (base + 255) & ~255
        self.ws_bytes = nbytes.value
        self._chk(self.lib.gmhc_bind(self.h, self.np, C.c_void_p(self.ws_ptr), self.ws_bytes,
                                     C.c_void_p(self.stream.cuda_stream)), "gmhc_bind")

    def _chk(self, st, where, h="self"):
        if st != OK:
            msg = ""
            if h == "self" and getattr(self, "h", None):
                msg = self.lib.gmhc_last_error(self.h).decode()
            raise GmhcError(st, where, msg)

    def close(self):
        if getattr(self, "h", None):
            self.lib.gmhc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup --------------------------------------------------------------------
    def load_particles(self, x, u, q):
        x, px = _host(np.asarray(x).reshape(self.d, -1))
        u, pu = _host(np.asarray(u).reshape(3, -1))
        q, pq = _host(np.asarray(q).ravel())
        assert q.size == self.np
        self._chk(self.lib.gmhc_load_particles(self.h, px, pu, pq, HOST), "gmhc_load_particles")

    def load_potentials(self, A0, U0):
        A0, pa = _host(np.asarray(A0).reshape(3, -1))
        U0, pu = _host(np.asarray(U0).reshape(3, -1))
        self._chk(self.lib.gmhc_load_potentials(self.h, pa, pu, HOST), "gmhc_load_potentials")

    def initialize(self):
        self._chk(self.lib.gmhc_initialize(self.h), "gmhc_initialize")

    # -- stepping -----------------------------------------------------------------
    def step(self, raise_on_error=True):
        r = StepReport()
        st = self.lib.gmhc_step(self.h, C.byref(r))
        if raise_on_error:
            self._chk(st, "gmhc_step")
        return st, _todict(r)

    def diagnostics(self):
        d = Diag()
        self._chk(self.lib.gmhc_diagnostics(self.h, C.byref(d)), "gmhc_diagnostics")
        return _todict(d)

    # -- read / write -------------------------------------------------------------
    def read_particles(self):
        x = np.zeros((self.d, self.np))
        P = np.zeros((3, self.np))
        v = np.zeros((3, self.np))
        self._chk(self.lib.gmhc_read_particles(self.h, x.ctypes.data_as(C.c_void_p),
                                               P.ctypes.data_as(C.c_void_p),
                                               v.ctypes.data_as(C.c_void_p), HOST), "gmhc_read_particles")
        return x, P, v

    def set_particle_state(self, x, P, vbar):
        x, px = _host(np.asarray(x).reshape(self.d, -1))
        P, pP = _host(np.asarray(P).reshape(3, -1))
        v, pv = _host(np.asarray(vbar).reshape(3, -1))
        self._chk(self.lib.gmhc_set_particle_state(self.h, px, pP, pv, HOST), "gmhc_set_particle_state")

    def read_field(self, which):
        nc = FIELD_NCOMP[which]
        out = np.zeros((nc, self.ng))
        self._chk(self.lib.gmhc_read_field(self.h, FIELD[which], out.ctypes.data_as(C.c_void_p), HOST),
                  "gmhc_read_field")
        return out if nc > 1 else out[0]

    def mode_amplitude(self, which, comp, mode):
        m = (C.c_int32 * 3)(*[int(v) for v in mode])
        a = C.c_double()
        self._chk(self.lib.gmhc_mode_amplitude(self.h, FIELD[which], comp, m, C.byref(a)),
                  "gmhc_mode_amplitude")
        return a.value

    # -- frozen-field orbit pass (test and benchmark hook) --------------------------
    def set_frozen_fields(self, gphi, An, Anp1, Uh):
        arrs = [_host(np.asarray(a).reshape(-1, self.ng)) for a in (gphi, An, Anp1, Uh)]
        self._chk(self.lib.gmhc_set_frozen_fields(self.h, *[p for _, p in arrs], HOST),
                  "gmhc_set_frozen_fields")

    def orbit_pass_frozen(self, iterate=False):
        r = PassReport()
        self._chk(self.lib.gmhc_orbit_pass_frozen(self.h, int(iterate), C.byref(r)), "gmhc_orbit_pass_frozen")
        return _todict(r)

    # -- checkpoint / restore of the accepted state ---------------------------------
    def state_bytes(self):
        n = C.c_size_t()
        self._chk(self.lib.gmhc_state_bytes(self.h, C.byref(n)), "gmhc_state_bytes")
        return n.value

    def save(self, out=None):
        """The accepted state as an image: into a new host uint8 array, or into `out`
        (a numpy uint8 array, or a torch uint8 tensor on this device)."""
        n = self.state_bytes()
        if out is None:
            out = np.zeros(n, dtype=np.uint8)
        if isinstance(out, np.ndarray):
            assert out.dtype == np.uint8 and out.size >= n and out.flags.c_contiguous
            self._chk(self.lib.gmhc_save(self.h, out.ctypes.data_as(C.c_void_p), out.size, HOST), "gmhc_save")
        else:
            assert out.dtype == self.torch.uint8 and out.numel() >= n and out.is_contiguous()
            self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
            self._chk(self.lib.gmhc_save(self.h, C.c_void_p(out.data_ptr()), out.numel(), DEVICE), "gmhc_save")
        return out

    def load(self, image):
        """Restore an image written by save() (numpy or device tensor)."""
        if isinstance(image, np.ndarray):
            image = np.ascontiguousarray(image, dtype=np.uint8)
            self._chk(self.lib.gmhc_load(self.h, image.ctypes.data_as(C.c_void_p), image.size, HOST), "gmhc_load")
        else:
            self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
            self._chk(self.lib.gmhc_load(self.h, C.c_void_p(image.data_ptr()), image.numel(), DEVICE), "gmhc_load")

    # -- device read-outs and the adjoint (torch float64 tensors on this device) ----
    def _dev(self, t):
        assert t.dtype == self.torch.float64 and t.is_contiguous() and t.device == self.device
        return C.c_void_p(t.data_ptr())

    def read_field_into(self, which, out):
        """Real-space field `which` of the accepted state into the device tensor out."""
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        self._chk(self.lib.gmhc_read_field(self.h, FIELD[which], self._dev(out), DEVICE), "gmhc_read_field")
        return out

    def read_particles_into(self, x=None, P=None, vbar=None):
        """Particle state (load order) into device tensors; None skips."""
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        p = [self._dev(t) if t is not None else None for t in (x, P, vbar)]
        self._chk(self.lib.gmhc_read_particles(self.h, *p, DEVICE), "gmhc_read_particles")

    def adjoint_bytes(self):
        n = C.c_size_t()
        self._chk(self.lib.gmhc_adjoint_bytes(self.h, C.byref(n)), "gmhc_adjoint_bytes")
        return n.value

    def adjoint_scratch(self):
        """A 256-byte aligned device scratch tensor for the adjoint calls."""
        n = self.adjoint_bytes()
        buf = self.torch.empty(n + 256, dtype=self.torch.uint8, device=self.device)
        off = (-buf.data_ptr()) % 256
        return buf[off:off + n]

    def energy_grad(self, out):
        """out [9][Ng] (device): the cotangent of the field energy of the accepted state."""
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        self._chk(self.lib.gmhc_energy_grad(self.h, self._dev(out), DEVICE), "gmhc_energy_grad")
        return out

    def adjoint_step(self, scratch, j, vbar, lx, lP, lf, gx, gP, gq, gf):
        """gmhc_adjoint_step on device tensors; returns its report."""
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        r = AdjointReport()
        args = [self._dev(t) for t in (j, vbar, lx, lP, lf, gx, gP, gq, gf)]
        self._chk(self.lib.gmhc_adjoint_step(self.h, C.c_void_p(scratch.data_ptr()), scratch.numel(), *args,
                                             C.byref(r)), "gmhc_adjoint_step")
        return _todict(r)

    def adjoint_initialize(self, scratch, lx, lP, lf, gx, gu, gq):
        self.stream.wait_stream(self.torch.cuda.current_stream(self.device))
        args = [self._dev(t) for t in (lx, lP, lf, gx, gu, gq)]
        self._chk(self.lib.gmhc_adjoint_initialize(self.h, C.c_void_p(scratch.data_ptr()), scratch.numel(), *args),
                  "gmhc_adjoint_initialize")

    def read_pass(self, iters=False, current=True, levels=False):
        """v_out, P^{n+1} and J (None unless current) of the last frozen pass, then with
        iters the per-particle evaluation counts and with levels the refinement levels."""
        vout = np.zeros((3, self.np))
        Pn1 = np.zeros((3, self.np))
        J = np.zeros((3, self.ng)) if current else None
        it = np.zeros(self.np, dtype=np.int32) if iters else None
        lv = np.zeros(self.np, dtype=np.int32) if levels else None
        ptr = lambda a: a.ctypes.data_as(C.c_void_p) if a is not None else None
        self._chk(self.lib.gmhc_read_pass(self.h, ptr(vout), ptr(Pn1), ptr(J), ptr(it), ptr(lv), HOST),
                  "gmhc_read_pass")
        return (vout, Pn1, J) + ((it,) if iters else ()) + ((lv,) if levels else ())


def orbit_pass_static(cfg, x, P, q, vin, gradphi, An, Anp1, Uh, vout, Pnp1, xnp1, J, iterate=False,
                      stream=None, report=True):
    """gmhc_orbit_pass_static on torch device tensors (FP64, contiguous; shapes as the
    header states).  Allocates nothing on the device; returns the pass report (a dict)
    or None."""
    lib = load_library()
    n = int(q.numel())
    ptr = [C.c_void_p(t.data_ptr()) for t in (x, P, q, vin, gradphi, An, Anp1, Uh)]
    out = [C.c_void_p(t.data_ptr()) for t in (vout, Pnp1, xnp1, J)]
    r = PassReport()
    st = lib.gmhc_orbit_pass_static(C.byref(cfg), n, *ptr, int(iterate), *out,
                                    C.c_void_p(stream.cuda_stream) if stream is not None else None,
                                    C.byref(r) if report else None)
    if st != OK:
        raise GmhcError(st, "gmhc_orbit_pass_static", lib.gmhc_last_error(None).decode())
    return _todict(r) if report else None
