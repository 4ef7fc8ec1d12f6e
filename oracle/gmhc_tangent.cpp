// gmhc_tangent.cpp -- forward-mode derivatives (the tangent-linear model) of a 1D
// GM-HC-CN run of the CPU oracle.
//
// TEST INFRASTRUCTURE ONLY, like gmhc_oracle.cpp: the independent reference for the
// GPU library's reverse-mode adjoint.  The paper defines no derivative of its step;
// this file differentiates the step it defines (Algorithm 1 with the orbit-averaged
// maps, the no-explicit-A_t GM-HC step, the secant velocity and the CN field step) in
// the plainest way there is: every real number of the run carries, beside its value,
// its derivatives along up to kMaxDir parameter directions (dual numbers), and every
// operation applies the chain rule to them.  Nothing here is a hand-derived Jacobian:
// the derivative of each formula is the one the arithmetic of dual numbers gives.
//
// The iterations are differentiated by running them to convergence with the derivatives
// carried along: the inner Picard loop of each particle and the outer damped-Picard loop
// on the mesh current stop only when the values pass the run's tests AND the derivative
// parts have settled (to the relative tolerance of the same tests, or to their rounding
// floor, see settled()).  The derivative of a
// contracting fixed-point iteration converges to the derivative of its fixed point
// (implicit-function theorem), so the result is the derivative of the converged step,
// independent of the iteration history.
//
// Scope: dim = 1, the quadratic shape S_2, damped Picard outer iteration, zero initial
// potentials (A^0 = U^0 = 0), FP64, no refinement.  The output is the field energy W
// and the kinetic energy K at the start and after `steps` steps, each with its
// derivatives along the directions seeded on the initial positions, mechanical
// momenta u = p / (m kappa) and charges (mass m = |q|).
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdint>
#include <limits>
#include <vector>

#include "orc_config.h"

extern "C" int orc_gl_rule(int n, double* x, double* w);

namespace {

using cplx = std::complex<double>;
const double kPi = 3.14159265358979323846264338327950288;
constexpr int kMaxDir = 16;

// Directions carried by the run in progress (a run is not reentrant).
int ND = 0;

// ---- dual numbers ------------------------------------------------------------
struct Dn {
  double v = 0.0;
  double d[kMaxDir] = {};
};

Dn cst(double a) {
  Dn r;
  r.v = a;
  return r;
}
Dn operator+(const Dn& a, const Dn& b) {
  Dn r;
  r.v = a.v + b.v;
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
Dn operator-(const Dn& a, const Dn& b) {
  Dn r;
  r.v = a.v - b.v;
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
Dn operator-(const Dn& a) {
  Dn r;
  r.v = -a.v;
  for (int k = 0; k < ND; ++k) r.d[k] = -a.d[k];
  return r;
}
Dn operator*(const Dn& a, const Dn& b) {
  Dn r;
  r.v = a.v * b.v;
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
Dn operator/(const Dn& a, const Dn& b) {
  Dn r;
  r.v = a.v / b.v;
  for (int k = 0; k < ND; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) / b.v;
  return r;
}
Dn operator+(const Dn& a, double b) { return a + cst(b); }
Dn operator+(double a, const Dn& b) { return cst(a) + b; }
Dn operator-(const Dn& a, double b) { return a - cst(b); }
Dn operator-(double a, const Dn& b) { return cst(a) - b; }
Dn operator*(const Dn& a, double b) {
  Dn r;
  r.v = a.v * b;
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] * b;
  return r;
}
Dn operator*(double a, const Dn& b) { return b * a; }
Dn operator/(const Dn& a, double b) { return a * (1.0 / b); }
Dn& operator+=(Dn& a, const Dn& b) { return a = a + b; }
Dn& operator-=(Dn& a, const Dn& b) { return a = a - b; }
Dn sqrt(const Dn& a) {
  Dn r;
  r.v = std::sqrt(a.v);
  for (int k = 0; k < ND; ++k) r.d[k] = a.d[k] / (2.0 * r.v);
  return r;
}
Dn fabs(const Dn& a) { return a.v < 0.0 ? -a : a; }

// ---- 1D mesh -------------------------------------------------------------------
struct Mesh1 {
  int n;
  double lo, L, h, dV;
  int wrap(int64_t i) const { return (int)(((i % n) + n) % n); }
};

// Centered quadratic B-spline S_2 (particle-shape paragraph of the solver section) and
// its derivative, for a dual argument.
Dn S2(const Dn& t) {
  const double a = std::fabs(t.v);
  if (a < 0.5) return 0.75 - t * t;
  if (a < 1.5) {
    Dn u = 1.5 - fabs(t);
    return 0.5 * (u * u);
  }
  return cst(0.0);
}
Dn dS2(const Dn& t) {
  const double a = std::fabs(t.v);
  if (a < 0.5) return -2.0 * t;
  if (a < 1.5) {
    Dn u = 1.5 - fabs(t);
    return t.v > 0.0 ? -u : u;
  }
  return cst(0.0);
}

// Real mesh array whose entries carry derivatives, and its split into layers (layer 0
// the values, layer k + 1 the derivatives along direction k) for the linear field step.
using DVec = std::vector<Dn>;
using CVec = std::vector<cplx>;

void fft(CVec& a, bool inverse) {  // radix-2, forward unnormalized, inverse scaled 1/n
  const int n = (int)a.size();
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(a[i], a[j]);
  }
  for (int len = 2; len <= n; len <<= 1) {
    const double ang = 2.0 * kPi / len * (inverse ? 1.0 : -1.0);
    for (int i = 0; i < n; i += len)
      for (int k = 0; k < len / 2; ++k) {
        const cplx w(std::cos(ang * k), std::sin(ang * k));
        const cplx u = a[i + k], v = a[i + k + len / 2] * w;
        a[i + k] = u + v;
        a[i + k + len / 2] = u - v;
      }
  }
  if (inverse)
    for (auto& z : a) z /= (double)n;
}

// Spectral field of every layer: S[l][m].
using Spec = std::vector<CVec>;

Spec to_spec(const Mesh1& M, const DVec& r) {
  Spec s(ND + 1, CVec(M.n));
  for (int l = 0; l <= ND; ++l) {
    for (int g = 0; g < M.n; ++g) s[l][g] = l ? r[g].d[l - 1] : r[g].v;
    fft(s[l], false);
  }
  return s;
}
DVec to_real(const Mesh1& M, const Spec& s) {
  DVec r(M.n);
  for (int l = 0; l <= ND; ++l) {
    CVec a = s[l];
    fft(a, true);
    for (int g = 0; g < M.n; ++g) (l ? r[g].d[l - 1] : r[g].v) = a[g].real();
  }
  return r;
}
Spec zero_spec(const Mesh1& M) { return Spec(ND + 1, CVec(M.n, 0.0)); }

// Wavenumber of index m (signed index, zero at the even-grid Nyquist index) and the
// Nyquist projector.
double kx(const Mesh1& M, int m) {
  if (m == M.n / 2) return 0.0;
  const int ms = m <= M.n / 2 ? m : m - M.n;
  return 2.0 * kPi * ms / M.L;
}
void project(const Mesh1& M, Spec& s, bool on) {
  if (!on) return;
  for (auto& l : s) l[M.n / 2] = 0.0;
}
Spec ddx(const Mesh1& M, const Spec& s) {
  Spec r = s;
  for (auto& l : r)
    for (int m = 0; m < M.n; ++m) l[m] *= cplx(0.0, kx(M, m));
  return r;
}

// ---- particle part -----------------------------------------------------------------
struct Part {
  Dn x, P[3], q, m, vbar[3];
};

struct TrialFields {  // real trial fields of one outer iteration
  DVec gphi, An[3], Anp1[3];
};

struct Dep {  // one particle's orbit-averaged shape, as (node, weight) pairs
  std::vector<std::pair<int, Dn>> w;
};

// Secant velocity of the relativistic kinetic energy, V(pa, pb) = (pa + pb) /
// (m (gamma(pa) + gamma(pb))).
Dn gamma_of(const Dn p[3], const Dn& m, double kappa) {
  Dn mk = m * kappa;
  return sqrt(1.0 + (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) / (mk * mk));
}
void vdg(const Dn pa[3], const Dn pb[3], const Dn& m, double kappa, Dn out[3]) {
  Dn den = m * (gamma_of(pa, m, kappa) + gamma_of(pb, m, kappa));
  for (int c = 0; c < 3; ++c) out[c] = (pa[c] + pb[c]) / den;
}
void cross(const Dn a[3], const Dn b[3], Dn o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
// Normalized HC magnetic map (definition of the normalized map) on u with tau.
void hc_map(const Dn um[3], const Dn tau[3], Dn up[3]) {
  Dn gm2 = 1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2];
  Dn tau2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];
  Dn ut = um[0] * tau[0] + um[1] * tau[1] + um[2] * tau[2];
  Dn sigma = gm2 - tau2;
  Dn X = tau2 + ut * ut;
  Dn R = sqrt(sigma * sigma + 4.0 * X);
  Dn g2 = sigma.v >= 0.0 ? 0.5 * (sigma + R) : 2.0 * X / (R - sigma);
  Dn gHC = sqrt(g2);
  Dn t[3] = {tau[0] / gHC, tau[1] / gHC, tau[2] / gHC};
  Dn t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  Dn s[3] = {2.0 * t[0] / (1.0 + t2), 2.0 * t[1] / (1.0 + t2), 2.0 * t[2] / (1.0 + t2)};
  Dn uxt[3], ustar[3], usxs[3];
  cross(um, t, uxt);
  for (int c = 0; c < 3; ++c) ustar[c] = um[c] + uxt[c];
  cross(ustar, s, usxs);
  for (int c = 0; c < 3; ++c) up[c] = um[c] + usxs[c];
}

struct Ctx {
  orc_config cfg;
  Mesh1 M;
  int ngl;
  double glx[64], glw[64];
};

// A_h(x) = sum_g F_g S_2((x - x_g)/h) of three real mesh arrays.
void interp3(const Ctx& C, const DVec F[3], const Dn& x, Dn out[3]) {
  const Mesh1& M = C.M;
  Dn xi = (x - M.lo) / M.h;
  const int64_t b = (int64_t)std::floor(xi.v);
  for (int c = 0; c < 3; ++c) out[c] = cst(0.0);
  for (int64_t i = b - 2; i <= b + 2; ++i) {
    Dn S = S2(xi - (double)i);
    if (S.v == 0.0) continue;
    const int g = M.wrap(i);
    for (int c = 0; c < 3; ++c) out[c] += F[c][g] * S;
  }
}

// One orbit evaluation v_out = F(v_in) (no-explicit-A_t GM-HC step, mechanical
// endpoints, electric-work secant velocities and their mean as the orbit velocity), with
// the knot-split Gauss-Legendre orbit quadrature of the straight orbit x + s dt v_x.
// dep, when given, receives the orbit-averaged shape of the evaluated orbit.
void orbit_eval(const Ctx& C, const TrialFields& F, const Part& p, const Dn vin[3], Dn vout[3], Dn Pn1[3],
                Dep* dep) {
  const Mesh1& M = C.M;
  const double dt = C.cfg.dt, kappa = C.cfg.kappa;
  Dn dx = dt * vin[0];
  // knot split: S_2 has knots at half-integer node offsets; a crossing counts when
  // strictly inside the orbit.
  Dn xi0 = (p.x - M.lo) / M.h, dxi = dx / M.h;
  std::vector<Dn> brk{cst(0.0)};
  const double e0 = xi0.v, e1 = xi0.v + dxi.v;
  if (e1 > e0) {
    for (int64_t j = (int64_t)std::floor(e0 - 0.5); j <= (int64_t)std::floor(e1 - 0.5) + 1; ++j) {
      Dn s = ((double)j + 0.5 - xi0) / dxi;
      if (s.v > 0.0 && s.v < 1.0) brk.push_back(s);
    }
  } else if (e1 < e0) {
    for (int64_t j = (int64_t)std::floor(e0 - 0.5) + 1; j >= (int64_t)std::floor(e1 - 0.5) - 1; --j) {
      Dn s = ((double)j + 0.5 - xi0) / dxi;
      if (s.v > 0.0 && s.v < 1.0) brk.push_back(s);
    }
  }
  brk.push_back(cst(1.0));
  std::sort(brk.begin(), brk.end(), [](const Dn& a, const Dn& b) { return a.v < b.v; });
  Dn gp = cst(0.0), D[3] = {cst(0.0), cst(0.0), cst(0.0)};
  for (size_t k = 0; k + 1 < brk.size(); ++k) {
    Dn a = brk[k], b = brk[k + 1];
    if (!(b.v > a.v)) continue;
    for (int qd = 0; qd < C.ngl; ++qd) {
      Dn s = a + (b - a) * C.glx[qd];
      Dn wq = (b - a) * C.glw[qd];
      Dn xs = xi0 + s * dxi;
      const int64_t bse = (int64_t)std::floor(xs.v);
      for (int64_t i = bse - 2; i <= bse + 2; ++i) {
        Dn t = xs - (double)i;
        Dn S = S2(t), dS = dS2(t) / M.h;
        if (S.v == 0.0 && dS.v == 0.0) continue;
        const int g = M.wrap(i);
        gp += wq * F.gphi[g] * S;
        for (int c = 0; c < 3; ++c) D[c] += wq * ((1.0 - s) * F.An[c][g] + s * F.Anp1[c][g]) * dS;
        if (dep && S.v != 0.0) dep->w.push_back({g, wq * S});
      }
    }
  }
  Dn Am[3], Ap[3];
  interp3(C, F.An, p.x, Am);
  interp3(C, F.Anp1, p.x + dx, Ap);
  const Dn& q = p.q;
  const Dn& m = p.m;
  Dn Aep[3], kick[3], pm[3];
  for (int c = 0; c < 3; ++c) {
    Aep[c] = 0.5 * (Am[c] + Ap[c]);
    kick[c] = 0.5 * dt * q * (D[c] * vin[0]);
    if (c == 0) kick[c] -= 0.5 * dt * q * gp;
    pm[c] = p.P[c] - q * Aep[c] + kick[c];
  }
  // B_eff of K = D~^T - D~ (D~ the 3x3 zero-padded 3x1 D): (0, -D_z, D_y).
  Dn Beff[3] = {cst(0.0), -D[2], D[1]};
  Dn um[3], tau[3], up[3], pp[3], pn[3], pn1[3], vEm[3], vEp[3];
  for (int c = 0; c < 3; ++c) {
    um[c] = pm[c] / (m * kappa);
    tau[c] = (dt * q / (2.0 * m)) * Beff[c];
  }
  hc_map(um, tau, up);
  for (int c = 0; c < 3; ++c) {
    pp[c] = (m * kappa) * up[c];
    Pn1[c] = pp[c] + q * Aep[c] + kick[c];
    pn[c] = p.P[c] - q * Am[c];
    pn1[c] = Pn1[c] - q * Ap[c];
  }
  vdg(pm, pn, m, kappa, vEm);
  vdg(pn1, pp, m, kappa, vEp);
  for (int c = 0; c < 3; ++c) vout[c] = 0.5 * (vEm[c] + vEp[c]);
}

// Settle test of the derivative parts of an iteration a = map(b): per direction, the
// change D = max_c |a.d - b.d| against the scale S = max_c |a.d|.  A direction has settled
// when D <= tol S, or when D has stopped contracting (D > prev / 2, with prev its change
// one iteration earlier): the iteration contracts by a fixed factor far below 1/2 until
// the rounding of the terms that make up the derivative is reached, so a change that no
// longer halves is that rounding floor (where the derivative is a small difference of
// larger terms, the floor lies above tol S).  prev holds kMaxDir changes (start: +inf).
bool settled(const Dn* a, const Dn* b, int n, double tol, double* prev) {
  bool all = true;
  for (int k = 0; k < ND; ++k) {
    double dmax = 0.0, smax = 0.0;
    for (int c = 0; c < n; ++c) {
      dmax = std::max(dmax, std::fabs(a[c].d[k] - b[c].d[k]));
      smax = std::max(smax, std::fabs(a[c].d[k]));
    }
    if (!(dmax <= tol * smax || dmax > 0.5 * prev[k])) all = false;
    prev[k] = dmax;
  }
  return all;
}

// Inner Picard loop of one particle (Algorithm 1, inner solve) until the values pass the
// mixed inner test and the derivatives have settled.  On success vin holds the v_in of
// the last evaluation, vout, Pn1 and dep its results.
bool inner_solve(const Ctx& C, const TrialFields& F, const Part& p, Dn vin[3], Dn vout[3], Dn Pn1[3], Dep& dep) {
  const orc_config& c = C.cfg;
  double prev[kMaxDir];
  std::fill(prev, prev + kMaxDir, std::numeric_limits<double>::infinity());
  for (int it = 0; it < 4 * c.max_inner; ++it) {
    dep.w.clear();
    orbit_eval(C, F, p, vin, vout, Pn1, &dep);
    double dmax = 0.0, vmax = 0.0, v2 = 0.0;
    bool finite = true;
    for (int k = 0; k < 3; ++k) {
      dmax = std::max(dmax, std::fabs(vout[k].v - vin[k].v));
      vmax = std::max(vmax, std::fabs(vout[k].v));
      v2 += vout[k].v * vout[k].v;
      finite = finite && std::isfinite(vout[k].v);
    }
    if (!finite || !(std::sqrt(v2) < c.kappa)) return false;
    const bool dset = settled(vout, vin, 3, c.tol_inner_rel, prev);
    if (dmax <= c.tol_inner_abs + c.tol_inner_rel * vmax && dset) return true;
    for (int k = 0; k < 3; ++k) vin[k] = vout[k];
  }
  return false;
}

// Spectral field state of the run (every layer).
struct State {
  Spec phi, psi, rho, A[3], U[3];
  DVec J[3];  // accepted current (seed of the next outer iteration)
};

// CN field step for the trial current j (Algorithm 1: project the trial current, advance
// charge by continuity, solve the CN potential equations mode by mode).  The step is
// linear in (state, j), so each layer is advanced on its own.
void field_step(const Ctx& C, const State& S, const DVec j[3], State& T, TrialFields& F) {
  const Mesh1& M = C.M;
  const double h = C.cfg.dt, kap2 = C.cfg.kappa * C.cfg.kappa;
  Spec jh[3];
  for (int c = 0; c < 3; ++c) {
    jh[c] = to_spec(M, j[c]);
    project(M, jh[c], C.cfg.project != 0);
  }
  T.phi = T.psi = T.rho = zero_spec(M);
  for (int c = 0; c < 3; ++c) T.A[c] = T.U[c] = zero_spec(M);
  Spec phih = zero_spec(M), Uh[3];
  for (int c = 0; c < 3; ++c) Uh[c] = zero_spec(M);
  for (int l = 0; l <= ND; ++l)
    for (int m = 0; m < M.n; ++m) {
      const double k = kx(M, m), a = kap2 * k * k, den = 1.0 + h * h * a / 4.0;
      T.rho[l][m] = S.rho[l][m] - h * cplx(0.0, k) * jh[0][l][m];
      const cplx rh = 0.5 * (S.rho[l][m] + T.rho[l][m]);
      T.phi[l][m] = ((1.0 - h * h * a / 4.0) * S.phi[l][m] + h * S.psi[l][m] + 0.5 * h * h * kap2 * C.cfg.sigma1 * rh) / den;
      T.psi[l][m] = 2.0 * (T.phi[l][m] - S.phi[l][m]) / h - S.psi[l][m];
      phih[l][m] = 0.5 * (S.phi[l][m] + T.phi[l][m]);
      for (int c = 0; c < 3; ++c) {
        T.A[c][l][m] = ((1.0 - h * h * a / 4.0) * S.A[c][l][m] + h * S.U[c][l][m] +
                        0.5 * h * h * kap2 * C.cfg.sigma2 * jh[c][l][m]) / den;
        T.U[c][l][m] = 2.0 * (T.A[c][l][m] - S.A[c][l][m]) / h - S.U[c][l][m];
        Uh[c][l][m] = 0.5 * (S.U[c][l][m] + T.U[c][l][m]);
      }
    }
  F.gphi = to_real(M, ddx(M, phih));
  for (int c = 0; c < 3; ++c) {
    F.An[c] = to_real(M, S.A[c]);
    F.Anp1[c] = to_real(M, T.A[c]);
  }
}

// Energies of the state: field energy W = sum (|E|^2 / (2 sigma1) + |B|^2 / (2 sigma2)) dV
// with E = -d_x phi - U, B = curl A = (0, -d_x A_z, d_x A_y); kinetic energy
// sum |p|^2 / (m (gamma + 1)) with p = P - q A_h(x).
void energies(const Ctx& C, const State& S, const std::vector<Part>& parts, Dn& W, Dn& K) {
  const Mesh1& M = C.M;
  DVec dphi = to_real(M, ddx(M, S.phi)), U[3], A[3];
  for (int c = 0; c < 3; ++c) {
    U[c] = to_real(M, S.U[c]);
    A[c] = to_real(M, S.A[c]);
  }
  DVec dAy = to_real(M, ddx(M, S.A[1])), dAz = to_real(M, ddx(M, S.A[2]));
  W = cst(0.0);
  for (int g = 0; g < M.n; ++g) {
    Dn Ex = -dphi[g] - U[0][g], Ey = -U[1][g], Ez = -U[2][g];
    Dn By = -dAz[g], Bz = dAy[g];
    Dn e2 = Ex * Ex + Ey * Ey + Ez * Ez, b2 = By * By + Bz * Bz;
    W += (e2 / (2.0 * C.cfg.sigma1) + b2 / (2.0 * C.cfg.sigma2)) * M.dV;
  }
  K = cst(0.0);
  for (const Part& p : parts) {
    Dn Ai[3], pm[3];
    interp3(C, A, p.x, Ai);
    for (int c = 0; c < 3; ++c) pm[c] = p.P[c] - p.q * Ai[c];
    Dn g = gamma_of(pm, p.m, C.cfg.kappa);
    K += (pm[0] * pm[0] + pm[1] * pm[1] + pm[2] * pm[2]) / (p.m * (g + 1.0));
  }
}

// Mixed outer tests of the values (RMS over 3 Ng components, max over nodes of the node
// norm), as the oracle's step applies them.
bool outer_pass(const Ctx& C, const DVec H[3], const DVec j[3]) {
  const int n = C.M.n;
  double sr = 0, sh = 0, sj = 0, mx = 0;
  const double ta = C.cfg.tol_outer_abs, tr = C.cfg.tol_outer_rel;
  for (int g = 0; g < n; ++g) {
    double r2 = 0, h2 = 0, j2 = 0;
    for (int c = 0; c < 3; ++c) {
      const double r = H[c][g].v - j[c][g].v;
      r2 += r * r;
      h2 += H[c][g].v * H[c][g].v;
      j2 += j[c][g].v * j[c][g].v;
    }
    sr += r2;
    sh += h2;
    sj += j2;
    mx = std::max(mx, std::sqrt(r2) / (ta + 0.5 * tr * (std::sqrt(h2) + std::sqrt(j2))));
  }
  const double n3 = 3.0 * n;
  const double rr = std::sqrt(sr / n3) / (ta + 0.5 * tr * (std::sqrt(sh / n3) + std::sqrt(sj / n3)));
  return rr <= 1.0 && mx <= 1.0;
}

// One implicit step (Algorithm 1) with damped Picard on the mesh current, run until the
// values pass the outer tests and the derivative parts of H(j) - j have settled.
int step(const Ctx& C, State& S, std::vector<Part>& parts, int64_t& outer) {
  const Mesh1& M = C.M;
  const int64_t np = (int64_t)parts.size();
  DVec j[3];
  for (int c = 0; c < 3; ++c) j[c] = S.J[c];
  std::vector<std::array<Dn, 3>> vw(np);
  for (int64_t i = 0; i < np; ++i)
    for (int c = 0; c < 3; ++c) vw[i][c] = parts[i].vbar[c];
  double prev[kMaxDir];
  std::fill(prev, prev + kMaxDir, std::numeric_limits<double>::infinity());
  for (int it = 0; it < 4 * C.cfg.max_outer; ++it) {
    State T;
    TrialFields F;
    field_step(C, S, j, T, F);
    std::vector<std::array<Dn, 3>> vin(np), Pn1(np);
    std::vector<Dep> dep(np);
    std::vector<int> ok(np, 1);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < np; ++i) {
      Dn v[3] = {vw[i][0], vw[i][1], vw[i][2]}, vo[3], P1[3];
      ok[i] = inner_solve(C, F, parts[i], v, vo, P1, dep[i]) ? 1 : 0;
      for (int c = 0; c < 3; ++c) {
        vin[i][c] = v[c];
        vw[i][c] = vo[c];
        Pn1[i][c] = P1[c];
      }
    }
    for (int64_t i = 0; i < np; ++i)
      if (!ok[i]) return -5;
    // orbit current deposit J_g = (1/dV) sum_i q_i v_out,i Sbar_ig, particle order
    DVec Jd[3];
    for (int c = 0; c < 3; ++c) Jd[c].assign(M.n, cst(0.0));
    for (int64_t i = 0; i < np; ++i)
      for (const auto& e : dep[i].w)
        for (int c = 0; c < 3; ++c) Jd[c][e.first] += parts[i].q * vw[i][c] * e.second / M.dV;
    DVec H[3];
    for (int c = 0; c < 3; ++c) {
      Spec s = to_spec(M, Jd[c]);
      project(M, s, C.cfg.project != 0);
      H[c] = to_real(M, s);
    }
    ++outer;
    std::vector<Dn> hf, jf;
    for (int c = 0; c < 3; ++c)
      for (int g = 0; g < M.n; ++g) {
        hf.push_back(H[c][g]);
        jf.push_back(j[c][g]);
      }
    const bool dset = settled(hf.data(), jf.data(), (int)hf.size(), C.cfg.tol_outer_rel, prev);
    const bool conv = outer_pass(C, H, j) && dset;
    if (conv) {  // commit (Algorithm 1): fields of j, particles of this evaluation
      S.phi = T.phi;
      S.psi = T.psi;
      S.rho = T.rho;
      for (int c = 0; c < 3; ++c) {
        S.A[c] = T.A[c];
        S.U[c] = T.U[c];
        S.J[c] = j[c];
      }
      for (int64_t i = 0; i < np; ++i) {
        Part& p = parts[i];
        Dn xe = p.x + C.cfg.dt * vin[i][0];
        const double k = std::floor((xe.v - M.lo) / M.L);  // periodic image, a constant shift
        p.x = xe - k * M.L;
        if (p.x.v >= M.lo + M.L) p.x -= cst(M.L);
        if (p.x.v < M.lo) p.x += cst(M.L);
        for (int c = 0; c < 3; ++c) {
          p.P[c] = Pn1[i][c];
          p.vbar[c] = vw[i][c];
        }
      }
      return 0;
    }
    for (int c = 0; c < 3; ++c)
      for (int g = 0; g < M.n; ++g) j[c][g] += C.cfg.beta * (H[c][g] - j[c][g]);
  }
  return -6;
}

// Initialization (Nyquist-projection paragraph and the constraint discussion) with zero
// initial potentials: projected charge and current from a point-shape deposit, the
// neutralizing background cancelling the mean charge, phi from Gauss's law
// (-Lap phi = sigma1 rho), psi = A = U = 0, canonical momenta P = p.
void initialize(const Ctx& C, std::vector<Part>& parts, State& S) {
  const Mesh1& M = C.M;
  DVec rho(M.n, cst(0.0)), J[3];
  for (int c = 0; c < 3; ++c) J[c].assign(M.n, cst(0.0));
  for (Part& p : parts) {
    Dn g = gamma_of(p.P, p.m, C.cfg.kappa);
    Dn v[3];
    for (int c = 0; c < 3; ++c) v[c] = p.P[c] / (p.m * g);
    Dn xi = (p.x - M.lo) / M.h;
    const int64_t b = (int64_t)std::floor(xi.v);
    for (int64_t i = b - 2; i <= b + 2; ++i) {
      Dn Sg = S2(xi - (double)i);
      if (Sg.v == 0.0) continue;
      const int gi = M.wrap(i);
      rho[gi] += p.q * Sg / M.dV;
      for (int c = 0; c < 3; ++c) J[c][gi] += p.q * v[c] * Sg / M.dV;
    }
    for (int c = 0; c < 3; ++c) p.vbar[c] = v[c];
  }
  S.rho = to_spec(M, rho);
  for (auto& l : S.rho) l[0] = 0.0;
  project(M, S.rho, C.cfg.project != 0);
  for (int c = 0; c < 3; ++c) {
    Spec s = to_spec(M, J[c]);
    project(M, s, C.cfg.project != 0);
    S.J[c] = to_real(M, s);
    S.A[c] = S.U[c] = zero_spec(M);
  }
  S.phi = S.psi = zero_spec(M);
  for (int l = 0; l <= ND; ++l)
    for (int m = 0; m < M.n; ++m) {
      const double k = kx(M, m);
      if (k != 0.0) S.phi[l][m] = C.cfg.sigma1 * S.rho[l][m] / (k * k);
    }
}

}  // namespace

extern "C" {

// Tangent-linear run: n particles x [n], u [3][n], q [n] (m = |q|) with nd <= 16 seed
// directions dx [nd][n], du [nd][3][n], dq [nd][n] (the derivatives of the inputs along
// each direction); steps implicit steps.  Out: E[4] = (W^0, K^0, W^T, K^T) and
// dE[4][nd] their derivatives along each direction; *outer the map evaluations summed
// over the steps.  Status 0, -1 (unsupported configuration), -5 (a particle solve
// failed), -6 (no outer convergence).
int orc_tangent_run(const orc_config* cfg, int64_t n, const double* x, const double* u, const double* q, int nd,
                    const double* dx, const double* du, const double* dq, int steps, double* E, double* dE,
                    int64_t* outer) {
  if (cfg->dim != 1 || (cfg->shape_order != 0 && cfg->shape_order != 2) || cfg->outer_scheme != 0 ||
      cfg->refine_levels != 0 || nd < 0 || nd > kMaxDir || cfg->gl_order < 1 || cfg->gl_order > 64)
    return -1;
  if (cfg->n[0] < 4 || (cfg->n[0] & (cfg->n[0] - 1)) != 0) return -1;
  ND = nd;
  Ctx C;
  C.cfg = *cfg;
  C.M.n = cfg->n[0];
  C.M.lo = cfg->lo[0];
  C.M.L = cfg->len[0];
  C.M.h = C.M.L / C.M.n;
  C.M.dV = C.M.h;
  C.ngl = cfg->gl_order;
  orc_gl_rule(C.ngl, C.glx, C.glw);
  std::vector<Part> parts(n);
  for (int64_t i = 0; i < n; ++i) {
    Part& p = parts[i];
    p.x = cst(x[i]);
    p.q = cst(q[i]);
    Dn uu[3];
    for (int c = 0; c < 3; ++c) uu[c] = cst(u[c * n + i]);
    for (int k = 0; k < nd; ++k) {
      p.x.d[k] = dx[k * n + i];
      p.q.d[k] = dq[k * n + i];
      for (int c = 0; c < 3; ++c) uu[c].d[k] = du[(k * 3 + c) * n + i];
    }
    p.m = fabs(p.q);
    for (int c = 0; c < 3; ++c) p.P[c] = (p.m * cfg->kappa) * uu[c];
  }
  State S;
  initialize(C, parts, S);
  Dn W0, K0;
  energies(C, S, parts, W0, K0);
  int64_t nout = 0;
  for (int s = 0; s < steps; ++s) {
    int st = step(C, S, parts, nout);
    if (st) return st;
  }
  Dn WT, KT;
  energies(C, S, parts, WT, KT);
  const Dn* r[4] = {&W0, &K0, &WT, &KT};
  for (int a = 0; a < 4; ++a) {
    E[a] = r[a]->v;
    for (int k = 0; k < nd; ++k) dE[a * nd + k] = r[a]->d[k];
  }
  if (outer) *outer = nout;
  return 0;
}

}  // extern "C"
