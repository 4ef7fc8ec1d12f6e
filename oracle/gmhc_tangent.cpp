// gmhc_tangent.cpp -- forward-mode derivatives (the tangent-linear model) of a GM-HC-CN
// run (1D, 2D or 3D) of the CPU oracle.
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
// Scope: dim 1, 2 or 3, the quadratic shape S_2, damped Picard outer iteration, zero initial
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

// ---- mesh (d = 1, 2 or 3) ------------------------------------------------------
// Node g = i0 + n0 (i1 + n1 i2) at lo + i h (periodic); unresolved axes have n = 1.
struct Mesh {
  int d;
  int n[3];
  double lo[3], L[3], h[3], dV;
  int Ng;
  int wrap(int l, int64_t i) const { return (int)(((i % n[l]) + n[l]) % n[l]); }
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

void fft1(cplx* a, int n, int stride, bool inverse) {  // radix-2, forward unnormalized
  std::vector<cplx> b(n);
  for (int i = 0; i < n; ++i) b[i] = a[(int64_t)i * stride];
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(b[i], b[j]);
  }
  for (int len = 2; len <= n; len <<= 1) {
    const double ang = 2.0 * kPi / len * (inverse ? 1.0 : -1.0);
    for (int i = 0; i < n; i += len)
      for (int k = 0; k < len / 2; ++k) {
        const cplx w(std::cos(ang * k), std::sin(ang * k));
        const cplx u = b[i + k], v = b[i + k + len / 2] * w;
        b[i + k] = u + v;
        b[i + k + len / 2] = u - v;
      }
  }
  for (int i = 0; i < n; ++i) a[(int64_t)i * stride] = inverse ? b[i] / (double)n : b[i];
}
// Multi-dimensional transform of one layer, one axis after the other.
void fft(const Mesh& M, CVec& a, bool inverse) {
  const int n0 = M.n[0], n1 = M.n[1], n2 = M.n[2];
  for (int r = 0; r < n1 * n2; ++r) fft1(a.data() + (int64_t)r * n0, n0, 1, inverse);
  if (M.d > 1)
    for (int z = 0; z < n2; ++z)
      for (int c = 0; c < n0; ++c) fft1(a.data() + (int64_t)z * n0 * n1 + c, n1, n0, inverse);
  if (M.d > 2)
    for (int c = 0; c < n0 * n1; ++c) fft1(a.data() + c, n2, n0 * n1, inverse);
}

// Spectral field of every layer: S[l][m].
using Spec = std::vector<CVec>;

Spec to_spec(const Mesh& M, const DVec& r) {
  Spec s(ND + 1, CVec(M.Ng));
  for (int l = 0; l <= ND; ++l) {
    for (int g = 0; g < M.Ng; ++g) s[l][g] = l ? r[g].d[l - 1] : r[g].v;
    fft(M, s[l], false);
  }
  return s;
}
DVec to_real(const Mesh& M, const Spec& s) {
  DVec r(M.Ng);
  for (int l = 0; l <= ND; ++l) {
    CVec a = s[l];
    fft(M, a, true);
    for (int g = 0; g < M.Ng; ++g) (l ? r[g].d[l - 1] : r[g].v) = a[g].real();
  }
  return r;
}
Spec zero_spec(const Mesh& M) { return Spec(ND + 1, CVec(M.Ng, 0.0)); }

// Wavenumbers of mode g (signed index, zero at an even-grid Nyquist index, as the spectral
// derivative of the paper's Nyquist paragraph), and whether g lies on a Nyquist plane.
void kvec(const Mesh& M, int g, double k[3], bool& nyq) {
  const int idx[3] = {g % M.n[0], (g / M.n[0]) % M.n[1], g / (M.n[0] * M.n[1])};
  nyq = false;
  for (int l = 0; l < 3; ++l) {
    k[l] = 0.0;
    if (l >= M.d) continue;
    if (idx[l] == M.n[l] / 2) {
      nyq = true;
      continue;
    }
    const int ms = idx[l] <= M.n[l] / 2 ? idx[l] : idx[l] - M.n[l];
    k[l] = 2.0 * kPi * ms / M.L[l];
  }
}
void project(const Mesh& M, Spec& s, bool on) {
  if (!on) return;
  for (int g = 0; g < M.Ng; ++g) {
    double k[3];
    bool nyq;
    kvec(M, g, k, nyq);
    if (nyq)
      for (auto& l : s) l[g] = 0.0;
  }
}
Spec dspec(const Mesh& M, const Spec& s, int ax) {  // d/dx_ax: i k_ax
  Spec r = s;
  for (int g = 0; g < M.Ng; ++g) {
    double k[3];
    bool nyq;
    kvec(M, g, k, nyq);
    for (auto& l : r) l[g] *= cplx(0.0, ax < M.d ? k[ax] : 0.0);
  }
  return r;
}

// ---- particle part -----------------------------------------------------------------
struct Part {
  Dn x[3], P[3], q, m, vbar[3];
};

struct TrialFields {  // real trial fields of one outer iteration
  DVec gphi[3], An[3], Anp1[3];
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
  Mesh M;
  int ngl;
  double glx[64], glw[64];
};

// Shape weights of the candidate nodes around a point with unit offsets xi[l]
// (five candidates per resolved axis; nodes outside the support get zero) and their
// derivatives with respect to the position, as (node, S, dS/dx_0, dS/dx_1).
struct NodeW {
  int g;
  Dn S, dS[3];
};
void node_weights(const Mesh& M, const Dn xi[3], std::vector<NodeW>& out) {
  out.clear();
  int64_t b[3];
  Dn S1[3][5], dS1[3][5];  // per axis: the five candidates around floor(xi)
  for (int l = 0; l < 3; ++l) {
    b[l] = l < M.d ? (int64_t)std::floor(xi[l].v) : 0;
    for (int o = 0; o < 5; ++o) {
      if (l < M.d) {
        S1[l][o] = S2(xi[l] - (double)(b[l] + o - 2));
        dS1[l][o] = dS2(xi[l] - (double)(b[l] + o - 2)) / M.h[l];
      } else {
        S1[l][o] = cst(o == 2 ? 1.0 : 0.0);
        dS1[l][o] = cst(0.0);
      }
    }
  }
  const int z0 = M.d > 2 ? 0 : 2, z1 = M.d > 2 ? 5 : 3, y0 = M.d > 1 ? 0 : 2, y1 = M.d > 1 ? 5 : 3;
  for (int oz = z0; oz < z1; ++oz)
    for (int oy = y0; oy < y1; ++oy)
      for (int ox = 0; ox < 5; ++ox) {
        NodeW w;
        w.S = S1[0][ox] * S1[1][oy] * S1[2][oz];
        w.dS[0] = dS1[0][ox] * S1[1][oy] * S1[2][oz];
        w.dS[1] = S1[0][ox] * dS1[1][oy] * S1[2][oz];
        w.dS[2] = S1[0][ox] * S1[1][oy] * dS1[2][oz];
        if (w.S.v == 0.0 && w.dS[0].v == 0.0 && w.dS[1].v == 0.0 && w.dS[2].v == 0.0) continue;
        w.g = M.wrap(0, b[0] + ox - 2) + M.n[0] * (M.wrap(1, b[1] + oy - 2) + M.n[1] * M.wrap(2, b[2] + oz - 2));
        out.push_back(w);
      }
}

// A_h(x) = sum_g F_g S_g(x) of three real mesh arrays.
void interp3(const Ctx& C, const DVec F[3], const Dn x[3], Dn out[3]) {
  const Mesh& M = C.M;
  Dn xi[3];
  for (int l = 0; l < 3; ++l) xi[l] = l < M.d ? (x[l] - M.lo[l]) / M.h[l] : cst(0.0);
  std::vector<NodeW> nw;
  node_weights(M, xi, nw);
  for (int c = 0; c < 3; ++c) out[c] = cst(0.0);
  for (const NodeW& w : nw)
    for (int c = 0; c < 3; ++c) out[c] += F[c][w.g] * w.S;
}

// One orbit evaluation v_out = F(v_in) (no-explicit-A_t GM-HC step, mechanical
// endpoints, electric-work secant velocities and their mean as the orbit velocity), with
// the knot-split Gauss-Legendre orbit quadrature of the straight orbit x + s dt v.
// dep, when given, receives the orbit-averaged shape of the evaluated orbit.
void orbit_eval(const Ctx& C, const TrialFields& F, const Part& p, const Dn vin[3], Dn vout[3], Dn Pn1[3],
                Dep* dep) {
  const Mesh& M = C.M;
  const int d = M.d;
  const double dt = C.cfg.dt, kappa = C.cfg.kappa;
  // knot split: S_2 has knots at half-integer node offsets on every axis; a crossing
  // counts when strictly inside the orbit.
  Dn xi0[3], dxi[3];
  std::vector<Dn> brk{cst(0.0)};
  for (int l = 0; l < 3; ++l) {
    xi0[l] = l < d ? (p.x[l] - M.lo[l]) / M.h[l] : cst(0.0);
    dxi[l] = l < d ? dt * vin[l] / M.h[l] : cst(0.0);
    if (l >= d || dxi[l].v == 0.0) continue;
    const double e0 = xi0[l].v, e1 = xi0[l].v + dxi[l].v;
    const int64_t ja = (int64_t)std::floor(std::min(e0, e1) - 0.5) - 1, jb = (int64_t)std::floor(std::max(e0, e1) - 0.5) + 1;
    for (int64_t j = ja; j <= jb; ++j) {
      Dn s = ((double)j + 0.5 - xi0[l]) / dxi[l];
      if (s.v > 0.0 && s.v < 1.0) brk.push_back(s);
    }
  }
  brk.push_back(cst(1.0));
  std::sort(brk.begin(), brk.end(), [](const Dn& a, const Dn& b) { return a.v < b.v; });
  Dn gp[3] = {cst(0.0), cst(0.0), cst(0.0)}, D[3][3];
  for (int c = 0; c < 3; ++c) D[c][0] = D[c][1] = D[c][2] = cst(0.0);
  std::vector<NodeW> nw;
  for (size_t k = 0; k + 1 < brk.size(); ++k) {
    Dn a = brk[k], b = brk[k + 1];
    if (!(b.v > a.v)) continue;
    for (int qd = 0; qd < C.ngl; ++qd) {
      Dn s = a + (b - a) * C.glx[qd];
      Dn wq = (b - a) * C.glw[qd];
      Dn xs[3] = {xi0[0] + s * dxi[0], xi0[1] + s * dxi[1], xi0[2] + s * dxi[2]};
      node_weights(M, xs, nw);
      for (const NodeW& w : nw) {
        for (int l = 0; l < d; ++l) gp[l] += wq * F.gphi[l][w.g] * w.S;
        for (int c = 0; c < 3; ++c) {
          Dn As = (1.0 - s) * F.An[c][w.g] + s * F.Anp1[c][w.g];
          for (int l = 0; l < d; ++l) D[c][l] += wq * As * w.dS[l];
        }
        if (dep && w.S.v != 0.0) dep->w.push_back({w.g, wq * w.S});
      }
    }
  }
  Dn Am[3], Ap[3], xe[3];
  interp3(C, F.An, p.x, Am);
  for (int l = 0; l < 3; ++l) xe[l] = l < d ? p.x[l] + dt * vin[l] : cst(0.0);
  interp3(C, F.Anp1, xe, Ap);
  const Dn& q = p.q;
  const Dn& m = p.m;
  Dn Aep[3], kick[3], pm[3];
  for (int c = 0; c < 3; ++c) {
    Aep[c] = 0.5 * (Am[c] + Ap[c]);
    Dn Dv = cst(0.0);
    for (int l = 0; l < d; ++l) Dv += D[c][l] * vin[l];
    kick[c] = 0.5 * dt * q * Dv;
    if (c < d) kick[c] -= 0.5 * dt * q * gp[c];
    pm[c] = p.P[c] - q * Aep[c] + kick[c];
  }
  // B_eff = (K23, -K13, K12) of K = D~^T - D~ with D~ the zero-padded 3x3 D.
  auto Dz = [&](int c, int l) { return l < d ? D[c][l] : cst(0.0); };
  Dn Beff[3] = {Dz(2, 1) - Dz(1, 2), -(Dz(2, 0) - Dz(0, 2)), Dz(1, 0) - Dz(0, 1)};
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
  const Mesh& M = C.M;
  const double h = C.cfg.dt, kap2 = C.cfg.kappa * C.cfg.kappa;
  Spec jh[3];
  for (int c = 0; c < 3; ++c) {
    jh[c] = to_spec(M, j[c]);
    project(M, jh[c], C.cfg.project != 0);
  }
  T.phi = T.psi = T.rho = zero_spec(M);
  for (int c = 0; c < 3; ++c) T.A[c] = T.U[c] = zero_spec(M);
  Spec phih = zero_spec(M);
  for (int g = 0; g < M.Ng; ++g) {
    double k[3];
    bool nyq;
    kvec(M, g, k, nyq);
    const double a = kap2 * (k[0] * k[0] + k[1] * k[1] + k[2] * k[2]), den = 1.0 + h * h * a / 4.0;
    for (int l = 0; l <= ND; ++l) {
      // continuity: rho^{n+1} = rho^n - dt i k . jh
      const cplx divj = cplx(0.0, k[0]) * jh[0][l][g] + cplx(0.0, k[1]) * jh[1][l][g] + cplx(0.0, k[2]) * jh[2][l][g];
      T.rho[l][g] = S.rho[l][g] - h * divj;
      const cplx rh = 0.5 * (S.rho[l][g] + T.rho[l][g]);
      T.phi[l][g] = ((1.0 - h * h * a / 4.0) * S.phi[l][g] + h * S.psi[l][g] + 0.5 * h * h * kap2 * C.cfg.sigma1 * rh) / den;
      T.psi[l][g] = 2.0 * (T.phi[l][g] - S.phi[l][g]) / h - S.psi[l][g];
      phih[l][g] = 0.5 * (S.phi[l][g] + T.phi[l][g]);
      for (int c = 0; c < 3; ++c) {
        T.A[c][l][g] = ((1.0 - h * h * a / 4.0) * S.A[c][l][g] + h * S.U[c][l][g] +
                        0.5 * h * h * kap2 * C.cfg.sigma2 * jh[c][l][g]) / den;
        T.U[c][l][g] = 2.0 * (T.A[c][l][g] - S.A[c][l][g]) / h - S.U[c][l][g];
      }
    }
  }
  for (int l = 0; l < M.d; ++l) F.gphi[l] = to_real(M, dspec(M, phih, l));
  for (int c = 0; c < 3; ++c) {
    F.An[c] = to_real(M, S.A[c]);
    F.Anp1[c] = to_real(M, T.A[c]);
  }
}

// Energies of the state: field energy W = sum (|E|^2 / (2 sigma1) + |B|^2 / (2 sigma2)) dV
// with E = -grad phi - U and B = curl A; kinetic energy
// sum |p|^2 / (m (gamma + 1)) with p = P - q A_h(x).
void energies(const Ctx& C, const State& S, const std::vector<Part>& parts, Dn& W, Dn& K) {
  const Mesh& M = C.M;
  DVec gph[3], U[3], A[3], dA[3][3];
  for (int l = 0; l < 3; ++l) gph[l] = to_real(M, dspec(M, S.phi, l));
  for (int c = 0; c < 3; ++c) {
    U[c] = to_real(M, S.U[c]);
    A[c] = to_real(M, S.A[c]);
    for (int l = 0; l < 3; ++l) dA[c][l] = to_real(M, dspec(M, S.A[c], l));
  }
  W = cst(0.0);
  for (int g = 0; g < M.Ng; ++g) {
    Dn E[3] = {-gph[0][g] - U[0][g], -gph[1][g] - U[1][g], -gph[2][g] - U[2][g]};
    Dn B[3] = {dA[2][1][g] - dA[1][2][g], dA[0][2][g] - dA[2][0][g], dA[1][0][g] - dA[0][1][g]};
    Dn e2 = E[0] * E[0] + E[1] * E[1] + E[2] * E[2], b2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
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
  const int n = C.M.Ng;
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
  const Mesh& M = C.M;
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
    for (int c = 0; c < 3; ++c) Jd[c].assign(M.Ng, cst(0.0));
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
      for (int g = 0; g < M.Ng; ++g) {
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
        for (int l = 0; l < M.d; ++l) {
          Dn xe = p.x[l] + C.cfg.dt * vin[i][l];
          const double k = std::floor((xe.v - M.lo[l]) / M.L[l]);  // periodic image, a constant shift
          p.x[l] = xe - k * M.L[l];
          if (p.x[l].v >= M.lo[l] + M.L[l]) p.x[l] -= cst(M.L[l]);
          if (p.x[l].v < M.lo[l]) p.x[l] += cst(M.L[l]);
        }
        for (int c = 0; c < 3; ++c) {
          p.P[c] = Pn1[i][c];
          p.vbar[c] = vw[i][c];
        }
      }
      return 0;
    }
    for (int c = 0; c < 3; ++c)
      for (int g = 0; g < M.Ng; ++g) j[c][g] += C.cfg.beta * (H[c][g] - j[c][g]);
  }
  return -6;
}

// Initialization (Nyquist-projection paragraph and the constraint discussion) with zero
// initial potentials: projected charge and current from a point-shape deposit, the
// neutralizing background cancelling the mean charge, phi from Gauss's law
// (-Lap phi = sigma1 rho), psi = A = U = 0, canonical momenta P = p.
void initialize(const Ctx& C, std::vector<Part>& parts, State& S) {
  const Mesh& M = C.M;
  DVec rho(M.Ng, cst(0.0)), J[3];
  for (int c = 0; c < 3; ++c) J[c].assign(M.Ng, cst(0.0));
  std::vector<NodeW> nw;
  for (Part& p : parts) {
    Dn g = gamma_of(p.P, p.m, C.cfg.kappa);
    Dn v[3];
    for (int c = 0; c < 3; ++c) v[c] = p.P[c] / (p.m * g);
    Dn xi[3];
    for (int l = 0; l < 3; ++l) xi[l] = l < M.d ? (p.x[l] - M.lo[l]) / M.h[l] : cst(0.0);
    node_weights(M, xi, nw);
    for (const NodeW& w : nw) {
      if (w.S.v == 0.0) continue;
      rho[w.g] += p.q * w.S / M.dV;
      for (int c = 0; c < 3; ++c) J[c][w.g] += p.q * v[c] * w.S / M.dV;
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
  for (int g = 0; g < M.Ng; ++g) {
    double k[3];
    bool nyq;
    kvec(M, g, k, nyq);
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    if (k2 > 0.0)
      for (int l = 0; l <= ND; ++l) S.phi[l][g] = C.cfg.sigma1 * S.rho[l][g] / k2;
  }
}

}  // namespace

extern "C" {

// Tangent-linear run: n particles x [dim][n], u [3][n], q [n] (m = |q|) with nd <= 16 seed
// directions dx [nd][dim][n], du [nd][3][n], dq [nd][n] (the derivatives of the inputs along
// each direction); steps implicit steps.  Out: E[4] = (W^0, K^0, W^T, K^T) and
// dE[4][nd] their derivatives along each direction; *outer the map evaluations summed
// over the steps.  Status 0, -1 (unsupported configuration), -5 (a particle solve
// failed), -6 (no outer convergence).
int orc_tangent_run(const orc_config* cfg, int64_t n, const double* x, const double* u, const double* q, int nd,
                    const double* dx, const double* du, const double* dq, int steps, double* E, double* dE,
                    int64_t* outer) {
  if (cfg->dim < 1 || cfg->dim > 3 || (cfg->shape_order != 0 && cfg->shape_order != 2) || cfg->outer_scheme != 0 ||
      cfg->refine_levels != 0 || nd < 0 || nd > kMaxDir || cfg->gl_order < 1 || cfg->gl_order > 64)
    return -1;
  const int d = cfg->dim;
  ND = nd;
  Ctx C;
  C.cfg = *cfg;
  C.M.d = d;
  C.M.dV = 1.0;
  for (int l = 0; l < 3; ++l) {
    C.M.n[l] = l < d ? cfg->n[l] : 1;
    C.M.lo[l] = l < d ? cfg->lo[l] : 0.0;
    C.M.L[l] = l < d ? cfg->len[l] : 1.0;
    C.M.h[l] = C.M.L[l] / C.M.n[l];
    if (l < d) {
      if (C.M.n[l] < 4 || (C.M.n[l] & (C.M.n[l] - 1)) != 0) return -1;
      C.M.dV *= C.M.h[l];
    }
  }
  C.M.Ng = C.M.n[0] * C.M.n[1] * C.M.n[2];
  C.ngl = cfg->gl_order;
  orc_gl_rule(C.ngl, C.glx, C.glw);
  std::vector<Part> parts(n);
  for (int64_t i = 0; i < n; ++i) {
    Part& p = parts[i];
    p.q = cst(q[i]);
    Dn uu[3];
    for (int c = 0; c < 3; ++c) uu[c] = cst(u[c * n + i]);
    for (int l = 0; l < 3; ++l) p.x[l] = cst(l < d ? x[l * n + i] : 0.0);
    for (int k = 0; k < nd; ++k) {
      for (int l = 0; l < d; ++l) p.x[l].d[k] = dx[(k * d + l) * n + i];
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
