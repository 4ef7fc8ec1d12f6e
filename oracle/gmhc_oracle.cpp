// gmhc_oracle.cpp -- plain FP64 CPU oracle of the energy-conserving relativistic
// generalized-momentum Higuera-Cary / Crank-Nicolson (GM-HC-CN) potential PIC step
// of Christlieb, Chacon and Gong, "An Energy-Conserving Unstaggered
// Electromagnetic-Potential Particle-in-Cell Method, Part II".
//
// TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the GPU
// path is checked against.  It shares no code, header, table or generator with the
// GPU library, and only the test suite, the smoke check and the CPU-baseline leg of
// the benchmark may load it.  It is deliberately slow and literal: loops over
// particles, over Gauss-Legendre points on each knot-split orbit segment and over
// every candidate mesh node, with each formula written as the paper states it.
//
// Readings of points the paper leaves open are marked "Reading:" in the comments.
//
// Layout conventions (shared only as a specification with the GPU side):
//   mesh node g = i0 + n0*(i1 + n1*i2), node i at lo + i*h (periodic);
//   real mesh arrays are [component][Ng]; particle arrays are [component][Np].
#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include "orc_config.h"
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cplx = std::complex<double>;
const double kPi = 3.14159265358979323846264338327950288;

enum Status {
  ORC_OK = 0,
  ORC_EINVAL = -1,
  ORC_ESTATE = -2,
  ORC_EINNER = -5,
  ORC_ENOCONV = -6,
};

}  // namespace

extern "C" {

// Run parameters: struct orc_config in orc_config.h.

// One orbit evaluation v_out = F(v_in) of one particle at frozen trial fields.
struct orc_eval_out {
  double vout[3];       // orbit velocity from the two electric-work secant velocities
  double Pnp1[3];       // canonical momentum at n+1
  double pminus[3];     // mechanical momentum after the first half transform
  double pplus[3];      // after the HC rotation
  double pn[3];         // P^n - q A_h^n(x^n)
  double pnp1[3];       // P^{n+1} - q A_h^{n+1}(x^{n+1})
  double Aminus[3];     // A_h^n(x^n)
  double Aplus[3];      // A_h^{n+1}(x^n + dt v_in)
  double gradphibar[3]; // orbit gather of grad phi^{n+1/2}
  double Ubar[3];       // orbit gather of U^{n+1/2}
  double D[9];          // orbit discrete gradient, D[l*3+j] = int A_l(s) d_j S ds (j<d)
  double Beff[3];       // axial vector of K = D^T - D
  double gammaHC;       // HC Lorentz factor of the magnetic substep
  int32_t nseg;         // knot-split segments
};

struct orc_report {
  int32_t outer_iters;
  int32_t inner_max;        // max inner count over particles, final map evaluation
  double inner_mean;        // mean inner count, final map evaluation
  int64_t evaluations;      // orbit evaluations over all outer iterations
  double res_rms_ratio;     // RMS test ratio at exit (<=1 passes)
  double res_max_ratio;     // max-node test ratio at exit
  int32_t outer_updates;    // accepted outer updates (the algorithm's outer iterations are this + 1)
  int32_t refined;          // particles solved with sub-steps, final map evaluation
};

struct orc_diag {
  double t;
  int64_t step;
  double kinetic;           // sum m kappa^2 (gamma-1)
  double field;             // W
  double total;             // kinetic + field
  double energy_rel;        // |E - E0| / |E0|
  double gauss_rms;
  double lorenz_rms;
  double chain_rms;         // R_A of the last accepted step
  double work_residual;     // R_work of the last accepted step
  double vperp_rms;
  double res_rms_ratio;
  double res_max_ratio;
};

}  // extern "C"

namespace {

// ---------------------------------------------------------------------------
// Gauss-Legendre rule on [0,1]: Newton iteration on the Legendre polynomial P_n
// (three-term recurrence), nodes ascending.  Used on every knot-split orbit
// segment (results section: order eight on every knot-split interval).
void gauss_legendre01(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 200; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pn = (n == 1) ? z : p1;
      double pm = (n == 1) ? 1.0 : p0;
      dp = n * (z * pn - pm) / (z * z - 1.0);
      double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    // recompute derivative at the converged root
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double pn = (n == 1) ? z : p1;
    double pm = (n == 1) ? 1.0 : p0;
    dp = n * (z * pn - pm) / (z * z - 1.0);
    x[i] = 0.5 * (1.0 + z);
    w[i] = 0.5 * 2.0 / ((1.0 - z * z) * dp * dp);
  }
  // sort ascending by node
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (x[j] < x[i]) {
        std::swap(x[i], x[j]);
        std::swap(w[i], w[j]);
      }
}

// ---------------------------------------------------------------------------
// Centered quadratic B-spline S_2 (particle-shape paragraph of the solver section):
//   S2(xi) = 1/2 [ ((3/2-|xi|)_+)^2 - 3 ((1/2-|xi|)_+)^2 ],  and its derivative.
double S2(double xi) {
  double a = std::fabs(xi);
  double t1 = std::max(1.5 - a, 0.0);
  double t2 = std::max(0.5 - a, 0.0);
  return 0.5 * (t1 * t1 - 3.0 * t2 * t2);
}
double dS2(double xi) {
  double a = std::fabs(xi);
  double t1 = std::max(1.5 - a, 0.0);
  double t2 = std::max(0.5 - a, 0.0);
  double sg = (xi > 0.0) ? 1.0 : ((xi < 0.0) ? -1.0 : 0.0);
  return -sg * (t1 - 3.0 * t2);
}

// Centered linear B-spline S_1(xi) = (1-|xi|)_+, the degree the solver section raises
// to two (and the r = 1 case of the spline-degree comparison in the results section),
// and its derivative (one-sided value -sign(xi) inside the support, zero at the knots
// xi = 0 and |xi| = 1, where quadrature never evaluates it).
double S1(double xi) { return std::max(1.0 - std::fabs(xi), 0.0); }
double dS1(double xi) {
  double a = std::fabs(xi);
  if (a >= 1.0 || xi == 0.0) return 0.0;
  return xi > 0.0 ? -1.0 : 1.0;
}

// ---------------------------------------------------------------------------
// Mesh geometry.
struct Mesh {
  int d;
  int r;  // B-spline degree of the particle shape (1 or 2)
  int n[3];
  double lo[3], len[3], h[3];
  int64_t Ng;
  double dV;  // cell measure: product of h over the resolved axes
  int64_t node(int64_t i0, int64_t i1, int64_t i2) const {
    auto w = [](int64_t i, int nn) { return ((i % nn) + nn) % nn; };
    return w(i0, n[0]) + (int64_t)n[0] * (w(i1, n[1]) + (int64_t)n[1] * w(i2, n[2]));
  }
};

// Shape weights of all candidate nodes around one point.  For each resolved axis,
// five candidates floor(xi)-2 .. floor(xi)+2 are evaluated with the plain S_r
// definition (nodes outside the support simply get zero).
struct PointWeights {
  int64_t base[3];
  double S[3][5];
  double dS[3][5];  // derivative with respect to x (not xi)
  int cnt[3];
};

void point_weights(const Mesh& M, const double x[3], PointWeights& pw) {
  for (int l = 0; l < 3; ++l) {
    if (l < M.d) {
      double xi = (x[l] - M.lo[l]) / M.h[l];
      int64_t b = (int64_t)std::floor(xi) - 2;
      pw.base[l] = b;
      pw.cnt[l] = 5;
      for (int c = 0; c < 5; ++c) {
        double r = xi - (double)(b + c);
        pw.S[l][c] = M.r == 1 ? S1(r) : S2(r);
        pw.dS[l][c] = (M.r == 1 ? dS1(r) : dS2(r)) / M.h[l];
      }
    } else {
      pw.base[l] = 0;
      pw.cnt[l] = 1;
      pw.S[l][0] = 1.0;
      pw.dS[l][0] = 0.0;
    }
  }
}

// Point interpolant A_h(x) = sum_g A_g S_g(x) of a 3-component mesh array.
void interp3(const Mesh& M, const double* const F[3], const double x[3], double out[3]) {
  PointWeights pw;
  point_weights(M, x, pw);
  out[0] = out[1] = out[2] = 0.0;
  for (int c2 = 0; c2 < pw.cnt[2]; ++c2)
    for (int c1 = 0; c1 < pw.cnt[1]; ++c1)
      for (int c0 = 0; c0 < pw.cnt[0]; ++c0) {
        double S = pw.S[0][c0] * pw.S[1][c1] * pw.S[2][c2];
        int64_t g = M.node(pw.base[0] + c0, pw.base[1] + c1, pw.base[2] + c2);
        for (int c = 0; c < 3; ++c) out[c] += F[c][g] * S;
      }
}

// ---------------------------------------------------------------------------
// Knot split of the straight unwrapped orbit x(s) = x + s dx, s in [0,1]
// (orbit-averaged maps section; knot-split Gaussian quadrature).  Knots of S2
// centred at nodes lo + g h lie at lo + (j+1/2) h; those of S1 at the nodes lo + j h.  Reading: a crossing counts
// only if 0 < s < 1 strictly; zero-length segments are dropped.
void knot_split(const Mesh& M, const double x[3], const double dx[3], std::vector<double>& s) {
  s.clear();
  s.push_back(0.0);
  s.push_back(1.0);
  for (int l = 0; l < M.d; ++l) {
    if (dx[l] == 0.0) continue;
    double xi0 = (x[l] - M.lo[l]) / M.h[l];
    double dxi = dx[l] / M.h[l];
    double a = std::min(xi0, xi0 + dxi), b = std::max(xi0, xi0 + dxi);
    for (int64_t j = (int64_t)std::floor(a) - 1; j <= (int64_t)std::ceil(b) + 1; ++j) {
      double sk = ((double)j + (M.r == 1 ? 0.0 : 0.5) - xi0) / dxi;
      if (sk > 0.0 && sk < 1.0) s.push_back(sk);
    }
  }
  std::sort(s.begin(), s.end());
  s.erase(std::unique(s.begin(), s.end()), s.end());
}

struct FieldPtrs {
  const double* gphi[3];  // grad_h phi^{n+1/2}; components >= d are null (zero)
  const double* An[3];
  const double* Anp1[3];
  const double* Uh[3];    // U^{n+1/2}
};

struct Phys {
  double kappa, dt;
};

double gamma_of(const double p[3], double m, double kappa) {
  double u2 = (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) / (m * m * kappa * kappa);
  return std::sqrt(1.0 + u2);
}

// Secant (discrete-gradient) velocity of the relativistic kinetic energy:
//   V^dg(pa, pb) = (pa + pb) / (m (gamma(pa) + gamma(pb))).
void vdg(const double pa[3], const double pb[3], double m, double kappa, double out[3]) {
  double den = m * (gamma_of(pa, m, kappa) + gamma_of(pb, m, kappa));
  for (int c = 0; c < 3; ++c) out[c] = (pa[c] + pb[c]) / den;
}

void cross(const double a[3], const double b[3], double out[3]) {
  out[0] = a[1] * b[2] - a[2] * b[1];
  out[1] = a[2] * b[0] - a[0] * b[2];
  out[2] = a[0] * b[1] - a[1] * b[0];
}

// Normalized HC magnetic map (definition of the normalized map):
//   tau = (q dt / 2m) B, sigma = gamma^-2 - |tau|^2,
//   gamma_HC = sqrt( [sigma + sqrt(sigma^2 + 4(|tau|^2 + (u.tau)^2))] / 2 ),
//   t = tau/gamma_HC, s = 2t/(1+|t|^2), u* = u + u x t, u+ = u + u* x s.
// Reading: for sigma < 0 the same root is evaluated as 2X/(R - sigma) to avoid
// cancellation (identical mathematics).  Takes tau directly.
double hc_map_u(const double um[3], const double tau[3], double up[3]) {
  double gm2 = 1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2];
  double tau2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];
  double ut = um[0] * tau[0] + um[1] * tau[1] + um[2] * tau[2];
  double sigma = gm2 - tau2;
  double X = tau2 + ut * ut;
  double R = std::sqrt(sigma * sigma + 4.0 * X);
  double g2 = (sigma >= 0.0) ? 0.5 * (sigma + R) : 2.0 * X / (R - sigma);
  double gHC = std::sqrt(g2);
  double t[3] = {tau[0] / gHC, tau[1] / gHC, tau[2] / gHC};
  double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  double s[3] = {2.0 * t[0] / (1.0 + t2), 2.0 * t[1] / (1.0 + t2), 2.0 * t[2] / (1.0 + t2)};
  double uxt[3];
  cross(um, t, uxt);
  double ustar[3] = {um[0] + uxt[0], um[1] + uxt[1], um[2] + uxt[2]};
  double usxs[3];
  cross(ustar, s, usxs);
  for (int c = 0; c < 3; ++c) up[c] = um[c] + usxs[c];
  return gHC;
}

// Orbit quadrature accumulator: for one orbit (x, dx) accumulate, with GL on each
// knot-split segment, the gathers of grad phi^{n+1/2} and U^{n+1/2}, the orbit
// discrete gradient D (orbit discrete-gradient definition, A_g(s) linear in s),
// and optionally the orbit-averaged shape weights S-bar as (node, weight) pairs.
struct OrbitSums {
  double gphi[3];
  double Ubar[3];
  double D[3][3];
  int nseg;
};

void orbit_quadrature(const Mesh& M, const FieldPtrs* F, int ngl, const double* glx,
                      const double* glw, const double x[3], const double dx[3], OrbitSums* o,
                      std::vector<std::pair<int64_t, double>>* sbar) {
  std::vector<double> brk;
  knot_split(M, x, dx, brk);
  if (o) {
    std::memset(o, 0, sizeof(*o));
    o->nseg = (int)brk.size() - 1;
  }
  for (size_t k = 0; k + 1 < brk.size(); ++k) {
    double a = brk[k], b = brk[k + 1];
    for (int q = 0; q < ngl; ++q) {
      double s = a + (b - a) * glx[q];
      double wq = (b - a) * glw[q];
      double xs[3] = {x[0] + s * dx[0], x[1] + s * dx[1], x[2] + s * dx[2]};
      PointWeights pw;
      point_weights(M, xs, pw);
      for (int c2 = 0; c2 < pw.cnt[2]; ++c2)
        for (int c1 = 0; c1 < pw.cnt[1]; ++c1)
          for (int c0 = 0; c0 < pw.cnt[0]; ++c0) {
            double S = pw.S[0][c0] * pw.S[1][c1] * pw.S[2][c2];
            double dS[3] = {pw.dS[0][c0] * pw.S[1][c1] * pw.S[2][c2],
                            pw.S[0][c0] * pw.dS[1][c1] * pw.S[2][c2],
                            pw.S[0][c0] * pw.S[1][c1] * pw.dS[2][c2]};
            int64_t g = M.node(pw.base[0] + c0, pw.base[1] + c1, pw.base[2] + c2);
            if (o && F) {
              for (int l = 0; l < 3; ++l) {
                if (F->gphi[l]) o->gphi[l] += wq * F->gphi[l][g] * S;
                o->Ubar[l] += wq * F->Uh[l][g] * S;
                double Als = (1.0 - s) * F->An[l][g] + s * F->Anp1[l][g];
                for (int j = 0; j < M.d; ++j) o->D[l][j] += wq * Als * dS[j];
              }
            }
            if (sbar && S != 0.0) sbar->push_back({g, wq * S});
          }
    }
  }
}

// One orbit evaluation F(v_in) (no-explicit-A_t GM-HC step, mechanical endpoints,
// electric-work velocities and orbit velocity of the energy section).
void orbit_eval(const Mesh& M, const Phys& ph, const FieldPtrs& F, int ngl, const double* glx,
                const double* glw, const double x[3], const double P[3], double q, double m,
                const double vin[3], orc_eval_out* o) {
  const double dt = ph.dt, kappa = ph.kappa;
  double dx[3] = {0.0, 0.0, 0.0};
  for (int l = 0; l < M.d; ++l) dx[l] = dt * vin[l];
  OrbitSums os;
  orbit_quadrature(M, &F, ngl, glx, glw, x, dx, &os, nullptr);
  double xe[3] = {x[0] + dx[0], x[1] + dx[1], x[2] + dx[2]};
  double Am[3], Ap[3];
  interp3(M, F.An, x, Am);
  interp3(M, F.Anp1, xe, Ap);
  double Aep[3], Dv[3], kick[3];
  for (int c = 0; c < 3; ++c) {
    Aep[c] = 0.5 * (Am[c] + Ap[c]);
    Dv[c] = 0.0;
    for (int j = 0; j < M.d; ++j) Dv[c] += os.D[c][j] * vin[j];
    kick[c] = -0.5 * q * dt * os.gphi[c] + 0.5 * q * dt * Dv[c];
  }
  double pm[3];
  for (int c = 0; c < 3; ++c) pm[c] = P[c] - q * Aep[c] + kick[c];
  // B_eff(K), K = D~^T - D~ with D~ the 3x3 zero-padded D; B_eff = (K23, -K13, K12).
  double Beff[3] = {os.D[2][1] - os.D[1][2], -(os.D[2][0] - os.D[0][2]), os.D[1][0] - os.D[0][1]};
  double um[3] = {pm[0] / (m * kappa), pm[1] / (m * kappa), pm[2] / (m * kappa)};
  double tau[3] = {q * dt / (2.0 * m) * Beff[0], q * dt / (2.0 * m) * Beff[1],
                   q * dt / (2.0 * m) * Beff[2]};
  double up[3];
  double gHC = hc_map_u(um, tau, up);
  double pp[3] = {m * kappa * up[0], m * kappa * up[1], m * kappa * up[2]};
  double Pn1[3], pn[3], pn1[3];
  for (int c = 0; c < 3; ++c) {
    Pn1[c] = pp[c] + q * Aep[c] + kick[c];
    pn[c] = P[c] - q * Am[c];
    pn1[c] = Pn1[c] - q * Ap[c];
  }
  double vEm[3], vEp[3];
  vdg(pm, pn, m, kappa, vEm);
  vdg(pn1, pp, m, kappa, vEp);
  for (int c = 0; c < 3; ++c) {
    o->vout[c] = 0.5 * (vEm[c] + vEp[c]);
    o->Pnp1[c] = Pn1[c];
    o->pminus[c] = pm[c];
    o->pplus[c] = pp[c];
    o->pn[c] = pn[c];
    o->pnp1[c] = pn1[c];
    o->Aminus[c] = Am[c];
    o->Aplus[c] = Ap[c];
    o->gradphibar[c] = os.gphi[c];
    o->Ubar[c] = os.Ubar[c];
    o->Beff[c] = Beff[c];
    for (int j = 0; j < 3; ++j) o->D[c * 3 + j] = os.D[c][j];
  }
  o->gammaHC = gHC;
  o->nseg = os.nseg;
}

// ---------------------------------------------------------------------------
// FFT: iterative radix-2 Cooley-Tukey, forward unnormalized (exp(-i...)), inverse
// scaled by 1/N.  Multi-dimensional transforms apply it along each axis.
void fft1(cplx* a, int n, int stride, bool inverse) {
  std::vector<cplx> buf(n);
  for (int i = 0; i < n; ++i) buf[i] = a[(int64_t)i * stride];
  for (int i = 1, j = 0; i < n; ++i) {
    int bit = n >> 1;
    for (; j & bit; bit >>= 1) j ^= bit;
    j ^= bit;
    if (i < j) std::swap(buf[i], buf[j]);
  }
  for (int len = 2; len <= n; len <<= 1) {
    double ang = 2.0 * kPi / len * (inverse ? 1.0 : -1.0);
    for (int i = 0; i < n; i += len)
      for (int k = 0; k < len / 2; ++k) {
        cplx w(std::cos(ang * k), std::sin(ang * k));
        cplx u = buf[i + k], v = buf[i + k + len / 2] * w;
        buf[i + k] = u + v;
        buf[i + k + len / 2] = u - v;
      }
  }
  double sc = inverse ? 1.0 / n : 1.0;
  for (int i = 0; i < n; ++i) a[(int64_t)i * stride] = buf[i] * sc;
}

void fftn(const Mesh& M, cplx* a, bool inverse) {
  int n0 = M.n[0], n1 = M.n[1], n2 = M.n[2];
  if (n0 > 1)
    for (int i2 = 0; i2 < n2; ++i2)
      for (int i1 = 0; i1 < n1; ++i1) fft1(a + (int64_t)n0 * (i1 + (int64_t)n1 * i2), n0, 1, inverse);
  if (n1 > 1)
    for (int i2 = 0; i2 < n2; ++i2)
      for (int i0 = 0; i0 < n0; ++i0) fft1(a + i0 + (int64_t)n0 * n1 * i2, n1, n0, inverse);
  if (n2 > 1)
    for (int i1 = 0; i1 < n1; ++i1)
      for (int i0 = 0; i0 < n0; ++i0) fft1(a + i0 + (int64_t)n0 * i1, n2, n0 * n1, inverse);
}

// Spectral derivative symbol of axis l at unshifted index m: k = 2 pi m_s / L with
// the signed index m_s; zero at the even-grid Nyquist index (Nyquist paragraph).
double ksym(const Mesh& M, int l, int m) {
  int n = M.n[l];
  if (l >= M.d) return 0.0;
  if (n % 2 == 0 && m == n / 2) return 0.0;
  int ms = (m <= n / 2) ? m : m - n;
  return 2.0 * kPi * ms / M.len[l];
}

bool is_nyquist(const Mesh& M, int64_t g) {
  int64_t i0 = g % M.n[0], i1 = (g / M.n[0]) % M.n[1], i2 = g / ((int64_t)M.n[0] * M.n[1]);
  int64_t idx[3] = {i0, i1, i2};
  for (int l = 0; l < M.d; ++l)
    if (M.n[l] % 2 == 0 && idx[l] == M.n[l] / 2) return true;
  return false;
}

void kvec(const Mesh& M, int64_t g, double k[3]) {
  int64_t i0 = g % M.n[0], i1 = (g / M.n[0]) % M.n[1], i2 = g / ((int64_t)M.n[0] * M.n[1]);
  k[0] = ksym(M, 0, (int)i0);
  k[1] = ksym(M, 1, (int)i1);
  k[2] = ksym(M, 2, (int)i2);
}

using CVec = std::vector<cplx>;
using RVec = std::vector<double>;

CVec to_spec(const Mesh& M, const double* r) {
  CVec a(M.Ng);
  for (int64_t g = 0; g < M.Ng; ++g) a[g] = cplx(r[g], 0.0);
  fftn(M, a.data(), false);
  return a;
}
RVec to_real(const Mesh& M, const CVec& s) {
  CVec a = s;
  fftn(M, a.data(), true);
  RVec r(M.Ng);
  for (int64_t g = 0; g < M.Ng; ++g) r[g] = a[g].real();
  return r;
}
// Nyquist projector: zero every mode on an even-grid Nyquist plane.
void project(const Mesh& M, CVec& a) {
  for (int64_t g = 0; g < M.Ng; ++g)
    if (is_nyquist(M, g)) a[g] = 0.0;
}
// d/dx_l in spectral space (i k_l)
CVec dspec(const Mesh& M, const CVec& a, int l) {
  CVec b(M.Ng);
  for (int64_t g = 0; g < M.Ng; ++g) {
    double k[3];
    kvec(M, g, k);
    b[g] = cplx(0.0, k[l]) * a[g];
  }
  return b;
}

// ---------------------------------------------------------------------------
struct Sim {
  orc_config cfg;
  Mesh M;
  Phys ph;
  std::vector<double> glx, glw;
  // particles
  int64_t np = 0;
  RVec x[3], P[3], vbar[3], q, m;
  // accepted spectral field state at time level n
  CVec phi, psi, rho, A[3], U[3];
  RVec Jacc[3];  // accepted current J^{n-1/2}: initial trial of the next step
  bool initialized = false;
  double t = 0.0;
  int64_t step = 0;
  double E0 = 0.0;
  double last_chain_rms = 0.0, last_work = 0.0, last_rms_ratio = 0.0, last_max_ratio = 0.0;
  // frozen fields for single-pass tests
  RVec fz_gphi[3], fz_An[3], fz_Anp1[3], fz_Uh[3];
  bool have_frozen = false;
  // refinement level of each particle within the current step (0: the full step)
  std::vector<int32_t> level;
};

int setup_mesh(const orc_config* c, Mesh& M, bool need_pow2 = false) {
  if (c->dim < 1 || c->dim > 3) return ORC_EINVAL;
  M.d = c->dim;
  M.r = c->shape_order == 0 ? 2 : c->shape_order;
  if (M.r != 1 && M.r != 2) return ORC_EINVAL;
  M.Ng = 1;
  M.dV = 1.0;
  for (int l = 0; l < 3; ++l) {
    M.n[l] = (l < c->dim) ? c->n[l] : 1;
    M.lo[l] = (l < c->dim) ? c->lo[l] : 0.0;
    M.len[l] = (l < c->dim) ? c->len[l] : 1.0;
    if (M.n[l] < 1) return ORC_EINVAL;
    if (l < c->dim) {
      if (need_pow2 && (M.n[l] & (M.n[l] - 1)) != 0) return ORC_EINVAL;  // radix-2 FFT
      if (!(M.len[l] > 0.0)) return ORC_EINVAL;
    }
    M.h[l] = M.len[l] / M.n[l];
    M.Ng *= M.n[l];
    if (l < c->dim) M.dV *= M.h[l];
  }
  return ORC_OK;
}

FieldPtrs make_ptrs(const Sim& S, const RVec gphi[3], const RVec An[3], const RVec Anp1[3],
                    const RVec Uh[3]) {
  FieldPtrs F;
  for (int l = 0; l < 3; ++l) {
    F.gphi[l] = (l < S.M.d) ? gphi[l].data() : nullptr;
    F.An[l] = An[l].data();
    F.Anp1[l] = Anp1[l].data();
    F.Uh[l] = Uh[l].data();
  }
  return F;
}

// ---- Convergence-triggered particle refinement (spline-degree comparison of the
// results section): a particle whose inner solve over the full step fails is solved
// again with K = 2, 4, ..., 2^refine_levels equal particle sub-steps of dt/K while the
// field step stays fixed.  The paper says only that; the rest is this reading:
//  * sub-step k covers the fraction [k/K, (k+1)/K] of the step, with the step's fields
//    restricted to it: grad phi^{n+1/2} and U^{n+1/2} as they are, and as vector
//    potentials at its ends A(k/K) and A((k+1)/K) of the interpolant
//    A(s) = (1-s) A^n + s A^{n+1} that the orbit discrete gradient already uses.  The
//    sub-step is the full-step particle map with these fields and dt/K, started from the
//    position and canonical momentum the previous sub-step ended with; the endpoint
//    potential of one sub-step is then the starting one of the next.
//  * each sub-step runs the same inner Picard loop (tests and limit), warm-started from
//    the particle's warm start (k = 0) or the previous sub-step's v_out.
//  * the orbit current is the time average of the sub-step orbit currents,
//    J += (1/K) sum_k q v_out,k Sbar_k / dV.  With this weight the particle work of the
//    sub-steps, sum_k (dt/K) q v_out,k . (-grad-phi-bar_k - U-bar_k), equals the mesh work
//    of the deposit term by term (the particle-grid work identity of the energy proof),
//    so a refined step conserves energy like an unrefined one.
//  * within a step a particle's level only rises (every step starts at the full step),
//    so once the levels have settled the outer map is one fixed function of the trial
//    current.
//  * the accepted orbit velocity of a refined particle (its warm start for the next
//    evaluation) is the mean of its sub-step v_out; its position is the end of its last
//    sub-step.
const int kMaxRefine = 3;

struct SubStep {
  double x[3];     // start of the sub-step orbit (unwrapped)
  double vin[3];   // converged v_in: the orbit x + s (dt/K) v_in, s in [0, 1]
  double vout[3];  // its v_out
};

// One particle's solve over the field step.
struct ParticleSolve {
  bool ok = false;
  int evals = 0;              // orbit evaluations, failed attempts included
  int level = 0;              // level of the accepted solve (K = 2^level sub-steps); after a
                              // failure at every level, refine_levels + 1
  std::vector<SubStep> sub;   // sub-steps of a refined solve (empty at level 0)
  double vin[3] = {0, 0, 0};  // level 0: converged v_in; refined: mean over sub-steps
  double vout[3] = {0, 0, 0}; // level 0: its v_out; refined: mean over sub-steps
  double Pn1[3] = {0, 0, 0};  // canonical momentum at the end of the step
  double xend[3] = {0, 0, 0}; // end position (unwrapped)
  double Ra2 = 0.0;           // sum over sub-steps of |R_A|^2
  double work = 0.0;          // particle work / dt: sum_k (1/K) q v_out,k . (-gphibar_k - Ubar_k)
};

// Inner Picard loop of one particle over one (sub-)step of length ph.dt at fields F,
// from the warm start v (Algorithm 1, inner solve): true when the mixed test passes with
// finite, subluminal iterates.  v ends as the v_in of the last evaluation o.  With
// iterate false, one evaluation of v and success.
bool inner_solve(const Sim& S, const Phys& ph, const FieldPtrs& F, const double x[3], const double P[3],
                 int64_t i, bool iterate, double v[3], orc_eval_out& o, int& evals) {
  const int ngl = (int)S.glx.size();
  const int maxit = iterate ? S.cfg.max_inner : 1;
  for (int it = 1; it <= maxit; ++it) {
    orbit_eval(S.M, ph, F, ngl, S.glx.data(), S.glw.data(), x, P, S.q[i], S.m[i], v, &o);
    ++evals;
    if (!iterate) return true;
    double vn = std::sqrt(o.vout[0] * o.vout[0] + o.vout[1] * o.vout[1] + o.vout[2] * o.vout[2]);
    if (!std::isfinite(vn) || !(vn < S.cfg.kappa)) return false;  // finite and subluminal
    double dmax = 0.0, vmax = 0.0;
    for (int c = 0; c < 3; ++c) {
      dmax = std::max(dmax, std::fabs(o.vout[c] - v[c]));
      vmax = std::max(vmax, std::fabs(o.vout[c]));
    }
    if (dmax <= S.cfg.tol_inner_abs + S.cfg.tol_inner_rel * vmax) return true;
    for (int c = 0; c < 3; ++c) v[c] = o.vout[c];
  }
  return false;
}

// Solve particle i over the step whose vector potential at the fractions j / kmax of the
// step is Ab[j] (j = 0..kmax, kmax = 2^refine_levels; Ab[0] = A^n, Ab[kmax] = A^{n+1}),
// with grad phi and U from F0, from the warm start vw, starting at level level0 and
// rising on failure up to refine_levels (iterate only).
void solve_particle(const Sim& S, const std::vector<std::array<const double*, 3>>& Ab, const FieldPtrs& F0,
                    int64_t i, const double vw[3], int level0, bool iterate, ParticleSolve& ps) {
  const Mesh& M = S.M;
  const int kmax = (int)Ab.size() - 1;
  const int top = iterate ? S.cfg.refine_levels : 0;
  for (int L = level0; L <= std::max(level0, top); ++L) {
    const int K = 1 << L;
    const double dtk = S.cfg.dt / K;
    const Phys ph{S.cfg.kappa, dtk};
    double x[3] = {S.x[0][i], S.x[1][i], S.x[2][i]};
    double P[3] = {S.P[0][i], S.P[1][i], S.P[2][i]};
    double warm[3] = {vw[0], vw[1], vw[2]};
    double vsum[3] = {0, 0, 0}, isum[3] = {0, 0, 0};
    ps.level = L;
    ps.sub.clear();
    ps.Ra2 = 0.0;
    ps.work = 0.0;
    bool ok = true;
    for (int k = 0; k < K && ok; ++k) {
      FieldPtrs F = F0;
      for (int c = 0; c < 3; ++c) {
        F.An[c] = Ab[k * (kmax / K)][c];
        F.Anp1[c] = Ab[(k + 1) * (kmax / K)][c];
      }
      double v[3] = {warm[0], warm[1], warm[2]};
      orc_eval_out o{};
      ok = inner_solve(S, ph, F, x, P, i, iterate, v, o, ps.evals);
      // the evaluation's chain-rule residual and work (accept-pass diagnostics)
      double Ra = 0.0, wk = 0.0;
      for (int c = 0; c < 3; ++c) {
        double Dv = 0.0;
        for (int j = 0; j < M.d; ++j) Dv += o.D[c * 3 + j] * v[j];
        double r = o.Aplus[c] - o.Aminus[c] - dtk * (o.Ubar[c] + Dv);
        Ra += r * r;
        wk += S.q[i] * o.vout[c] * (-o.gradphibar[c] - o.Ubar[c]);
      }
      ps.Ra2 += Ra;
      ps.work += wk / K;
      SubStep st;
      for (int c = 0; c < 3; ++c) {
        st.x[c] = x[c];
        st.vin[c] = v[c];
        st.vout[c] = o.vout[c];
        vsum[c] += o.vout[c];
        isum[c] += v[c];
        P[c] = o.Pnp1[c];
        warm[c] = o.vout[c];
      }
      if (K > 1) ps.sub.push_back(st);
      for (int l = 0; l < M.d; ++l) x[l] = x[l] + dtk * v[l];
      if (K == 1)
        for (int c = 0; c < 3; ++c) {
          ps.vin[c] = v[c];
          ps.vout[c] = o.vout[c];
        }
    }
    if (K > 1)
      for (int c = 0; c < 3; ++c) {
        ps.vin[c] = isum[c] / K;
        ps.vout[c] = vsum[c] / K;
      }
    for (int c = 0; c < 3; ++c) {
      ps.Pn1[c] = P[c];
      ps.xend[c] = x[c];
    }
    ps.ok = ok;
    if (ok) return;
  }
  // failed at every level: reported one past the finest (0 without refinement)
  ps.level = top > 0 ? top + 1 : 0;
}

// A^n, A^{n+1} and, with refinement, the interpolant A(j / kmax) = (1 - s) A^n + s A^{n+1}
// at the interior fractions s = j / kmax: store holds the interior arrays, Ab points at
// all kmax + 1.
void step_potentials(const Sim& S, const double* const An[3], const double* const Anp1[3],
                     std::vector<std::array<RVec, 3>>& store, std::vector<std::array<const double*, 3>>& Ab) {
  const int kmax = 1 << S.cfg.refine_levels;
  const int64_t Ng = S.M.Ng;
  store.assign(kmax > 1 ? kmax - 1 : 0, std::array<RVec, 3>{});
  Ab.assign(kmax + 1, std::array<const double*, 3>{});
  for (int c = 0; c < 3; ++c) {
    Ab[0][c] = An[c];
    Ab[kmax][c] = Anp1[c];
  }
  for (int j = 1; j < kmax; ++j) {
    const double s = (double)j / kmax;
    for (int c = 0; c < 3; ++c) {
      RVec& a = store[j - 1][c];
      a.resize(Ng);
      for (int64_t g = 0; g < Ng; ++g) a[g] = (1.0 - s) * An[c][g] + s * Anp1[c][g];
      Ab[j][c] = a.data();
    }
  }
}

// Orbit current deposit J_g = (1/dV) sum_i q_i vout_i Sbar_ig with Sbar from the
// orbit of v_in (reading: the evaluated orbit), summed over particles in index
// order so the result does not depend on the thread count.  A refined particle (sub
// non-empty) deposits the mean of its sub-step orbit currents.
void deposit(const Sim& S, const RVec vin[3], const RVec vout[3], RVec J[3],
             const std::vector<std::vector<SubStep>>* sub = nullptr) {
  const Mesh& M = S.M;
  const int ngl = (int)S.glx.size();
  for (int c = 0; c < 3; ++c) J[c].assign(M.Ng, 0.0);
  std::vector<std::pair<int64_t, double>> sb;
  for (int64_t i = 0; i < S.np; ++i) {
    if (sub && !(*sub)[i].empty()) {
      const std::vector<SubStep>& ss = (*sub)[i];
      const int K = (int)ss.size();
      for (const SubStep& st : ss) {
        double dx[3] = {0.0, 0.0, 0.0};
        for (int l = 0; l < M.d; ++l) dx[l] = (S.ph.dt / K) * st.vin[l];
        sb.clear();
        orbit_quadrature(M, nullptr, ngl, S.glx.data(), S.glw.data(), st.x, dx, nullptr, &sb);
        for (auto& e : sb)
          for (int c = 0; c < 3; ++c) J[c][e.first] += S.q[i] * st.vout[c] / K * e.second / M.dV;
      }
      continue;
    }
    double xi[3] = {S.x[0][i], S.x[1][i], S.x[2][i]};
    double dx[3] = {0.0, 0.0, 0.0};
    for (int l = 0; l < M.d; ++l) dx[l] = S.ph.dt * vin[l][i];
    sb.clear();
    orbit_quadrature(M, nullptr, ngl, S.glx.data(), S.glw.data(), xi, dx, nullptr, &sb);
    for (auto& e : sb)
      for (int c = 0; c < 3; ++c) J[c][e.first] += S.q[i] * vout[c][i] * e.second / M.dV;
  }
}

// Field step for a trial current j (Algorithm 1, "project the trial current,
// advance charge by continuity, and solve the CN potential equations").
struct Trial {
  CVec phi, psi, rho, A[3], U[3];
  RVec gphi[3], Anp1[3], Uh[3];
};

void field_solve(const Sim& S, const RVec j[3], Trial& T) {
  const Mesh& M = S.M;
  const double h = S.cfg.dt, kap2 = S.cfg.kappa * S.cfg.kappa;
  CVec jh[3];
  for (int c = 0; c < 3; ++c) {
    jh[c] = to_spec(M, j[c].data());
    if (S.cfg.project) project(M, jh[c]);
  }
  T.rho.assign(M.Ng, 0.0);
  T.phi.assign(M.Ng, 0.0);
  T.psi.assign(M.Ng, 0.0);
  for (int c = 0; c < 3; ++c) {
    T.A[c].assign(M.Ng, 0.0);
    T.U[c].assign(M.Ng, 0.0);
  }
  CVec phih(M.Ng), Uhh[3];
  for (int c = 0; c < 3; ++c) Uhh[c].assign(M.Ng, 0.0);
  for (int64_t g = 0; g < M.Ng; ++g) {
    double k[3];
    kvec(M, g, k);
    // continuity: rho^{n+1} = rho^n - dt div_h J^{n+1/2}
    cplx divj = 0.0;
    for (int l = 0; l < M.d; ++l) divj += cplx(0.0, k[l]) * jh[l][g];
    T.rho[g] = S.rho[g] - h * divj;
    cplx rho_half = 0.5 * (S.rho[g] + T.rho[g]);
    // CN for (phi, psi) and (A, U): eliminate the midpoint unknowns mode by mode.
    double a = kap2 * (k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
    double den = 1.0 + h * h * a / 4.0;
    T.phi[g] = ((1.0 - h * h * a / 4.0) * S.phi[g] + h * S.psi[g] +
                0.5 * h * h * kap2 * S.cfg.sigma1 * rho_half) / den;
    T.psi[g] = 2.0 * (T.phi[g] - S.phi[g]) / h - S.psi[g];
    phih[g] = 0.5 * (S.phi[g] + T.phi[g]);
    for (int c = 0; c < 3; ++c) {
      T.A[c][g] = ((1.0 - h * h * a / 4.0) * S.A[c][g] + h * S.U[c][g] +
                   0.5 * h * h * kap2 * S.cfg.sigma2 * jh[c][g]) / den;
      T.U[c][g] = 2.0 * (T.A[c][g] - S.A[c][g]) / h - S.U[c][g];
      Uhh[c][g] = 0.5 * (S.U[c][g] + T.U[c][g]);
    }
  }
  for (int l = 0; l < 3; ++l) {
    if (l < M.d)
      T.gphi[l] = to_real(M, dspec(M, phih, l));
    else
      T.gphi[l].assign(M.Ng, 0.0);
    T.Anp1[l] = to_real(M, T.A[l]);
    T.Uh[l] = to_real(M, Uhh[l]);
  }
}

// Mixed outer tests over the mesh current (nonlinear-tests equation): RMS over
// 3 Ng components and max over nodes of the Euclidean node norm.
void outer_tests(const Sim& S, const RVec H[3], const RVec j[3], double& rms_ratio,
                 double& max_ratio) {
  const int64_t Ng = S.M.Ng;
  double sr = 0, sh = 0, sj = 0, mx = 0;
  for (int64_t g = 0; g < Ng; ++g) {
    double r2 = 0, h2 = 0, j2 = 0;
    for (int c = 0; c < 3; ++c) {
      double r = H[c][g] - j[c][g];
      r2 += r * r;
      h2 += H[c][g] * H[c][g];
      j2 += j[c][g] * j[c][g];
    }
    sr += r2;
    sh += h2;
    sj += j2;
    double ratio = std::sqrt(r2) / (S.cfg.tol_outer_abs +
                                    0.5 * S.cfg.tol_outer_rel * (std::sqrt(h2) + std::sqrt(j2)));
    mx = std::max(mx, ratio);
  }
  double n3 = 3.0 * (double)Ng;
  double rr = std::sqrt(sr / n3), rh = std::sqrt(sh / n3), rj = std::sqrt(sj / n3);
  rms_ratio = rr / (S.cfg.tol_outer_abs + 0.5 * S.cfg.tol_outer_rel * (rh + rj));
  max_ratio = mx;
}

double wrap1(double v, double lo, double L) {
  // Reading: the accepted position is wrapped once per step into [lo, lo+L): the
  // periodic image v - k L with k = floor((v - lo) / L), the rounding of the quotient
  // corrected at the two ends of the interval.
  const double k = std::floor((v - lo) / L);
  double r = v - k * L;
  if (r >= lo + L) r -= L;
  if (r < lo) r += L;
  return r;
}

void real_fields(const Sim& S, RVec E[3], RVec B[3]) {
  const Mesh& M = S.M;
  for (int l = 0; l < 3; ++l) {
    RVec u = to_real(M, S.U[l]);
    RVec gp = (l < M.d) ? to_real(M, dspec(M, S.phi, l)) : RVec(M.Ng, 0.0);
    E[l].resize(M.Ng);
    for (int64_t g = 0; g < M.Ng; ++g) E[l][g] = -gp[g] - u[g];
  }
  // B = curl A
  CVec dA[3][3];  // dA[l][j] = d_j A_l
  for (int l = 0; l < 3; ++l)
    for (int j = 0; j < 3; ++j) dA[l][j] = dspec(M, S.A[l], j);
  CVec Bs[3];
  Bs[0].resize(M.Ng);
  Bs[1].resize(M.Ng);
  Bs[2].resize(M.Ng);
  for (int64_t g = 0; g < M.Ng; ++g) {
    Bs[0][g] = dA[2][1][g] - dA[1][2][g];
    Bs[1][g] = dA[0][2][g] - dA[2][0][g];
    Bs[2][g] = dA[1][0][g] - dA[0][1][g];
  }
  for (int l = 0; l < 3; ++l) B[l] = to_real(M, Bs[l]);
}

double field_energy(const Sim& S) {
  RVec E[3], B[3];
  real_fields(S, E, B);
  double W = 0.0;
  for (int64_t g = 0; g < S.M.Ng; ++g) {
    double e2 = E[0][g] * E[0][g] + E[1][g] * E[1][g] + E[2][g] * E[2][g];
    double b2 = B[0][g] * B[0][g] + B[1][g] * B[1][g] + B[2][g] * B[2][g];
    W += (e2 / (2.0 * S.cfg.sigma1) + b2 / (2.0 * S.cfg.sigma2)) * S.M.dV;
  }
  return W;
}

// Kinetic energy from the committed state: p = P - q A_h(x);
// m kappa^2 (gamma - 1) written as |p|^2 / (m (gamma + 1)).
double kinetic_energy(const Sim& S, double* vperp_rms) {
  RVec Ar[3];
  for (int l = 0; l < 3; ++l) Ar[l] = to_real(S.M, S.A[l]);
  const double* Ap[3] = {Ar[0].data(), Ar[1].data(), Ar[2].data()};
  double K = 0.0, vp = 0.0, wq = 0.0;
  for (int64_t i = 0; i < S.np; ++i) {
    double xi[3] = {S.x[0][i], S.x[1][i], S.x[2][i]};
    double Ai[3];
    interp3(S.M, Ap, xi, Ai);
    double p[3] = {S.P[0][i] - S.q[i] * Ai[0], S.P[1][i] - S.q[i] * Ai[1],
                   S.P[2][i] - S.q[i] * Ai[2]};
    double g = gamma_of(p, S.m[i], S.cfg.kappa);
    double p2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    K += p2 / (S.m[i] * (g + 1.0));
    double vy = p[1] / (S.m[i] * g), vz = p[2] / (S.m[i] * g);
    vp += std::fabs(S.q[i]) * (vy * vy + vz * vz);
    wq += std::fabs(S.q[i]);
  }
  if (vperp_rms) *vperp_rms = (wq > 0) ? std::sqrt(vp / wq) : 0.0;
  return K;
}

void constraint_rms(const Sim& S, double& gauss, double& lorenz) {
  const Mesh& M = S.M;
  const double kap2 = S.cfg.kappa * S.cfg.kappa;
  // R_G = div_h E - sigma1 rho, E = -grad phi - U ; R_L = psi/kappa^2 + div_h A
  CVec divE(M.Ng, 0.0), divA(M.Ng, 0.0);
  for (int l = 0; l < M.d; ++l) {
    CVec gp = dspec(M, S.phi, l);
    CVec Ex(M.Ng);
    for (int64_t g = 0; g < M.Ng; ++g) Ex[g] = -gp[g] - S.U[l][g];
    CVec dE = dspec(M, Ex, l), dAl = dspec(M, S.A[l], l);
    for (int64_t g = 0; g < M.Ng; ++g) {
      divE[g] += dE[g];
      divA[g] += dAl[g];
    }
  }
  CVec RG(M.Ng), RL(M.Ng);
  for (int64_t g = 0; g < M.Ng; ++g) {
    RG[g] = divE[g] - S.cfg.sigma1 * S.rho[g];
    RL[g] = S.psi[g] / kap2 + divA[g];
  }
  RVec rg = to_real(M, RG), rl = to_real(M, RL);
  double sg = 0, sl = 0;
  for (int64_t g = 0; g < M.Ng; ++g) {
    sg += rg[g] * rg[g];
    sl += rl[g] * rl[g];
  }
  gauss = std::sqrt(sg / M.Ng);
  lorenz = std::sqrt(sl / M.Ng);
}

void set_threads(const Sim& S) {
#ifdef _OPENMP
  if (S.cfg.threads > 0) omp_set_num_threads(S.cfg.threads);
#else
  (void)S;
#endif
}

}  // namespace

// ===========================================================================
// C interface (ctypes).
extern "C" {

int orc_gl_rule(int n, double* x, double* w) {
  if (n < 1 || n > 64) return ORC_EINVAL;
  gauss_legendre01(n, x, w);
  return ORC_OK;
}

void orc_shape(double xi, double* S, double* dS) {
  *S = S2(xi);
  *dS = dS2(xi);
}

void orc_shape_r(int r, double xi, double* S, double* dS) {
  *S = r == 1 ? S1(xi) : S2(xi);
  *dS = r == 1 ? dS1(xi) : dS2(xi);
}

double orc_hc_map(const double* um, const double* tau, double* up) { return hc_map_u(um, tau, up); }

void orc_vdg(const double* pa, const double* pb, double m, double kappa, double* out) {
  vdg(pa, pb, m, kappa, out);
}

// In-place complex FFT over a mesh (re, im arrays of length Ng).
int orc_fft(const orc_config* cfg, double* re, double* im, int inverse) {
  Mesh M;
  int st = setup_mesh(cfg, M, true);
  if (st) return st;
  CVec a(M.Ng);
  for (int64_t g = 0; g < M.Ng; ++g) a[g] = cplx(re[g], im[g]);
  fftn(M, a.data(), inverse != 0);
  for (int64_t g = 0; g < M.Ng; ++g) {
    re[g] = a[g].real();
    im[g] = a[g].imag();
  }
  return ORC_OK;
}

// Knot split of one orbit: writes the sorted breakpoints (including 0 and 1).
int orc_knot_split(const orc_config* cfg, const double* x, const double* dx, double* s, int cap) {
  Mesh M;
  int st = setup_mesh(cfg, M);
  if (st) return st;
  std::vector<double> b;
  double xx[3] = {x[0], M.d > 1 ? x[1] : 0.0, M.d > 2 ? x[2] : 0.0};
  double dd[3] = {dx[0], M.d > 1 ? dx[1] : 0.0, M.d > 2 ? dx[2] : 0.0};
  knot_split(M, xx, dd, b);
  if ((int)b.size() > cap) return ORC_EINVAL;
  for (size_t k = 0; k < b.size(); ++k) s[k] = b[k];
  return (int)b.size();
}

// Orbit-averaged shape S-bar of one orbit as (node, weight) pairs, merged per node.
int orc_orbit_weights(const orc_config* cfg, const double* x, const double* dx, int64_t* nodes,
                      double* w, int cap) {
  Mesh M;
  int st = setup_mesh(cfg, M);
  if (st) return st;
  std::vector<double> glx(cfg->gl_order), glw(cfg->gl_order);
  gauss_legendre01(cfg->gl_order, glx.data(), glw.data());
  double xx[3] = {x[0], M.d > 1 ? x[1] : 0.0, M.d > 2 ? x[2] : 0.0};
  double dd[3] = {dx[0], M.d > 1 ? dx[1] : 0.0, M.d > 2 ? dx[2] : 0.0};
  std::vector<std::pair<int64_t, double>> sb;
  orbit_quadrature(M, nullptr, cfg->gl_order, glx.data(), glw.data(), xx, dd, nullptr, &sb);
  std::sort(sb.begin(), sb.end(),
            [](const std::pair<int64_t, double>& a, const std::pair<int64_t, double>& b) {
              return a.first < b.first;
            });
  int cnt = 0;
  for (size_t k = 0; k < sb.size(); ++k) {
    if (cnt > 0 && nodes[cnt - 1] == sb[k].first) {
      w[cnt - 1] += sb[k].second;
      continue;
    }
    if (cnt >= cap) return ORC_EINVAL;
    nodes[cnt] = sb[k].first;
    w[cnt] = sb[k].second;
    ++cnt;
  }
  return cnt;
}

// Point interpolant of a 3-component mesh array.
int orc_interp(const orc_config* cfg, const double* F, const double* x, double* out) {
  Mesh M;
  int st = setup_mesh(cfg, M);
  if (st) return st;
  const double* Fp[3] = {F, F + M.Ng, F + 2 * M.Ng};
  double xx[3] = {x[0], M.d > 1 ? x[1] : 0.0, M.d > 2 ? x[2] : 0.0};
  interp3(M, Fp, xx, out);
  return ORC_OK;
}

// Single orbit evaluation with explicit fields:
//   gphi [d][Ng], An/Anp1/Uh [3][Ng]; x [d]; P, vin [3].
int orc_orbit_eval(const orc_config* cfg, const double* gphi, const double* An, const double* Anp1,
                   const double* Uh, const double* x, const double* P, double q, double m,
                   const double* vin, orc_eval_out* out) {
  Mesh M;
  int st = setup_mesh(cfg, M);
  if (st) return st;
  std::vector<double> glx(cfg->gl_order), glw(cfg->gl_order);
  gauss_legendre01(cfg->gl_order, glx.data(), glw.data());
  FieldPtrs F;
  for (int l = 0; l < 3; ++l) {
    F.gphi[l] = (l < M.d) ? gphi + l * M.Ng : nullptr;
    F.An[l] = An + l * M.Ng;
    F.Anp1[l] = Anp1 + l * M.Ng;
    F.Uh[l] = Uh + l * M.Ng;
  }
  Phys ph{cfg->kappa, cfg->dt};
  double xx[3] = {x[0], M.d > 1 ? x[1] : 0.0, M.d > 2 ? x[2] : 0.0};
  orbit_eval(M, ph, F, cfg->gl_order, glx.data(), glw.data(), xx, P, q, m, vin, out);
  return ORC_OK;
}

void* orc_create(const orc_config* cfg, int* status) {
  Mesh M;
  int st = setup_mesh(cfg, M, true);
  if (!st && (cfg->gl_order < 1 || cfg->gl_order > 64)) st = ORC_EINVAL;
  if (!st && !(cfg->dt > 0.0 && cfg->kappa > 0.0)) st = ORC_EINVAL;
  // The energy theorem needs sigma1 = kappa^2 sigma2 (Maxwell-compatible scaling).
  if (!st && std::fabs(cfg->sigma1 - cfg->kappa * cfg->kappa * cfg->sigma2) >
                 1e-14 * std::fabs(cfg->sigma1))
    st = ORC_EINVAL;
  if (!st && (cfg->max_outer < 1 || cfg->max_inner < 1)) st = ORC_EINVAL;
  if (!st && (cfg->refine_levels < 0 || cfg->refine_levels > kMaxRefine)) st = ORC_EINVAL;
  if (status) *status = st;
  if (st) return nullptr;
  Sim* S = new Sim();
  S->cfg = *cfg;
  S->M = M;
  S->ph = Phys{cfg->kappa, cfg->dt};
  S->glx.resize(cfg->gl_order);
  S->glw.resize(cfg->gl_order);
  gauss_legendre01(cfg->gl_order, S->glx.data(), S->glw.data());
  S->phi.assign(M.Ng, 0.0);
  S->psi.assign(M.Ng, 0.0);
  S->rho.assign(M.Ng, 0.0);
  for (int c = 0; c < 3; ++c) {
    S->A[c].assign(M.Ng, 0.0);
    S->U[c].assign(M.Ng, 0.0);
    S->Jacc[c].assign(M.Ng, 0.0);
  }
  return S;
}

void orc_destroy(void* h) { delete static_cast<Sim*>(h); }

// Particles: x [d][n], u = p/(m kappa) [3][n], q [n]; m = |q|.
int orc_load_particles(void* h, int64_t n, const double* x, const double* u, const double* q) {
  Sim& S = *static_cast<Sim*>(h);
  if (n < 0) return ORC_EINVAL;
  S.np = n;
  for (int c = 0; c < 3; ++c) {
    S.x[c].assign(n, 0.0);
    S.P[c].assign(n, 0.0);
    S.vbar[c].assign(n, 0.0);
  }
  S.q.assign(q, q + n);
  S.m.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    S.m[i] = std::fabs(q[i]);
    if (!(S.m[i] > 0.0)) return ORC_EINVAL;
    for (int l = 0; l < S.M.d; ++l) S.x[l][i] = x[l * n + i];
    for (int c = 0; c < 3; ++c) S.P[c][i] = S.m[i] * S.cfg.kappa * u[c * n + i];  // p for now
  }
  S.initialized = false;
  return ORC_OK;
}

int orc_load_potentials(void* h, const double* A0, const double* U0) {
  Sim& S = *static_cast<Sim*>(h);
  for (int c = 0; c < 3; ++c) {
    S.A[c] = to_spec(S.M, A0 + c * S.M.Ng);
    S.U[c] = to_spec(S.M, U0 + c * S.M.Ng);
  }
  return ORC_OK;
}

// Initialization (Nyquist paragraph and the constraint discussion): rho^0 and J^0
// from a point-shape deposit, projected; phi^0 from Gauss's law
// -Lap phi = sigma1 rho + div U; psi^0 = -kappa^2 div A (Lorenz gauge);
// canonical momenta P = p + q A_h^0(x) from the projected A^0.
// Reading: the immobile background is uniform and cancels the k=0 charge exactly.
int orc_initialize(void* h) {
  Sim& S = *static_cast<Sim*>(h);
  const Mesh& M = S.M;
  const double kap = S.cfg.kappa, kap2 = kap * kap;
  RVec rho_r(M.Ng, 0.0), J_r[3];
  for (int c = 0; c < 3; ++c) J_r[c].assign(M.Ng, 0.0);
  for (int64_t i = 0; i < S.np; ++i) {
    double xi[3] = {S.x[0][i], S.x[1][i], S.x[2][i]};
    double p[3] = {S.P[0][i], S.P[1][i], S.P[2][i]};
    double g = gamma_of(p, S.m[i], kap);
    double v[3] = {p[0] / (S.m[i] * g), p[1] / (S.m[i] * g), p[2] / (S.m[i] * g)};
    PointWeights pw;
    point_weights(M, xi, pw);
    for (int c2 = 0; c2 < pw.cnt[2]; ++c2)
      for (int c1 = 0; c1 < pw.cnt[1]; ++c1)
        for (int c0 = 0; c0 < pw.cnt[0]; ++c0) {
          double Sg = pw.S[0][c0] * pw.S[1][c1] * pw.S[2][c2];
          int64_t gi = M.node(pw.base[0] + c0, pw.base[1] + c1, pw.base[2] + c2);
          rho_r[gi] += S.q[i] * Sg / M.dV;
          for (int c = 0; c < 3; ++c) J_r[c][gi] += S.q[i] * v[c] * Sg / M.dV;
        }
    for (int c = 0; c < 3; ++c) S.vbar[c][i] = v[c];
  }
  S.rho = to_spec(M, rho_r.data());
  S.rho[0] = 0.0;  // neutralizing background
  if (S.cfg.project) {
    project(M, S.rho);
    for (int c = 0; c < 3; ++c) {
      project(M, S.A[c]);
      project(M, S.U[c]);
    }
  }
  for (int c = 0; c < 3; ++c) {
    CVec jh = to_spec(M, J_r[c].data());
    if (S.cfg.project) project(M, jh);
    S.Jacc[c] = to_real(M, jh);
  }
  // phi^0 from Gauss's law, psi^0 from the Lorenz gauge.
  CVec divU(M.Ng, 0.0), divA(M.Ng, 0.0);
  for (int l = 0; l < M.d; ++l) {
    CVec a = dspec(M, S.U[l], l), b = dspec(M, S.A[l], l);
    for (int64_t g = 0; g < M.Ng; ++g) {
      divU[g] += a[g];
      divA[g] += b[g];
    }
  }
  for (int64_t g = 0; g < M.Ng; ++g) {
    double k[3];
    kvec(M, g, k);
    double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    S.phi[g] = (k2 > 0.0) ? (S.cfg.sigma1 * S.rho[g] + divU[g]) / k2 : cplx(0.0, 0.0);
    S.psi[g] = -kap2 * divA[g];
  }
  // canonical momenta
  RVec Ar[3];
  for (int c = 0; c < 3; ++c) Ar[c] = to_real(M, S.A[c]);
  const double* Ap[3] = {Ar[0].data(), Ar[1].data(), Ar[2].data()};
  for (int64_t i = 0; i < S.np; ++i) {
    double xi[3] = {S.x[0][i], S.x[1][i], S.x[2][i]};
    double Ai[3];
    interp3(M, Ap, xi, Ai);
    for (int c = 0; c < 3; ++c) S.P[c][i] += S.q[i] * Ai[c];
  }
  S.t = 0.0;
  S.step = 0;
  S.initialized = true;
  double vp;
  S.E0 = kinetic_energy(S, &vp) + field_energy(S);
  S.last_chain_rms = S.last_work = S.last_rms_ratio = S.last_max_ratio = 0.0;
  return ORC_OK;
}

// Overwrite the canonical particle state (x [d][n], P [3][n], vbar [3][n]).
int orc_set_particle_state(void* h, const double* x, const double* P, const double* vbar) {
  Sim& S = *static_cast<Sim*>(h);
  for (int64_t i = 0; i < S.np; ++i) {
    for (int l = 0; l < S.M.d; ++l) S.x[l][i] = x[l * S.np + i];
    for (int c = 0; c < 3; ++c) {
      S.P[c][i] = P[c * S.np + i];
      S.vbar[c][i] = vbar[c * S.np + i];
    }
  }
  return ORC_OK;
}

int orc_read_particles(void* h, double* x, double* P, double* vbar) {
  Sim& S = *static_cast<Sim*>(h);
  for (int64_t i = 0; i < S.np; ++i) {
    if (x)
      for (int l = 0; l < S.M.d; ++l) x[l * S.np + i] = S.x[l][i];
    for (int c = 0; c < 3; ++c) {
      if (P) P[c * S.np + i] = S.P[c][i];
      if (vbar) vbar[c * S.np + i] = S.vbar[c][i];
    }
  }
  return ORC_OK;
}

// Field read-out in real space: 0 phi, 1 psi, 2 A[3], 3 U[3], 4 rho, 5 J(accepted)[3],
// 6 E[3], 7 B[3].
int orc_read_field(void* h, int which, double* dst) {
  Sim& S = *static_cast<Sim*>(h);
  const Mesh& M = S.M;
  auto put = [&](const RVec& r, int c) { std::memcpy(dst + c * M.Ng, r.data(), sizeof(double) * M.Ng); };
  switch (which) {
    case 0: put(to_real(M, S.phi), 0); break;
    case 1: put(to_real(M, S.psi), 0); break;
    case 2: for (int c = 0; c < 3; ++c) put(to_real(M, S.A[c]), c); break;
    case 3: for (int c = 0; c < 3; ++c) put(to_real(M, S.U[c]), c); break;
    case 4: put(to_real(M, S.rho), 0); break;
    case 5: for (int c = 0; c < 3; ++c) put(S.Jacc[c], c); break;
    case 6:
    case 7: {
      RVec E[3], B[3];
      real_fields(S, E, B);
      for (int c = 0; c < 3; ++c) put(which == 6 ? E[c] : B[c], c);
      break;
    }
    default: return ORC_EINVAL;
  }
  return ORC_OK;
}

// Advance only the fields by one CN step with a prescribed current j [3][Ng]
// (used by the field-solve tests; particles are untouched).
int orc_cn_advance(void* h, const double* j) {
  Sim& S = *static_cast<Sim*>(h);
  RVec jj[3];
  for (int c = 0; c < 3; ++c) jj[c].assign(j + c * S.M.Ng, j + (c + 1) * S.M.Ng);
  Trial T;
  field_solve(S, jj, T);
  S.phi = T.phi;
  S.psi = T.psi;
  S.rho = T.rho;
  for (int c = 0; c < 3; ++c) {
    S.A[c] = T.A[c];
    S.U[c] = T.U[c];
    S.Jacc[c] = jj[c];
  }
  S.t += S.cfg.dt;
  S.step += 1;
  return ORC_OK;
}

// Set spectral field state directly from real arrays (phi, psi [Ng], A, U [3][Ng], rho [Ng]).
int orc_set_fields(void* h, const double* phi, const double* psi, const double* A, const double* U,
                   const double* rho) {
  Sim& S = *static_cast<Sim*>(h);
  S.phi = to_spec(S.M, phi);
  S.psi = to_spec(S.M, psi);
  S.rho = to_spec(S.M, rho);
  for (int c = 0; c < 3; ++c) {
    S.A[c] = to_spec(S.M, A + c * S.M.Ng);
    S.U[c] = to_spec(S.M, U + c * S.M.Ng);
  }
  return ORC_OK;
}

// One evaluation of the outer map at the trial current j (Algorithm 1, one residual
// evaluation): field step, inner Picard solve of every particle warm-started from vw
// (with refinement of the particles whose full-step solve fails, when enabled), orbit
// current deposit and projection H(j), and the mixed outer tests.  On return vw holds
// each particle's last v_out (the sub-step mean for a refined one).  Returns ORC_EINNER
// if any particle solve failed.
struct OuterEval {
  Trial T;
  RVec H[3];
  RVec vin_f[3], Pn1[3], xend[3], Ra2, work;
  std::vector<std::vector<SubStep>> sub;  // sub-steps of refined particles (else empty)
  double rr = 0.0, mr = 0.0;
};

int evaluate_outer(Sim& S, const RVec An[3], const RVec j[3], RVec vw[3], OuterEval& E, orc_report& R) {
  const Mesh& M = S.M;
  const int64_t np = S.np;
  field_solve(S, j, E.T);
  FieldPtrs F = make_ptrs(S, E.T.gphi, An, E.T.Anp1, E.T.Uh);
  std::vector<std::array<RVec, 3>> Astore;
  std::vector<std::array<const double*, 3>> Ab;
  step_potentials(S, F.An, F.Anp1, Astore, Ab);
  for (int c = 0; c < 3; ++c) {
    E.vin_f[c].assign(np, 0.0);
    E.Pn1[c].assign(np, 0.0);
    E.xend[c].assign(np, 0.0);
  }
  E.Ra2.assign(np, 0.0);
  E.work.assign(np, 0.0);
  E.sub.assign(np, std::vector<SubStep>());
  std::vector<int32_t> iters(np), fail(np);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < np; ++i) {
    double v0[3] = {vw[0][i], vw[1][i], vw[2][i]};
    ParticleSolve ps;
    solve_particle(S, Ab, F, i, v0, S.level[i], true, ps);
    iters[i] = ps.evals;
    fail[i] = ps.ok ? 0 : 1;
    if (ps.ok) S.level[i] = ps.level;
    for (int c = 0; c < 3; ++c) {
      E.vin_f[c][i] = ps.vin[c];
      vw[c][i] = ps.vout[c];
      E.Pn1[c][i] = ps.Pn1[c];
      E.xend[c][i] = ps.xend[c];
    }
    E.Ra2[i] = ps.Ra2;
    E.work[i] = ps.work;
    E.sub[i] = std::move(ps.sub);
  }
  int64_t nfail = 0, evals = 0;
  int imax = 0, refined = 0;
  double isum = 0.0;
  for (int64_t i = 0; i < np; ++i) {
    nfail += fail[i];
    evals += iters[i];
    imax = std::max(imax, iters[i]);
    isum += iters[i];
    refined += E.sub[i].empty() ? 0 : 1;
  }
  R.outer_iters += 1;
  R.evaluations += evals;
  R.inner_max = imax;
  R.inner_mean = np ? isum / np : 0.0;
  R.refined = refined;
  if (nfail) return ORC_EINNER;
  RVec Jorb[3];
  deposit(S, E.vin_f, vw, Jorb, &E.sub);
  for (int c = 0; c < 3; ++c) {
    CVec jh = to_spec(M, Jorb[c].data());
    if (S.cfg.project) project(M, jh);
    E.H[c] = to_real(M, jh);
  }
  outer_tests(S, E.H, j, E.rr, E.mr);
  R.res_rms_ratio = E.rr;
  R.res_max_ratio = E.mr;
  return ORC_OK;
}

// Commit the state of the converged evaluation E at current j (Algorithm 1, commit).
void commit_step(Sim& S, const RVec j[3], const RVec vw[3], const OuterEval& E) {
  const Mesh& M = S.M;
  const int64_t np = S.np;
  const double dt = S.cfg.dt;
  double sRa = 0.0, swk = 0.0;
  for (int64_t i = 0; i < np; ++i) {
    sRa += E.Ra2[i];
    swk += E.work[i];
  }
  double mesh_work = 0.0;
  for (int c = 0; c < 3; ++c)
    for (int64_t g = 0; g < M.Ng; ++g) {
      double gp = (c < M.d) ? E.T.gphi[c][g] : 0.0;
      mesh_work += E.H[c][g] * (-gp - E.T.Uh[c][g]) * M.dV;
    }
  S.last_chain_rms = np ? std::sqrt(sRa / (3.0 * np)) : 0.0;
  S.last_work = dt * (swk - mesh_work);
  S.last_rms_ratio = E.rr;
  S.last_max_ratio = E.mr;
  S.phi = E.T.phi;
  S.psi = E.T.psi;
  S.rho = E.T.rho;
  for (int c = 0; c < 3; ++c) {
    S.A[c] = E.T.A[c];
    S.U[c] = E.T.U[c];
    S.Jacc[c] = j[c];
    S.vbar[c] = vw[c];
    S.P[c] = E.Pn1[c];
  }
  for (int l = 0; l < M.d; ++l)
    for (int64_t i = 0; i < np; ++i) S.x[l][i] = wrap1(E.xend[l][i], M.lo[l], M.len[l]);
  S.t += dt;
  S.step += 1;
}

// Solve the regularized normal equations of the Anderson step, G x = b with G symmetric
// positive definite (n <= 8, row-major), by the Cholesky factorization G = L L^T and two
// triangular solves; false when G is not numerically positive definite or the result is
// not finite (an unusable history).
bool spd_solve(const std::vector<double>& G, const std::vector<double>& b, int n, std::vector<double>& x) {
  std::vector<double> L(n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = G[j * n + j];
    for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    L[j * n + j] = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double v = G[i * n + j];
      for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = v / L[j * n + j];
    }
  }
  std::vector<double> y(n, 0.0);
  for (int i = 0; i < n; ++i) {  // L y = b
    double v = b[i];
    for (int k = 0; k < i; ++k) v -= L[i * n + k] * y[k];
    y[i] = v / L[i * n + i];
  }
  x.assign(n, 0.0);
  for (int i = n - 1; i >= 0; --i) {  // L^T x = y
    double v = y[i];
    for (int k = i + 1; k < n; ++k) v -= L[k * n + i] * x[k];
    x[i] = v / L[i * n + i];
    if (!std::isfinite(x[i])) return false;
  }
  return true;
}

double dot3(const RVec a[3], const RVec b[3]) {
  double s = 0.0;
  for (int c = 0; c < 3; ++c)
    for (size_t g = 0; g < a[c].size(); ++g) s += a[c][g] * b[c][g];
  return s;
}

// Advance one implicit step (Algorithm 1).  The outer unknown is the mesh current j,
// started from the accepted current.  Outer scheme 0: damped Picard j <- j + beta r.
// Outer scheme 1 (the paper's solver, section on the implicit solver): limited-memory
// type-II Anderson with regularization, history reset and backtracking, with a damped
// Picard direction when the history is unusable or its direction is rejected.  Every
// evaluation of the outer map counts against max_outer.
int orc_step(void* h, orc_report* rep) {
  Sim& S = *static_cast<Sim*>(h);
  if (!S.initialized) return ORC_ESTATE;
  set_threads(S);
  const Mesh& M = S.M;
  const int64_t Ng = M.Ng;
  RVec An[3];
  for (int c = 0; c < 3; ++c) An[c] = to_real(M, S.A[c]);
  RVec j[3], vw[3];
  for (int c = 0; c < 3; ++c) {
    j[c] = S.Jacc[c];
    vw[c] = S.vbar[c];  // inner warm start, carried from evaluation to evaluation
  }
  S.level.assign(S.np, 0);  // every step starts with full-step particle solves
  orc_report R{};
  auto finish = [&](int st) {
    if (rep) *rep = R;
    return st;
  };
  OuterEval E;
  int st = evaluate_outer(S, An, j, vw, E, R);
  if (st) return finish(st);
  if (E.rr <= 1.0 && E.mr <= 1.0) {
    commit_step(S, j, vw, E);
    return finish(ORC_OK);
  }
  const bool anderson = S.cfg.outer_scheme == 1;
  const int mem = std::max(1, std::min(S.cfg.anderson_m, 8));
  std::vector<std::array<RVec, 3>> dJ, dR;  // history columns, oldest first
  RVec r[3];
  for (int c = 0; c < 3; ++c) {
    r[c].resize(Ng);
    for (int64_t g = 0; g < Ng; ++g) r[c][g] = E.H[c][g] - j[c][g];
  }
  while (R.outer_iters < S.cfg.max_outer) {
    const int k = R.outer_iters;  // outer iterations done so far
    bool accepted = false;
    for (int pass = 0; pass < 2 && !accepted; ++pass) {
      // pass 0: Anderson direction (when eligible and the history is usable); pass 1: damped Picard
      const bool use_a = anderson && pass == 0 && k >= S.cfg.anderson_start && !dJ.empty();
      if (pass == 0 && !use_a) continue;
      RVec d[3];
      for (int c = 0; c < 3; ++c) {
        d[c].resize(Ng);
        for (int64_t g = 0; g < Ng; ++g) d[c][g] = S.cfg.beta * r[c][g];
      }
      if (use_a) {
        const int mh = (int)dR.size();
        std::vector<double> G(mh * mh), b(mh), gam;
        double tr = 0.0;
        for (int a1 = 0; a1 < mh; ++a1) {
          b[a1] = dot3(dR[a1].data(), r);
          for (int a2 = 0; a2 < mh; ++a2) G[a1 * mh + a2] = dot3(dR[a1].data(), dR[a2].data());
          tr += G[a1 * mh + a1];
        }
        for (int a1 = 0; a1 < mh; ++a1) G[a1 * mh + a1] += S.cfg.anderson_lambda * tr / mh;
        if (!spd_solve(G, b, mh, gam)) {
          dJ.clear();
          dR.clear();
          continue;  // unusable history: damped Picard
        }
        for (int a1 = 0; a1 < mh; ++a1)
          for (int c = 0; c < 3; ++c)
            for (int64_t g = 0; g < Ng; ++g)
              d[c][g] -= gam[a1] * (dJ[a1][c][g] + S.cfg.beta * dR[a1][c][g]);
      }
      // backtracking along d: alpha = 1, 1/2, ..., 2^-ls_halvings
      double alpha = 1.0;
      for (int hh = 0; hh <= S.cfg.ls_halvings && R.outer_iters < S.cfg.max_outer; ++hh, alpha *= 0.5) {
        RVec jt[3], vt[3];
        for (int c = 0; c < 3; ++c) {
          jt[c].resize(Ng);
          for (int64_t g = 0; g < Ng; ++g) jt[c][g] = j[c][g] + alpha * d[c][g];
          vt[c] = vw[c];
        }
        OuterEval Et;
        st = evaluate_outer(S, An, jt, vt, Et, R);
        if (st) return finish(st);
        for (int c = 0; c < 3; ++c) vw[c] = vt[c];
        if (Et.rr <= 1.0 && Et.mr <= 1.0) {
          commit_step(S, jt, vw, Et);
          return finish(ORC_OK);
        }
        if (use_a && Et.rr > S.cfg.ls_growth * E.rr) {
          dJ.clear();  // the residual grew too much along the Anderson direction
          dR.clear();
        }
        if (Et.rr <= (1.0 - S.cfg.ls_decrease * alpha) * E.rr && Et.mr <= S.cfg.ls_growth * E.mr) {
          // accept: record the differences, move to the trial
          std::array<RVec, 3> cj, cr;
          for (int c = 0; c < 3; ++c) {
            cj[c].resize(Ng);
            cr[c].resize(Ng);
            for (int64_t g = 0; g < Ng; ++g) {
              const double rt = Et.H[c][g] - jt[c][g];
              cj[c][g] = jt[c][g] - j[c][g];
              cr[c][g] = rt - r[c][g];
              r[c][g] = rt;
              j[c][g] = jt[c][g];
            }
          }
          if (anderson) {
            dJ.push_back(cj);
            dR.push_back(cr);
            if ((int)dJ.size() > mem) {
              dJ.erase(dJ.begin());
              dR.erase(dR.begin());
            }
          }
          E = std::move(Et);
          accepted = true;
          ++R.outer_updates;
          break;
        }
        if (!anderson) {
          // plain damped Picard takes every step (no line search)
          std::array<RVec, 3> dummy;
          (void)dummy;
          for (int c = 0; c < 3; ++c)
            for (int64_t g = 0; g < Ng; ++g) {
              r[c][g] = Et.H[c][g] - jt[c][g];
              j[c][g] = jt[c][g];
            }
          E = std::move(Et);
          accepted = true;
          ++R.outer_updates;
          break;
        }
      }
      if (!accepted && use_a) {
        dJ.clear();  // rejected Anderson direction: retry with damped Picard
        dR.clear();
      }
    }
    if (!accepted) return finish(ORC_ENOCONV);
  }
  return finish(ORC_ENOCONV);
}

int orc_diagnostics(void* h, orc_diag* d) {
  Sim& S = *static_cast<Sim*>(h);
  if (!S.initialized) return ORC_ESTATE;
  std::memset(d, 0, sizeof(*d));
  d->t = S.t;
  d->step = S.step;
  d->kinetic = kinetic_energy(S, &d->vperp_rms);
  d->field = field_energy(S);
  d->total = d->kinetic + d->field;
  d->energy_rel = (S.E0 != 0.0) ? std::fabs(d->total - S.E0) / std::fabs(S.E0) : 0.0;
  constraint_rms(S, d->gauss_rms, d->lorenz_rms);
  d->chain_rms = S.last_chain_rms;
  d->work_residual = S.last_work;
  d->res_rms_ratio = S.last_rms_ratio;
  d->res_max_ratio = S.last_max_ratio;
  return ORC_OK;
}

// Mode amplitude |f_hat_m| / Ng of one component of a field read-out (unnormalized DFT).
int orc_mode_amplitude(void* h, int which, int comp, const int32_t* mode, double* amp) {
  Sim& S = *static_cast<Sim*>(h);
  const Mesh& M = S.M;
  int nc = (which == 2 || which == 3 || which >= 5) ? 3 : 1;
  if (comp < 0 || comp >= nc) return ORC_EINVAL;
  RVec buf((size_t)nc * M.Ng);
  int st = orc_read_field(h, which, buf.data());
  if (st) return st;
  CVec a = to_spec(M, buf.data() + (size_t)comp * M.Ng);
  int64_t i[3];
  for (int l = 0; l < 3; ++l) i[l] = ((mode[l] % M.n[l]) + M.n[l]) % M.n[l];
  int64_t g = i[0] + (int64_t)M.n[0] * (i[1] + (int64_t)M.n[1] * i[2]);
  *amp = std::abs(a[g]) / (double)M.Ng;
  return ORC_OK;
}

// One frozen-field orbit pass over all loaded particles with the fields given
// explicitly: a single evaluation v_out = F(v_in) per particle (iterate = 0), or the
// inner Picard loop to the inner tolerance (iterate = 1, v_in warm start) with
// refinement of failed particles when refine_levels > 0.  Writes v_out [3][n], P^{n+1}
// [3][n], the unprojected orbit current J [3][Ng], orbit evaluations per particle, the
// level each particle was solved at, its converged v_in [3][n] and its end position
// xend [d][n] (unwrapped); any output may be null.  level_in (may be null: all 0) sets the
// level each particle starts at (iterate = 1; at most refine_levels).  Returns the number
// of particles whose solve failed (iterate = 1), or -1 for an invalid level_in.
int64_t orc_orbit_pass(void* h, const double* gphi, const double* An, const double* Anp1,
                       const double* Uh, const double* vin, int iterate, double* vout, double* Pn1,
                       double* J, int32_t* iters, const int32_t* level_in, int32_t* level_out,
                       double* vin_out, double* xend) {
  Sim& S = *static_cast<Sim*>(h);
  set_threads(S);
  const Mesh& M = S.M;
  const int64_t np = S.np;
  FieldPtrs F;
  for (int l = 0; l < 3; ++l) {
    F.gphi[l] = (l < M.d) ? gphi + l * M.Ng : nullptr;
    F.An[l] = An + l * M.Ng;
    F.Anp1[l] = Anp1 + l * M.Ng;
    F.Uh[l] = Uh + l * M.Ng;
  }
  if (level_in)
    for (int64_t i = 0; i < np; ++i)
      if (level_in[i] < 0 || level_in[i] > (iterate ? S.cfg.refine_levels : 0)) return -1;
  std::vector<std::array<RVec, 3>> Astore;
  std::vector<std::array<const double*, 3>> Ab;
  step_potentials(S, F.An, F.Anp1, Astore, Ab);
  RVec vi[3], vo[3];
  for (int c = 0; c < 3; ++c) {
    vi[c].assign(np, 0.0);
    vo[c].assign(np, 0.0);
  }
  std::vector<std::vector<SubStep>> sub(np);
  int64_t nfail = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : nfail)
  for (int64_t i = 0; i < np; ++i) {
    double v0[3] = {vin[i], vin[np + i], vin[2 * np + i]};
    ParticleSolve ps;
    solve_particle(S, Ab, F, i, v0, level_in ? level_in[i] : 0, iterate != 0, ps);
    if (iters) iters[i] = ps.evals;
    if (level_out) level_out[i] = ps.level;
    if (!ps.ok) nfail += 1;
    for (int c = 0; c < 3; ++c) {
      vi[c][i] = ps.vin[c];
      vo[c][i] = ps.vout[c];
      if (vout) vout[c * np + i] = ps.vout[c];
      if (Pn1) Pn1[c * np + i] = ps.Pn1[c];
      if (vin_out) vin_out[c * np + i] = ps.vin[c];
    }
    if (xend)
      for (int l = 0; l < M.d; ++l) xend[l * np + i] = ps.xend[l];
    sub[i] = std::move(ps.sub);
  }
  if (J) {
    RVec Jr[3];
    deposit(S, vi, vo, Jr, &sub);
    for (int c = 0; c < 3; ++c) std::memcpy(J + c * M.Ng, Jr[c].data(), sizeof(double) * M.Ng);
  }
  return nfail;
}

// Trial fields of one field solve at the accepted state with current j [3][Ng]:
// gphi [d][Ng], Anp1 [3][Ng], Uh [3][Ng], plus A^n [3][Ng].  No state change.
int orc_trial_fields(void* h, const double* j, double* gphi, double* An, double* Anp1, double* Uh) {
  Sim& S = *static_cast<Sim*>(h);
  const Mesh& M = S.M;
  RVec jj[3];
  for (int c = 0; c < 3; ++c) jj[c].assign(j + c * M.Ng, j + (c + 1) * M.Ng);
  Trial T;
  field_solve(S, jj, T);
  for (int l = 0; l < M.d; ++l) std::memcpy(gphi + l * M.Ng, T.gphi[l].data(), sizeof(double) * M.Ng);
  for (int c = 0; c < 3; ++c) {
    RVec a = to_real(M, S.A[c]);
    std::memcpy(An + c * M.Ng, a.data(), sizeof(double) * M.Ng);
    std::memcpy(Anp1 + c * M.Ng, T.Anp1[c].data(), sizeof(double) * M.Ng);
    std::memcpy(Uh + c * M.Ng, T.Uh[c].data(), sizeof(double) * M.Ng);
  }
  return ORC_OK;
}

int64_t orc_num_particles(void* h) { return static_cast<Sim*>(h)->np; }

// OpenMP threads a parallel region of the oracle runs with (for reporting timings).
int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// The Anderson step's small solve (spd_solve) on its own, for the tests: x of G x = b;
// ORC_OK, or ORC_EINVAL when G is not numerically positive definite.
int orc_spd_solve(int n, const double* G, const double* b, double* x) {
  if (n < 1 || n > 8) return ORC_EINVAL;
  std::vector<double> g(G, G + n * n), bb(b, b + n), xx;
  if (!spd_solve(g, bb, n, xx)) return ORC_EINVAL;
  for (int i = 0; i < n; ++i) x[i] = xx[i];
  return ORC_OK;
}

}  // extern "C"
