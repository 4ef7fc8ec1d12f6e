// adjoint.hip -- reverse-mode adjoint of the implicit step and of initialization for
// runs in one, two or three dimensions with the quadratic shape in FP64.
//
// The paper defines the step (Algorithm 1) but no derivative of it.  The adjoint here
// differentiates the converged step, not its iteration history: the step's unknowns
// (every particle's orbit velocity vbar and the mesh current j) satisfy
//     vbar_i = F_i(vbar_i; x_i, P_i, q_i, Phi(j))      (inner fixed point, per particle)
//     j      = H(vbar, x, q)                          (outer fixed point on the mesh)
// with Phi(j) the trial fields of the CN field step (grad phi^{n+1/2}, A^n, A^{n+1}) and
// H the projected orbit current.  The outputs are x^{n+1} = x + dt vbar_x, P^{n+1} of
// the evaluation and the new field state.  By the implicit-function theorem, with
// cotangents (lx, lP, lf) of the outputs, the adjoint unknowns mu_v (per particle) and
// mu_j (mesh) solve
//     mu_v,i = (I - dF_i/dvbar)^-T [ dt lx_i e_x + (dP^{n+1}_i/dvbar)^T lP_i
//                                    + (dH/dvbar_i)^T mu_j ]
//     mu_j   = (dState'/dj)^T lf + (dPhi/dj)^T sum_i (dF_i/dPhi)^T mu_v,i
//                                + (dPhi/dj)^T sum_i (dP^{n+1}_i/dPhi)^T lP_i
// and the input cotangents follow by one more transposed product.  The per-particle
// 3x3 system is solved directly (F depends on vbar only through its d resolved
// components, so only d columns of dF/dvbar are nonzero); the mesh equation is iterated
// like the outer Picard iteration it transposes, with the same damping, until mu_j
// settles.
//
// Kernels: k_adj_particle (one thread per particle; the hand-written reverse sweep of the
// orbit gathers, the GM-HC push with its gamma_HC, B_eff and K chain, the secant
// velocity and the orbit deposit), k_adj_iter (one transposed outer iteration per launch
// from the values k_adj_particle cached: the transposed deposit, the per-particle solve
// and the scatter of the field cotangents, summed in a fixed order within each wave and
// as exact fixed-point sums across waves), k_adj_field (one thread per Fourier mode; the
// conjugate transpose of the projected continuity / CN update), k_energy_grad and
// k_adj_init_field, and small reductions.
#include <hip/hip_runtime.h>
#include <limits.h>
#include <math.h>

#include <type_traits>

#include "adjoint.h"
#include "gmhc_internal.h"

namespace gmhc {

namespace {

// ---- quadratic B-spline S_2 and its first two derivatives --------------------------
__device__ __forceinline__ double s2(double t) {
  const double a = fabs(t);
  if (a < 0.5) return 0.75 - t * t;
  if (a < 1.5) return 0.5 * (1.5 - a) * (1.5 - a);
  return 0.0;
}
__device__ __forceinline__ double s2d(double t) {
  const double a = fabs(t);
  if (a < 0.5) return -2.0 * t;
  if (a < 1.5) return t > 0.0 ? -(1.5 - a) : (1.5 - a);
  return 0.0;
}
__device__ __forceinline__ double s2dd(double t) {
  const double a = fabs(t);
  if (a < 0.5) return -2.0;
  if (a < 1.5) return 1.0;
  return 0.0;
}
__device__ __forceinline__ int wrapi(int i, int n) { return ((i % n) + n) % n; }

__device__ __forceinline__ void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Weights of the 3^D stencil nodes around a point xs (unit offsets) and their first and
// second derivatives with respect to the position: node (o_0, o_1) of the stencil, its
// mesh index, S, dS/dx_j and d2S/dx_j dx_k.
template <int D>
struct NodeWeights {
  int i0[3];
  double w[3][3], w1[3][3], w2[3][3];  // per axis and offset -1, 0, +1: S_2, S_2' / h, S_2'' / h^2
  __device__ __forceinline__ void at(const Mesh& M, const double xs[D]) {
    int b[D];
    for (int l = 0; l < D; ++l) b[l] = (int)floor(xs[l] + 0.5);
    at_base(M, xs, b);
  }
  // the same with the stencil's centre node given (a segment's node, taken at its midpoint)
  __device__ __forceinline__ void at_base(const Mesh& M, const double xs[D], const int b[D]) {
#pragma unroll
    for (int l = 0; l < D; ++l) {
      i0[l] = b[l];
      const double ih = M.inv_h[l];
#pragma unroll
      for (int o = 0; o < 3; ++o) {
        const double t = xs[l] - (double)(i0[l] + o - 1);
        w[l][o] = s2(t);
        w1[l][o] = s2d(t) * ih;
        w2[l][o] = s2dd(t) * ih * ih;
      }
    }
  }
  // node k = ox + 3 (oy + 3 oz) of the stencil
  __device__ __forceinline__ static int off(int l, int k) { return l == 0 ? k % 3 : (l == 1 ? (k / 3) % 3 : k / 9); }
  __device__ __forceinline__ int node(const Mesh& M, int k) const {
    int g = wrapi(i0[0] + off(0, k) - 1, M.n[0]);
    if (D > 1) g += M.n[0] * wrapi(i0[D > 1 ? 1 : 0] + off(1, k) - 1, M.n[1]);
    if (D > 2) g += M.n[0] * M.n[1] * wrapi(i0[D > 2 ? 2 : 0] + off(2, k) - 1, M.n[2]);
    return g;
  }
  __device__ __forceinline__ int unode(int l, int k) const { return i0[l] + off(l, k) - 1; }
  __device__ __forceinline__ void vals(int k, double& S, double dS[D], double ddS[D][D]) const {
    const int o[3] = {k % 3, (k / 3) % 3, k / 9};
    S = 1.0;
    for (int l = 0; l < D; ++l) S *= w[l][o[l]];
    for (int j = 0; j < D; ++j) {
      dS[j] = 1.0;
      for (int l = 0; l < D; ++l) dS[j] *= l == j ? w1[l][o[l]] : w[l][o[l]];
      for (int m = 0; m < D; ++m) {
        ddS[j][m] = 1.0;
        for (int l = 0; l < D; ++l) {
          const int ord = (l == j) + (l == m);
          ddS[j][m] *= ord == 0 ? w[l][o[l]] : (ord == 1 ? w1[l][o[l]] : w2[l][o[l]]);
        }
      }
    }
  }
};
template <int D>
constexpr int kStencil = D == 1 ? 3 : (D == 2 ? 9 : 27);

// Orbit quantities of one particle: the gathers the evaluation uses (grad-phi-bar, D,
// A^-, A^+), their derivatives with respect to the start x_j and the displacement
// dx_j = dt vbar_j, and the gathers of the adjoint current mu along the orbit (the
// transpose of the deposit).
template <int D>
struct Gath {
  double Gp[D], Dm[3][D], Am[3], Ap[3];
  double Gp_x[D][D], Gp_dx[D][D], D_x[3][D][D], D_dx[3][D][D], Am_x[3][D], Ap_x[3][D];
  double Mc[3], Mx[D], Mdx[D];
};

// Knot-split walk of the orbit xi(s) = xi0 + s dxi, s in [0, 1] (knots of S_2 at
// half-integer node offsets on every axis), calling f(s, wq) at every Gauss-Legendre
// point of every segment.
template <int D, class Fn>
__device__ __forceinline__ void walk_orbit(const AdjArgs& a, const double xi0[D], const double dxi[D], Fn&& f) {
  double kn[D], sk[D];
  for (int l = 0; l < D; ++l) {
    kn[l] = dxi[l] > 0.0 ? floor(xi0[l] - 0.5) + 1.5 : ceil(xi0[l] - 0.5) - 0.5;
    sk[l] = dxi[l] != 0.0 ? (kn[l] - xi0[l]) / dxi[l] : 2.0;
  }
  double sa = 0.0;
  for (int c = 0; c <= D * (kMaxCross + 1); ++c) {
    double sb = 1.0;
    for (int l = 0; l < D; ++l)
      if (sk[l] > sa && sk[l] < sb) sb = sk[l];
    if (sb > sa) {
      const double len = sb - sa;
      for (int k = 0; k < a.ngl; ++k) f(sa + len * a.glx[k], len * a.glw[k]);
    }
    if (sb >= 1.0) break;
    for (int l = 0; l < D; ++l)
      if (sk[l] <= sb) {
        kn[l] += dxi[l] > 0.0 ? 1.0 : -1.0;
        sk[l] = (kn[l] - xi0[l]) / dxi[l];
      }
    sa = sb;
  }
}

// The knot-split segments [sa, sb] of the same walk, one step at a time, so that the
// lanes of a wave can take their segments in lockstep: step() gives the lane's segment of
// this step (false for a step of zero length or a finished walk), advance() moves past it.
template <int D>
struct SegWalk {
  double kn[D], sk[D], sa, sb;
  bool live;
  __device__ __forceinline__ void init(const double xi0[D], const double dxi[D], bool on) {
    for (int l = 0; l < D; ++l) {
      kn[l] = dxi[l] > 0.0 ? floor(xi0[l] - 0.5) + 1.5 : ceil(xi0[l] - 0.5) - 0.5;
      sk[l] = dxi[l] != 0.0 ? (kn[l] - xi0[l]) / dxi[l] : 2.0;
    }
    sa = sb = 0.0;
    live = on;
  }
  __device__ __forceinline__ bool step() {
    if (!live) return false;
    sb = 1.0;
    for (int l = 0; l < D; ++l)
      if (sk[l] > sa && sk[l] < sb) sb = sk[l];
    return sb > sa;
  }
  __device__ __forceinline__ void advance(const double xi0[D], const double dxi[D]) {
    if (!live) return;
    if (sb >= 1.0) {
      live = false;
      return;
    }
    for (int l = 0; l < D; ++l)
      if (sk[l] <= sb) {
        kn[l] += dxi[l] > 0.0 ? 1.0 : -1.0;
        sk[l] = (kn[l] - xi0[l]) / dxi[l];
      }
    sa = sb;
  }
};

template <int D, bool MU>
__device__ void gather(const AdjArgs& a, const double x[D], const double v[3], Gath<D>& G) {
  const Mesh& M = a.M;
  const int64_t Ng = M.Ng;
  double xi0[D], dxi[D];
  for (int l = 0; l < D; ++l) {
    xi0[l] = (x[l] - M.lo[l]) * M.inv_h[l];
    dxi[l] = a.dt * v[l] * M.inv_h[l];
  }
  G = Gath<D>{};
  NodeWeights<D> nw;
  walk_orbit<D>(a, xi0, dxi, [&](double s, double wq) {
    double xs[D];
    for (int l = 0; l < D; ++l) xs[l] = xi0[l] + s * dxi[l];
    nw.at(M, xs);
    #pragma unroll
    for (int k = 0; k < kStencil<D>; ++k) {
      double S, dS[D], ddS[D][D];
      nw.vals(k, S, dS, ddS);
      const int g = nw.node(M, k);
      for (int l = 0; l < D; ++l) {
        const double gp = a.gphi[l * Ng + g];
        G.Gp[l] += wq * S * gp;
        for (int j = 0; j < D; ++j) {
          G.Gp_x[l][j] += wq * dS[j] * gp;
          G.Gp_dx[l][j] += wq * s * dS[j] * gp;
        }
      }
      double vm = 0.0;
      for (int c = 0; c < 3; ++c) {
        const double As = (1.0 - s) * a.An[c * Ng + g] + s * a.Anp1[c * Ng + g];
        for (int l = 0; l < D; ++l) {
          G.Dm[c][l] += wq * dS[l] * As;
          for (int j = 0; j < D; ++j) {
            G.D_x[c][l][j] += wq * ddS[l][j] * As;
            G.D_dx[c][l][j] += wq * s * ddS[l][j] * As;
          }
        }
        if (MU) {
          const double m = a.mu[c * Ng + g];
          G.Mc[c] += wq * S * m;
          vm += v[c] * m;
        }
      }
      if (MU)
        for (int j = 0; j < D; ++j) {
          G.Mx[j] += wq * dS[j] * vm;
          G.Mdx[j] += wq * s * dS[j] * vm;
        }
    }
  });
  // endpoint interpolants A^n(x) and A^{n+1}(x + dx)
  for (int e = 0; e < 2; ++e) {
    double xs[D];
    for (int l = 0; l < D; ++l) xs[l] = xi0[l] + (e ? dxi[l] : 0.0);
    nw.at(M, xs);
    const double* F = e ? a.Anp1 : a.An;
    #pragma unroll
    for (int k = 0; k < kStencil<D>; ++k) {
      double S, dS[D], ddS[D][D];
      nw.vals(k, S, dS, ddS);
      const int g = nw.node(M, k);
      for (int c = 0; c < 3; ++c) {
        const double f = F[c * Ng + g];
        (e ? G.Ap : G.Am)[c] += S * f;
        for (int j = 0; j < D; ++j) (e ? G.Ap_x : G.Am_x)[c][j] += dS[j] * f;
      }
    }
  }
}

// Forward values of one evaluation (no-explicit-A_t GM-HC step, mechanical endpoints,
// electric-work secant velocities) that the reverse sweep needs.
template <int D>
struct Fwd {
  double q, m, mk, dt, kappa, v[D];
  double Gp[D], Dm[3][D], Am[3], Ap[3];
  double Aep[3], kick[3], pm[3], um[3], tau[3], up[3], pp[3], Pn1[3], pn[3], pn1[3];
  double gm2, sigma, X, R, gHC, t[3], t2, s[3], ustar[3], ut;
  double vEm[3], vEp[3];
  // B_eff = (K23, -K13, K12) of K = D~^T - D~, D~ the zero-padded 3x3 D
  __device__ __forceinline__ double dz(int c, int l) const { return l < D ? Dm[c][l] : 0.0; }
};

__device__ double gam(const double p[3], double mk) { return sqrt(1.0 + dot3(p, p) / (mk * mk)); }

template <int D>
__device__ void forward(const Gath<D>& G, const double P[3], double q, double m, const double v[3], double dt,
                        double kappa, Fwd<D>& f) {
  f.q = q;
  f.m = m;
  f.mk = m * kappa;
  f.dt = dt;
  f.kappa = kappa;
  for (int l = 0; l < D; ++l) {
    f.v[l] = v[l];
    f.Gp[l] = G.Gp[l];
  }
  for (int c = 0; c < 3; ++c) {
    double Dv = 0.0;
    for (int l = 0; l < D; ++l) {
      f.Dm[c][l] = G.Dm[c][l];
      Dv += G.Dm[c][l] * v[l];
    }
    f.Am[c] = G.Am[c];
    f.Ap[c] = G.Ap[c];
    f.Aep[c] = 0.5 * (G.Am[c] + G.Ap[c]);
    f.kick[c] = 0.5 * dt * q * (Dv - (c < D ? G.Gp[c] : 0.0));
    f.pm[c] = P[c] - q * f.Aep[c] + f.kick[c];
    f.um[c] = f.pm[c] / f.mk;
  }
  const double Beff[3] = {f.dz(2, 1) - f.dz(1, 2), -(f.dz(2, 0) - f.dz(0, 2)), f.dz(1, 0) - f.dz(0, 1)};
  for (int c = 0; c < 3; ++c) f.tau[c] = dt * q / (2.0 * m) * Beff[c];
  // normalized HC map
  f.gm2 = 1.0 + dot3(f.um, f.um);
  const double tau2 = dot3(f.tau, f.tau);
  f.ut = dot3(f.um, f.tau);
  f.sigma = f.gm2 - tau2;
  f.X = tau2 + f.ut * f.ut;
  f.R = sqrt(f.sigma * f.sigma + 4.0 * f.X);
  const double g2 = f.sigma >= 0.0 ? 0.5 * (f.sigma + f.R) : 2.0 * f.X / (f.R - f.sigma);
  f.gHC = sqrt(g2);
  for (int c = 0; c < 3; ++c) f.t[c] = f.tau[c] / f.gHC;
  f.t2 = dot3(f.t, f.t);
  for (int c = 0; c < 3; ++c) f.s[c] = 2.0 * f.t[c] / (1.0 + f.t2);
  double uxt[3], usxs[3];
  cross3(f.um, f.t, uxt);
  for (int c = 0; c < 3; ++c) f.ustar[c] = f.um[c] + uxt[c];
  cross3(f.ustar, f.s, usxs);
  for (int c = 0; c < 3; ++c) {
    f.up[c] = f.um[c] + usxs[c];
    f.pp[c] = f.mk * f.up[c];
    f.Pn1[c] = f.pp[c] + q * f.Aep[c] + f.kick[c];
    f.pn[c] = P[c] - q * f.Am[c];
    f.pn1[c] = f.Pn1[c] - q * f.Ap[c];
  }
  const double gm = gam(f.pm, f.mk), gn = gam(f.pn, f.mk), gn1 = gam(f.pn1, f.mk), gp = gam(f.pp, f.mk);
  for (int c = 0; c < 3; ++c) {
    f.vEm[c] = (f.pm[c] + f.pn[c]) / (m * (gm + gn));
    f.vEp[c] = (f.pn1[c] + f.pp[c]) / (m * (gn1 + gp));
  }
}

// Reverse sweep of the secant velocity V(a, b) = (a + b) / (m (gamma(a) + gamma(b))):
// adds the cotangents of a, b and m for the cotangent fb of V.
__device__ void vdg_rev(const double pa[3], const double pb[3], const double f[3], double m, double mk,
                        const double fb[3], double ab[3], double bb[3], double& mb) {
  const double ga = gam(pa, mk), gb = gam(pb, mk), G = ga + gb;
  double S[3];
  for (int c = 0; c < 3; ++c) S[c] = pa[c] + pb[c];
  const double fs = dot3(fb, S);
  const double k = fs / (m * G * G);
  for (int c = 0; c < 3; ++c) {
    ab[c] += fb[c] / (m * G) - k * pa[c] / (mk * mk * ga);
    bb[c] += fb[c] / (m * G) - k * pb[c] / (mk * mk * gb);
  }
  // m enters through the prefactor 1/m and through gamma: d gamma(a)/dm = -(|a|/mk)^2 / (m gamma(a))
  const double dga = -dot3(pa, pa) / (mk * mk) / (m * ga), dgb = -dot3(pb, pb) / (mk * mk) / (m * gb);
  mb += -dot3(fb, f) / m - dot3(fb, f) / G * (dga + dgb);
}

// Cotangents of the evaluation's inputs for the cotangents wv of v_out and wP of P^{n+1}.
template <int D>
struct Rev {
  double Gp[D], Dm[3][D], Am[3], Ap[3];  // gathers
  double P[3], q, m, v[D];               // direct inputs (v through the kick only)
};

template <int D>
__device__ void reverse(const Fwd<D>& f, const double wv[3], const double wP[3], Rev<D>& r) {
  r = Rev<D>{};
  const double m = f.m, mk = f.mk, q = f.q, dt = f.dt;
  double vEb[3], pmb[3] = {}, pnb[3] = {}, pn1b[3] = {}, ppb[3] = {}, Pn1b[3], Aepb[3] = {}, kickb[3] = {};
  for (int c = 0; c < 3; ++c) {
    vEb[c] = 0.5 * wv[c];
    Pn1b[c] = wP[c];
  }
  vdg_rev(f.pm, f.pn, f.vEm, m, mk, vEb, pmb, pnb, r.m);
  vdg_rev(f.pn1, f.pp, f.vEp, m, mk, vEb, pn1b, ppb, r.m);
  for (int c = 0; c < 3; ++c) {
    // pn1 = Pn1 - q Ap ; pn = P - q Am
    Pn1b[c] += pn1b[c];
    r.Ap[c] -= q * pn1b[c];
    r.q -= pn1b[c] * f.Ap[c];
    r.P[c] += pnb[c];
    r.Am[c] -= q * pnb[c];
    r.q -= pnb[c] * f.Am[c];
    // Pn1 = pp + q Aep + kick
    ppb[c] += Pn1b[c];
    Aepb[c] += q * Pn1b[c];
    kickb[c] += Pn1b[c];
    r.q += Pn1b[c] * f.Aep[c];
  }
  // pp = mk up
  double upb[3];
  for (int c = 0; c < 3; ++c) upb[c] = mk * ppb[c];
  r.m += f.kappa * dot3(ppb, f.up);
  // normalized HC map, reversed: up = um + ustar x s, ustar = um + um x t,
  // s = 2 t / (1 + |t|^2), t = tau / gamma_HC, gamma_HC^2 = (sigma + R) / 2,
  // R^2 = sigma^2 + 4 X, X = |tau|^2 + (u.tau)^2, sigma = 1 + |u|^2 - |tau|^2.
  double umb[3], ustarb[3], sb[3], tb[3], taub[3];
  for (int c = 0; c < 3; ++c) umb[c] = upb[c];
  cross3(f.s, upb, ustarb);  // d(ustar x s)/d ustar
  cross3(upb, f.ustar, sb);  // d(ustar x s)/d s
  for (int c = 0; c < 3; ++c) umb[c] += ustarb[c];
  {
    double a1[3];
    cross3(f.t, ustarb, a1);  // d(um x t)/d um
    for (int c = 0; c < 3; ++c) umb[c] += a1[c];
    cross3(ustarb, f.um, tb);  // d(um x t)/d t
  }
  const double den = 1.0 + f.t2, st = dot3(sb, f.t);
  for (int c = 0; c < 3; ++c) tb[c] += 2.0 * sb[c] / den - 4.0 * st / (den * den) * f.t[c];
  for (int c = 0; c < 3; ++c) taub[c] = tb[c] / f.gHC;
  const double gHCb = -dot3(tb, f.t) / f.gHC;
  const double g2b = gHCb / (2.0 * f.gHC);
  // d g2 / d sigma = (1 + sigma / R) / 2, written without cancellation for sigma < 0
  const double dsig = f.sigma >= 0.0 ? 0.5 * (1.0 + f.sigma / f.R) : 2.0 * f.X / (f.R * (f.R - f.sigma));
  const double sigmab = g2b * dsig;
  const double Xb = g2b / f.R;
  const double tau2b = Xb - sigmab;
  const double utb = 2.0 * f.ut * Xb;
  const double gm2b = sigmab;
  for (int c = 0; c < 3; ++c) {
    umb[c] += utb * f.tau[c] + 2.0 * gm2b * f.um[c];
    taub[c] += utb * f.um[c] + 2.0 * tau2b * f.tau[c];
  }
  // tau = (dt q / 2m) B_eff, B_eff = (D_zy - D_yz, -(D_zx - D_xz), D_yx - D_xy) (zero-padded D)
  const double Beff[3] = {f.dz(2, 1) - f.dz(1, 2), -(f.dz(2, 0) - f.dz(0, 2)), f.dz(1, 0) - f.dz(0, 1)};
  const double kq = dt * q / (2.0 * m);
  r.q += dt / (2.0 * m) * dot3(taub, Beff);
  r.m -= dot3(taub, f.tau) / m;
  const double Bb[3] = {kq * taub[0], kq * taub[1], kq * taub[2]};
  r.Dm[2][0] -= Bb[1];
  r.Dm[1][0] += Bb[2];
  if (D > 1) {
    r.Dm[2][D > 1 ? 1 : 0] += Bb[0];
    r.Dm[0][D > 1 ? 1 : 0] -= Bb[2];
  }
  if (D > 2) {
    r.Dm[1][D > 2 ? 2 : 0] -= Bb[0];
    r.Dm[0][D > 2 ? 2 : 0] += Bb[1];
  }
  // um = pm / mk
  for (int c = 0; c < 3; ++c) pmb[c] += umb[c] / mk;
  r.m -= dot3(umb, f.um) / m;
  // pm = P - q Aep + kick
  for (int c = 0; c < 3; ++c) {
    r.P[c] += pmb[c];
    Aepb[c] -= q * pmb[c];
    kickb[c] += pmb[c];
    r.q -= pmb[c] * f.Aep[c];
  }
  // kick = (dt q / 2) (D v - grad-phi-bar)
  for (int c = 0; c < 3; ++c) {
    double Dv = 0.0;
    for (int l = 0; l < D; ++l) {
      r.Dm[c][l] += 0.5 * dt * q * f.v[l] * kickb[c];
      r.v[l] += 0.5 * dt * q * f.Dm[c][l] * kickb[c];
      Dv += f.Dm[c][l] * f.v[l];
    }
    r.q += 0.5 * dt * (Dv - (c < D ? f.Gp[c] : 0.0)) * kickb[c];
  }
  for (int l = 0; l < D; ++l) r.Gp[l] -= 0.5 * dt * q * kickb[l];
  // Aep = (Am + Ap) / 2
  for (int c = 0; c < 3; ++c) {
    r.Am[c] += 0.5 * Aepb[c];
    r.Ap[c] += 0.5 * Aepb[c];
  }
}

// Cotangent of vbar_j (through the kick and through the orbit gathers) and of x_j.
template <int D>
__device__ __forceinline__ double rev_v(const Rev<D>& r, const Gath<D>& G, double dt, int j) {
  double s = 0.0;
  for (int l = 0; l < D; ++l) s += r.Gp[l] * G.Gp_dx[l][j];
  for (int c = 0; c < 3; ++c) {
    for (int l = 0; l < D; ++l) s += r.Dm[c][l] * G.D_dx[c][l][j];
    s += r.Ap[c] * G.Ap_x[c][j];
  }
  return r.v[j] + dt * s;
}
template <int D>
__device__ __forceinline__ double rev_x(const Rev<D>& r, const Gath<D>& G, int j) {
  double s = 0.0;
  for (int l = 0; l < D; ++l) s += r.Gp[l] * G.Gp_x[l][j];
  for (int c = 0; c < 3; ++c) {
    for (int l = 0; l < D; ++l) s += r.Dm[c][l] * G.D_x[c][l][j];
    s += r.Am[c] * G.Am_x[c][j] + r.Ap[c] * G.Ap_x[c][j];
  }
  return s;
}

// Solve (I - J^T) mu = rhs for the transposed inner system, with J[c][j] = dv_out,c /
// dvbar_j nonzero for j < D only (Cramer's rule on the 3x3 matrix).
template <int D>
__device__ __forceinline__ void inner_solve(const double J[3][D], const double rhs[3], double mu[3]) {
  double A[3][3];
  for (int j = 0; j < 3; ++j)
    for (int c = 0; c < 3; ++c) A[j][c] = (j == c ? 1.0 : 0.0) - (j < D ? J[c][j < D ? j : 0] : 0.0);
  const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                     A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
  for (int k = 0; k < 3; ++k) {
    double B[3][3];
    for (int j = 0; j < 3; ++j)
      for (int c = 0; c < 3; ++c) B[j][c] = c == k ? rhs[j] : A[j][c];
    mu[k] = (B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1]) - B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0]) +
             B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0])) / det;
  }
}

// Gather cotangents of one reverse sweep as a flat list: grad-phi-bar (D), D (3 D),
// A^- (3), A^+ (3).
template <int D>
__device__ __forceinline__ void rev_gath(const Rev<D>& r, double g[adj_ngath(D)]) {
  for (int l = 0; l < D; ++l) g[l] = r.Gp[l];
  for (int c = 0; c < 3; ++c) {
    for (int l = 0; l < D; ++l) g[D + c * D + l] = r.Dm[c][l];
    g[4 * D + c] = r.Am[c];
    g[4 * D + 3 + c] = r.Ap[c];
  }
}

// Exact fixed-point accumulation of one workgroup's scattered values: a window of
// kWinX x kWinY (1D: kWinX) consecutive unwrapped nodes from wlo per field array in LDS,
// summed with 64-bit integer LDS atomics and added to the global accumulator once per
// workgroup; values at nodes outside the window go to the global accumulator directly.
// Integer sums are exact, so the result does not depend on the order of arrival.
template <int D>
constexpr int kWinX = D == 1 ? 32 : 16;
template <int D>
constexpr int kWinY = D == 1 ? 1 : (D == 2 ? 8 : 4);
template <int D>
constexpr int kWinZ = D == 3 ? 4 : 1;
template <int D>
constexpr int kWinNodes = kWinX<D> * kWinY<D> * kWinZ<D>;

// Sum of a 64-bit integer over the 64 lanes of a wave (all lanes active), left on every
// lane: partners lane ^ 1 and lane ^ 2 (quad permutations), lane ^ 7 within eight lanes
// (half-row mirror), lane ^ 8 (row rotation by eight), then the row swaps lane ^ 16 and
// lane ^ 32.  Integer addition is exact, so the total does not depend on the order.
template <int CTRL>
__device__ __forceinline__ long long dpp_i64(long long x) {
  const uint64_t u = (uint64_t)x;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return (long long)(((uint64_t)hi << 32) | lo);
}
template <bool ROW16>
__device__ __forceinline__ long long swap_i64(long long x) {
  const uint64_t u = (uint64_t)x;
  const uint32_t lo = (uint32_t)u, hi = (uint32_t)(u >> 32);
  // the swap exchanges half the rows of its two operands; given the value twice, one
  // result is the lane's own value and the other its partner's, and their sum is the pair's
  if (ROW16) {
    const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
    return (long long)((((uint64_t)h[0] << 32) | l[0]) + (((uint64_t)h[1] << 32) | l[1]));
  } else {
    const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
    return (long long)((((uint64_t)h[0] << 32) | l[0]) + (((uint64_t)h[1] << 32) | l[1]));
  }
}
__device__ __forceinline__ long long wave_sum_i64(long long x) {
  x += dpp_i64<0xB1>(x);   // quad_perm [1, 0, 3, 2]: lane ^ 1
  x += dpp_i64<0x4E>(x);   // quad_perm [2, 3, 0, 1]: lane ^ 2
  x += dpp_i64<0x141>(x);  // row_half_mirror: lane ^ 7
  x += dpp_i64<0x128>(x);  // row_ror:8: lane ^ 8
  x = swap_i64<true>(x);   // lane ^ 16
  return swap_i64<false>(x);  // lane ^ 32
}

// Reduce-scatter of 32 64-bit values (integers or FP64) per lane over the wave (all lanes
// active): after it, lane l holds the wave total of value slot32(l), and the lanes with l
// even hold one copy of each of the 32 totals.  Each step halves the values a lane holds:
// it keeps one half and adds its partner's copy of that half (partners lane ^ 32 and
// lane ^ 16 by the row swaps, lane ^ 8, lane ^ 7 and lane ^ 2 by DPP); the last step adds
// the lane ^ 1 partner's copy of the one value left.  The six partners span the wave, and
// the order of the additions is fixed, so FP64 totals are the same on every run.
__device__ __forceinline__ uint64_t bits64(long long x) { return (uint64_t)x; }
__device__ __forceinline__ uint64_t bits64(double x) { return (uint64_t)__double_as_longlong(x); }
template <class T>
__device__ __forceinline__ T from64(uint64_t u) {
  if constexpr (std::is_floating_point<T>::value) return __longlong_as_double((long long)u);
  else return (T)u;
}
template <bool ROW16, class T>
__device__ __forceinline__ T swap2(T A, T B) {
  // the lower rows of the swap keep A and receive the partner's A, the upper rows keep B
  // and receive the partner's B
  const uint64_t a = bits64(A), b = bits64(B);
  const uint32_t alo = (uint32_t)a, ahi = (uint32_t)(a >> 32), blo = (uint32_t)b, bhi = (uint32_t)(b >> 32);
  if (ROW16) {
    const auto l = __builtin_amdgcn_permlane16_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane16_swap(ahi, bhi, false, false);
    return from64<T>(((uint64_t)h[0] << 32) | l[0]) + from64<T>(((uint64_t)h[1] << 32) | l[1]);
  } else {
    const auto l = __builtin_amdgcn_permlane32_swap(alo, blo, false, false);
    const auto h = __builtin_amdgcn_permlane32_swap(ahi, bhi, false, false);
    return from64<T>(((uint64_t)h[0] << 32) | l[0]) + from64<T>(((uint64_t)h[1] << 32) | l[1]);
  }
}
template <int CTRL, class T>
__device__ __forceinline__ T dpp64(T x) {
  const uint64_t u = bits64(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return from64<T>(((uint64_t)hi << 32) | lo);
}
template <int H, int CTRL, class T>
__device__ __forceinline__ void dpp_half(T* v, bool up) {
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const T send = up ? v[j] : v[j + H];
    const T keep = up ? v[j + H] : v[j];
    v[j] = keep + dpp64<CTRL>(send);
  }
}
template <class T>
__device__ __forceinline__ T rs32(T (&v)[32], int lane) {
#pragma unroll
  for (int j = 0; j < 16; ++j) v[j] = swap2<false>(v[j], v[j + 16]);
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = swap2<true>(v[j], v[j + 8]);
  dpp_half<4, 0x128>(v, (lane & 8) != 0);  // row_ror:8
  dpp_half<2, 0x141>(v, (lane & 4) != 0);  // row_half_mirror
  dpp_half<1, 0x4E>(v, (lane & 2) != 0);   // quad_perm [2, 3, 0, 1]
  return v[0] + dpp64<0xB1>(v[0]);         // quad_perm [1, 0, 3, 2]
}
__device__ __forceinline__ int slot32(int lane) {
  return 16 * ((lane >> 5) & 1) + 8 * ((lane >> 4) & 1) + 4 * ((lane >> 3) & 1) + 2 * ((lane >> 2) & 1) +
         ((lane >> 1) & 1);
}

template <int D>
struct WinAcc {
  unsigned long long* s;  // [D + 6][kWinNodes] pairs
  unsigned long long* g;  // global [D + 6][Ng] pairs
  int wlo[3];
  const Mesh* M;
  double up;
  // window-relative index of an unwrapped node, -1 outside the window
  __device__ __forceinline__ int rel(const int node[D]) const {
    int r = 0;
    bool in = true;
    for (int l = 0; l < D; ++l) {
      const int o = node[l] - wlo[l];
      const int e = l == 0 ? kWinX<D> : (l == 1 ? kWinY<D> : kWinZ<D>);
      in = in && o >= 0 && o < e;
      r += l == 0 ? o : (l == 1 ? o * kWinX<D> : o * kWinX<D> * kWinY<D>);
    }
    return in ? r : -1;
  }
  // The put of NE entries by a whole wave whose lanes all target the same window nodes
  // (every lane active; a lane without a value passes zeros): entry e has the value
  // val(e) on each lane and the window entry ent(e) (field * window nodes + node, the
  // same on every lane).  The values are summed over the wave in FP64 by reduce-scatters
  // of 32 entries at a time (a fixed order of additions), and the lane holding a total
  // splits it into limbs and adds them: one LDS atomic per entry and limb instead of one
  // per lane, and one split per entry instead of one per lane.
  template <int NE, class Val, class Ent>
  __device__ __forceinline__ void put_all(Val&& val, Ent&& ent, int lane) const {
#pragma unroll
    for (int c0 = 0; c0 < NE; c0 += 32) {
      double v[32];
#pragma unroll
      for (int i = 0; i < 32; ++i) v[i] = c0 + i < NE ? val(c0 + i) : 0.0;
      const double tot = rs32(v, lane);
      const int e = c0 + slot32(lane);
      if ((lane & 1) == 0 && e < NE && tot != 0.0) {
        long long H, L;
        fix_split(tot, up, H, L);
        const int k = 2 * ent(e);
        if (H) atomicAdd(s + k, (unsigned long long)H);
        if (L) atomicAdd(s + k + 1, (unsigned long long)L);
      }
    }
  }
  // The put of a whole wave (every lane active; a lane without a value passes v = 0).
  // Lanes whose limbs go to the same window entry are summed across the wave first and
  // added by one lane, which takes the 64-way same-address serialization off the LDS
  // atomics; up to two such groups are taken, the rest add their own limbs.  Integer sums
  // do not depend on the grouping, so every entry ends with the same bits as when each
  // lane adds its own limbs.
  __device__ __forceinline__ void put_wave(int f, int r, const int node[D], double v, int lane) const {
    long long H, L;
    fix_split(v, up, H, L);
    const bool c = (H | L) != 0;
    if (c && r < 0) {
      int gi = wrapi(node[0], M->n[0]);
      if (D > 1) gi += M->n[0] * wrapi(node[D > 1 ? 1 : 0], M->n[1]);
      if (D > 2) gi += M->n[0] * M->n[1] * wrapi(node[D > 2 ? 2 : 0], M->n[2]);
      if (H) atomicAdd(g + 2 * ((int64_t)f * M->Ng + gi), (unsigned long long)H);
      if (L) atomicAdd(g + 2 * ((int64_t)f * M->Ng + gi) + 1, (unsigned long long)L);
    }
    bool pend = c && r >= 0;
    uint64_t act = __ballot(pend);
#pragma unroll 1
    for (int round = 0; round < 2 && act != 0; ++round) {
      const int lead = __ffsll((long long)act) - 1;  // wave-uniform
      const int rl = __builtin_amdgcn_readlane(r, lead);
      const bool mine = pend && r == rl;
      const long long hs = wave_sum_i64(mine ? H : 0ll), ls = wave_sum_i64(mine ? L : 0ll);
      if (lane == lead) {
        const int k = 2 * (f * kWinNodes<D> + rl);
        if (hs) atomicAdd(s + k, (unsigned long long)hs);
        if (ls) atomicAdd(s + k + 1, (unsigned long long)ls);
      }
      pend = pend && !mine;
      act = __ballot(pend);
    }
    if (pend) {
      const int k = 2 * (f * kWinNodes<D> + r);
      if (H) atomicAdd(s + k, (unsigned long long)H);
      if (L) atomicAdd(s + k + 1, (unsigned long long)L);
    }
  }
};

// Gather of the adjoint current mu along the orbit (the transposed deposit): Mc = sum_g
// mu_g int S_g, Mdx_j = sum_g (v . mu_g) int s dS_g/dx_j.
template <int D>
__device__ __forceinline__ void gather_mu(const AdjArgs& a, const double xi0[D], const double dxi[D],
                                         const double v[3], double Mc[3], double Mdx[D]) {
  const Mesh& M = a.M;
  const int64_t Ng = M.Ng;
  Mc[0] = Mc[1] = Mc[2] = 0.0;
  for (int j = 0; j < D; ++j) Mdx[j] = 0.0;
  NodeWeights<D> nw;
  walk_orbit<D>(a, xi0, dxi, [&](double s, double wq) {
    double xs[D];
    for (int l = 0; l < D; ++l) xs[l] = xi0[l] + s * dxi[l];
    nw.at(M, xs);
    #pragma unroll
    for (int k = 0; k < kStencil<D>; ++k) {
      double S, dS[D], ddS[D][D];
      nw.vals(k, S, dS, ddS);
      const int g = nw.node(M, k);
      double vm = 0.0;
      for (int c = 0; c < 3; ++c) {
        const double m = a.mu[c * Ng + g];
        Mc[c] += wq * S * m;
        vm += v[c] * m;
      }
      for (int j = 0; j < D; ++j) Mdx[j] += wq * s * dS[j] * vm;
    }
  });
}

// ADJ_PREP: the reverse sweeps of one particle's evaluation for the unit cotangents and lP;
// ADJ_FINAL: the sweep for the converged (mu_v, lP), which gives the input cotangents.
// Occupancy target by measurement: two waves per SIMD in 1D (the final sweep then spills
// 60 B per lane), the register file of one wave in 2D and 3D.
template <int D, bool FINAL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(D == 1 ? 2 : 1))) void k_adj_particle(
    AdjArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.np) return;
  const Mesh& M = a.M;
  constexpr int NG = adj_ngath(D);
  const int64_t li = a.id[i];
  const double q = a.q[i], m = fabs(q);
  double x[D], P[3], v[3], lP[3], lx[D];
  for (int l = 0; l < D; ++l) {
    x[l] = a.x[l * a.ps + i];
    lx[l] = a.lx[l * a.np + li];
  }
  for (int c = 0; c < 3; ++c) {
    P[c] = a.P[c * a.ps + i];
    v[c] = a.vbar[c * a.np + li];
    lP[c] = a.lP[c * a.np + li];
  }
  Gath<D> G;
  gather<D, FINAL>(a, x, v, G);
  Fwd<D> f;
  forward<D>(G, P, q, m, v, a.dt, a.kappa, f);
  Rev<D> r;
  // the nonzero columns j < D of dF/dvbar, and the part of the right side that does not
  // depend on the adjoint current; the final sweep reads both back from the cache the
  // preparing sweep of the same step wrote
  double J[3][D], base[D];
  if (FINAL) {
    for (int c = 0; c < 3; ++c)
      for (int j = 0; j < D; ++j) J[c][j] = a.cache[(c * D + j) * a.ps + i];
    for (int j = 0; j < D; ++j) base[j] = a.cache[(3 * D + j) * a.ps + i];
  } else {
    for (int c = 0; c < 3; ++c) {
      const double e[3] = {c == 0 ? 1.0 : 0.0, c == 1 ? 1.0 : 0.0, c == 2 ? 1.0 : 0.0}, z[3] = {0.0, 0.0, 0.0};
      reverse<D>(f, e, z, r);
      for (int j = 0; j < D; ++j) J[c][j] = rev_v<D>(r, G, a.dt, j);
      double g[NG];
      rev_gath<D>(r, g);
      for (int k = 0; k < NG; ++k) a.cache[(4 * D + c * NG + k) * a.ps + i] = g[k];
    }
    // right side: x^{n+1} = x + dt vbar, P^{n+1}(vbar), and the transposed deposit
    const double z3[3] = {0.0, 0.0, 0.0};
    reverse<D>(f, z3, lP, r);
    for (int j = 0; j < D; ++j) base[j] = a.dt * lx[j] + rev_v<D>(r, G, a.dt, j);
  }
  if (!FINAL) {
    double g[NG];
    rev_gath<D>(r, g);
    for (int k = 0; k < NG; ++k) a.cache[(4 * D + 3 * NG + k) * a.ps + i] = g[k];
    for (int c = 0; c < 3; ++c)
      for (int j = 0; j < D; ++j) a.cache[(c * D + j) * a.ps + i] = J[c][j];
    for (int j = 0; j < D; ++j) a.cache[(3 * D + j) * a.ps + i] = base[j];
    return;
  }
  const double qdv = q / M.dV;
  double rhs[3], mv[3];
  for (int c = 0; c < 3; ++c) rhs[c] = qdv * G.Mc[c];
  for (int j = 0; j < D; ++j) rhs[j] += base[j] + qdv * a.dt * G.Mdx[j];
  inner_solve<D>(J, rhs, mv);
  reverse<D>(f, mv, lP, r);
  for (int j = 0; j < D; ++j) a.gx[j * a.np + li] = lx[j] + rev_x<D>(r, G, j) + qdv * G.Mx[j];
  for (int c = 0; c < 3; ++c) a.gP[c * a.np + li] = r.P[c];
  a.gq[li] = r.q + (q < 0.0 ? -r.m : r.m) + dot3(v, G.Mc) / M.dV;
}

// ADJ_BOUND (SCAT false) and ADJ_SCATTER (SCAT true): one transposed outer iteration from
// the cached values.  The reverse sweep is linear in its cotangents, so the gather
// cotangents for (mu_v, lP) are sum_c mu_v,c (those of e_c) + (those of lP).  The two
// modes are separate instantiations, so the bound pass carries none of the scatter's
// registers or LDS.  Occupancy target of the scatter by measurement: three waves per SIMD
// in 2D and 3D (68 and 240 B of spill per lane; 5% and 7% faster than two), and 1D's own
// three (four was slower).
template <int D, bool SCAT>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(SCAT && D > 1 ? 3 : 1))) void k_adj_iter(
    AdjArgs a) {
  constexpr int NG = adj_ngath(D);
  constexpr int NV = D + 6;
  __shared__ double red[kBlock];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < a.np;
  const Mesh& M = a.M;
  double xi0[D], dxi[D], g[NG];
  for (int l = 0; l < D; ++l) xi0[l] = dxi[l] = 0.0;
  for (int k = 0; k < NG; ++k) g[k] = 0.0;
  if (live) {
    const int64_t li = a.id[i];
    const double q = a.q[i];
    double v[3];
    for (int c = 0; c < 3; ++c) v[c] = a.vbar[c * a.np + li];
    for (int l = 0; l < D; ++l) {
      xi0[l] = (a.x[l * a.ps + i] - M.lo[l]) * M.inv_h[l];
      dxi[l] = a.dt * v[l] * M.inv_h[l];
    }
    double rhs[3] = {0.0, 0.0, 0.0}, Mdx[D];
    for (int j = 0; j < D; ++j) Mdx[j] = 0.0;
    if (a.mu) gather_mu<D>(a, xi0, dxi, v, rhs, Mdx);
    const double qdv = q / M.dV;
    for (int c = 0; c < 3; ++c) rhs[c] *= qdv;
    for (int j = 0; j < D; ++j) rhs[j] += a.cache[(3 * D + j) * a.ps + i] + qdv * a.dt * Mdx[j];
    double J[3][D], mv[3];
    for (int c = 0; c < 3; ++c)
      for (int j = 0; j < D; ++j) J[c][j] = a.cache[(c * D + j) * a.ps + i];
    inner_solve<D>(J, rhs, mv);
#pragma unroll
    for (int k = 0; k < NG; ++k) {
      double s = a.cache[(4 * D + 3 * NG + k) * a.ps + i];
      for (int c = 0; c < 3; ++c) s += mv[c] * a.cache[(4 * D + c * NG + k) * a.ps + i];
      g[k] = s;
    }
  }
  if (!SCAT) {  // per-block sum of the bound, fixed order
    double bound = 0.0;
    for (int l = 0; l < D; ++l) bound += fabs(g[l]);
    for (int c = 0; c < 3; ++c) {
      for (int l = 0; l < D; ++l) bound += 2.0 * M.inv_h[l] * fabs(g[D + c * D + l]);
      bound += fabs(g[4 * D + c]) + fabs(g[4 * D + 3 + c]);
    }
    red[threadIdx.x] = live ? bound : 0.0;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.partials[blockIdx.x] = red[0];
    return;
  }
  __shared__ unsigned long long sacc[2 * NV * kWinNodes<D>];
  __shared__ int swlo[3];
  // The window is taken periodically: each lane's nodes are moved by whole periods to lie
  // within half a period of the block's first particle (always live), so a block whose
  // particles straddle the periodic seam (a cell-sorted block at node 0 holds particles
  // just below the top of the box) still shares one window.  The shift sh only relabels
  // the nodes; the weights and the wrapped mesh indices are unchanged.
  __shared__ double sref[3];
  if (threadIdx.x < 3) swlo[threadIdx.x] = INT_MAX;
  if (threadIdx.x == 0)
    for (int l = 0; l < D; ++l) sref[l] = xi0[l];
  for (int k = threadIdx.x; k < 2 * NV * kWinNodes<D>; k += kBlock) sacc[k] = 0ull;
  __syncthreads();
  int sh[D];
  for (int l = 0; l < D; ++l) {
    const double nl = (double)M.n[l];
    sh[l] = live ? -M.n[l] * (int)rint((xi0[l] - sref[l]) / nl) : 0;
  }
  if (live)
    for (int l = 0; l < D; ++l) atomicMin(&swlo[l], (int)floor(fmin(xi0[l], xi0[l] + dxi[l]) + 0.5) - 1 + sh[l]);
  __syncthreads();
  WinAcc<D> w{sacc, a.acc, {swlo[0], swlo[1], swlo[2]}, &M, a.fx[0]};
  const int lane = threadIdx.x & 63;
  // Every lane of the wave takes part (a lane with no particle, or no segment at a step,
  // puts zeros), so the puts can sum across the wave.  Within a knot-split segment the
  // stencil nodes stay the same, so each node's weights are integrated over the segment's
  // Gauss points first (int S, int (1 - s) dS/dx_l, int s dS/dx_l) and scattered once per
  // segment.
  SegWalk<D> sw;
  sw.init(xi0, dxi, live);
#pragma unroll 1
  for (int step = 0; step <= D * (kMaxCross + 1); ++step) {
    if (__ballot(sw.live) == 0) break;
    const bool has = sw.step();
    const double sa = has ? sw.sa : 0.0, sb = has ? sw.sb : 0.0, len = sb - sa;
    int base[D];
    for (int l = 0; l < D; ++l) base[l] = (int)floor(xi0[l] + 0.5 * (sa + sb) * dxi[l] + 0.5);
    // NP parts of the stencil at a time, which bounds the nodes' integrals held live
    constexpr int NP = (D == 3 ? 9 : (D == 2 ? 3 : 1)), NK = kStencil<D> / NP;
#pragma unroll 1
    for (int pl = 0; pl < NP; ++pl) {
      double I0[NK], Ia[NK][D], Ib[NK][D];
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        I0[k] = 0.0;
        for (int l = 0; l < D; ++l) Ia[k][l] = Ib[k][l] = 0.0;
      }
      for (int q = 0; q < a.ngl; ++q) {
        const double s = sa + len * a.glx[q], wq = len * a.glw[q];
        double xs[D];
        for (int l = 0; l < D; ++l) xs[l] = xi0[l] + s * dxi[l];
#pragma unroll
        for (int k = 0; k < NK; ++k) {
          // node offsets from the base (x at compile time; y and z depend on the part) and
          // the node's weight and derivative per axis, evaluated at the offset itself
          const int o[3] = {k % 3, NK >= 9 ? (k / 3) % 3 : (D == 2 ? pl : pl % 3),
                            NK == 27 ? k / 9 : (NK == 9 ? pl : pl / 3)};
          double wv[3], dv[3];
#pragma unroll
          for (int l = 0; l < D; ++l) {
            const double t = xs[l] - (double)(base[l] + o[l] - 1);
            wv[l] = s2(t);
            dv[l] = s2d(t) * M.inv_h[l];
          }
          double S = 1.0, dS[D];
          for (int l = 0; l < D; ++l) S *= wv[l];
          for (int j = 0; j < D; ++j) {
            dS[j] = 1.0;
            for (int l = 0; l < D; ++l) dS[j] *= l == j ? dv[l] : wv[l];
          }
          I0[k] += wq * S;
          for (int l = 0; l < D; ++l) {
            Ia[k][l] += wq * (1.0 - s) * dS[l];
            Ib[k][l] += wq * s * dS[l];
          }
        }
      }
      // Sorted particles: the lanes of a wave fall in a few groups that share their base
      // node (one to three in 2D, three or four in 3D at 20 particles per cell), and a
      // group whose part nodes lie in the window has all its entries summed over the wave
      // at once.  Lanes left over put each entry on their own.
      bool pend = has;
#pragma unroll 1
      for (int grp = 0; grp < 8; ++grp) {
        const uint64_t pm = __ballot(pend);
        if (pm == 0) break;
        const int lead = __ffsll((long long)pm) - 1;
        int bl[D];
        bool mine = pend;
        for (int l = 0; l < D; ++l) {
          bl[l] = __builtin_amdgcn_readlane(base[l] + sh[l], lead);
          mine = mine && base[l] + sh[l] == bl[l];
        }
        bool inwin = true;
#pragma unroll
        for (int k = 0; k < NK; ++k) {
          int node[D];
          for (int l = 0; l < D; ++l) node[l] = bl[l] + NodeWeights<D>::off(l, k + NK * pl) - 1;
          inwin = inwin && w.rel(node) >= 0;
        }
        if (!inwin) break;
        // entry e = k NV + f: I0_k g_f (f < D), then the A^n and A^{n+1} integrals
        w.template put_all<NK * NV>(
            [&](int e) -> double {
              const int k = e / NV, f = e % NV;
              if (!mine) return 0.0;
              if (f < D) return I0[k] * g[f];
              const int c = f < D + 3 ? f - D : f - D - 3;
              double v = 0.0;
              for (int l = 0; l < D; ++l) v += (f < D + 3 ? Ia[k][l] : Ib[k][l]) * g[D + c * D + l];
              return v;
            },
            [&](int e) -> int {
              const int k = e / NV, f = e % NV;
              int node[D];
              for (int l = 0; l < D; ++l) node[l] = bl[l] + NodeWeights<D>::off(l, k + NK * pl) - 1;
              return f * kWinNodes<D> + w.rel(node);
            },
            lane);
        pend = pend && !mine;
      }
      if (__ballot(pend) == 0) continue;
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        int node[D];
        for (int l = 0; l < D; ++l) node[l] = base[l] + NodeWeights<D>::off(l, k + NK * pl) - 1 + sh[l];
        const int r = w.rel(node);
        for (int l = 0; l < D; ++l) w.put_wave(l, r, node, pend ? I0[k] * g[l] : 0.0, lane);
        for (int c = 0; c < 3; ++c) {
          double va = 0.0, vb = 0.0;
          for (int l = 0; l < D; ++l) {
            va += Ia[k][l] * g[D + c * D + l];
            vb += Ib[k][l] * g[D + c * D + l];
          }
          w.put_wave(D + c, r, node, pend ? va : 0.0, lane);
          w.put_wave(D + 3 + c, r, node, pend ? vb : 0.0, lane);
        }
      }
    }
    sw.advance(xi0, dxi);
  }
  // the endpoint interpolants A^- (at x) and A^+ (at x + dt vbar)
#pragma unroll 1
  for (int e = 0; e < 2; ++e) {
    double xs[D], ge[3];
    int b[D];
    for (int l = 0; l < D; ++l) {
      xs[l] = xi0[l] + (e ? dxi[l] : 0.0);
      b[l] = (int)floor(xs[l] + 0.5);
    }
    for (int c = 0; c < 3; ++c) ge[c] = live ? (e ? g[4 * D + 3 + c] : g[4 * D + c]) : 0.0;
    if (__ballot(live) == 0) break;
    // the stencil weights per axis; entry e = 3 k + c holds S_k ge_c
    double ax[D][3];
    for (int l = 0; l < D; ++l)
      for (int o = 0; o < 3; ++o) ax[l][o] = s2(xs[l] - (double)(b[l] + o - 1));
    // the groups of lanes sharing their nearest node, as for the segments (in 3D the
    // 81 entries of a group cost more than putting each value on its own: measured)
    bool pend = live;
#pragma unroll 1
    for (int grp = 0; grp < (D < 3 ? 4 : 0); ++grp) {
      const uint64_t pm = __ballot(pend);
      if (pm == 0) break;
      const int lead = __ffsll((long long)pm) - 1;
      int bl[D], lo[D], hi[D];
      bool mine = pend;
      for (int l = 0; l < D; ++l) {
        bl[l] = __builtin_amdgcn_readlane(b[l] + sh[l], lead);
        mine = mine && b[l] + sh[l] == bl[l];
        lo[l] = bl[l] - 1;
        hi[l] = bl[l] + 1;
      }
      if (w.rel(lo) < 0 || w.rel(hi) < 0) break;
      w.template put_all<3 * kStencil<D>>(
          [&](int en) -> double {
            const int k = en / 3, c = en % 3;
            double S = 1.0;
            for (int l = 0; l < D; ++l) S *= ax[l][NodeWeights<D>::off(l, k)];
            return mine ? S * ge[c] : 0.0;
          },
          [&](int en) -> int {
            const int k = en / 3, c = en % 3;
            int node[D];
            for (int l = 0; l < D; ++l) node[l] = bl[l] + NodeWeights<D>::off(l, k) - 1;
            return ((e ? D + 3 : D) + c) * kWinNodes<D> + w.rel(node);
          },
          lane);
      pend = pend && !mine;
    }
    if (__ballot(pend) == 0) continue;
#pragma unroll 1
    for (int k = 0; k < kStencil<D>; ++k) {
      int node[D];
      double S = 1.0;
#pragma unroll
      for (int l = 0; l < D; ++l) {
        node[l] = b[l] + NodeWeights<D>::off(l, k) - 1;
        S *= s2(xs[l] - (double)node[l]);
        node[l] += sh[l];
      }
      const int r = w.rel(node);
      for (int c = 0; c < 3; ++c) w.put_wave((e ? D + 3 : D) + c, r, node, pend ? S * ge[c] : 0.0, lane);
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < NV * kWinNodes<D>; k += kBlock) {
    const unsigned long long H = sacc[2 * k], L = sacc[2 * k + 1];
    if (H | L) {
      const int f = k / kWinNodes<D>, rel = k % kWinNodes<D>;
      int gi = wrapi(swlo[0] + rel % kWinX<D>, M.n[0]);
      if (D > 1) gi += M.n[0] * wrapi(swlo[1] + (rel / kWinX<D>) % kWinY<D>, M.n[1]);
      if (D > 2) gi += M.n[0] * M.n[1] * wrapi(swlo[2] + rel / (kWinX<D> * kWinY<D>), M.n[2]);
      unsigned long long* dst = a.acc + 2 * ((int64_t)f * M.Ng + gi);
      if (H) atomicAdd(dst, H);
      if (L) atomicAdd(dst + 1, L);
    }
  }
}

}  // namespace

// ---- mesh side ---------------------------------------------------------------------

namespace {
__device__ __forceinline__ double2 cadd2(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csc(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// i k * a
__device__ __forceinline__ double2 cik2(double k, double2 a) { return make_double2(-k * a.y, k * a.x); }

__device__ __forceinline__ void wavevec(const Mesh& M, int64_t g, double k[3], bool& nyq) {
  int64_t idx[3] = {g & (M.n[0] - 1), (g >> M.ln[0]) & (M.n[1] - 1), g >> (M.ln[0] + M.ln[1])};
  nyq = false;
  for (int l = 0; l < 3; ++l) {
    k[l] = 0.0;
    if (l >= M.d) continue;
    const int n = M.n[l];
    if (idx[l] == n / 2) {
      nyq = true;
      continue;
    }
    const int64_t ms = idx[l] <= n / 2 ? idx[l] : idx[l] - n;
    k[l] = M.kf[l] * (double)ms;
  }
}
}  // namespace


// Conjugate transpose, mode by mode, of the field step of Algorithm 1: projection of the
// trial current, continuity rho' = rho - dt i k.jh, the CN pairs
//   phi' = (c1 phi + dt psi + e1 (rho + rho')) / .. , psi' = 2 (phi' - phi) / dt - psi,
//   A'   = c1 A + c2 U + e2 jh,                       U'   = 2 (A' - A) / dt - U,
// and the trial fields i k (phi + phi') / 2, A, A'.  Real coefficients stay; i k becomes -i k.
__global__ __launch_bounds__(kBlock) void k_adj_field(AdjFieldArgs a) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const Mesh& M = a.M;
  const int64_t Ng = M.Ng;
  if (g >= Ng) return;
  const int d = M.d;
  double k[3];
  bool nyq;
  wavevec(M, g, k, nyq);
  const double h = a.dt;
  const double av = a.kappa2 * (k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
  const double q4 = 0.25 * h * h * av, den = 1.0 + q4;
  const double c1 = (1.0 - q4) / den, c2 = h / den;
  const double e1 = 0.25 * h * h * a.kappa2 * a.sigma1 / den, e2 = 0.5 * h * h * a.kappa2 * a.sigma2 / den;
  const double2 z = make_double2(0.0, 0.0);
  double2 phb1 = a.Lf[g], psb1 = a.Lf[Ng + g], rhb1 = a.Lf[2 * Ng + g];
  double2 Ab1[3], Ub1[3], Ab[3] = {z, z, z}, Ub[3] = {z, z, z}, jb[3] = {z, z, z};
  for (int c = 0; c < 3; ++c) {
    Ab1[c] = a.Lf[(3 + c) * Ng + g];
    Ub1[c] = a.Lf[(6 + c) * Ng + g];
  }
  double2 phb = z, psb = z, rhb = z;
  if (a.Pb) {  // trial fields
    for (int l = 0; l < d; ++l) {
      const double2 t = csc(cik2(-k[l], a.Pb[l * Ng + g]), 0.5);
      phb = cadd2(phb, t);
      phb1 = cadd2(phb1, t);
    }
    for (int c = 0; c < 3; ++c) {
      Ab[c] = cadd2(Ab[c], a.Pb[(d + c) * Ng + g]);
      Ab1[c] = cadd2(Ab1[c], a.Pb[(d + 3 + c) * Ng + g]);
    }
  }
  for (int c = 0; c < 3; ++c) {  // U' = 2 (A' - A) / h - U
    Ab1[c] = cadd2(Ab1[c], csc(Ub1[c], 2.0 / h));
    Ab[c] = cadd2(Ab[c], csc(Ub1[c], -2.0 / h));
    Ub[c] = cadd2(Ub[c], csc(Ub1[c], -1.0));
  }
  for (int c = 0; c < 3; ++c) {  // A' = c1 A + c2 U + e2 jh
    Ab[c] = cadd2(Ab[c], csc(Ab1[c], c1));
    Ub[c] = cadd2(Ub[c], csc(Ab1[c], c2));
    jb[c] = cadd2(jb[c], csc(Ab1[c], e2));
  }
  // psi' = 2 (phi' - phi) / h - psi
  phb1 = cadd2(phb1, csc(psb1, 2.0 / h));
  phb = cadd2(phb, csc(psb1, -2.0 / h));
  psb = cadd2(psb, csc(psb1, -1.0));
  // phi' = c1 phi + c2 psi + e1 (rho + rho')
  phb = cadd2(phb, csc(phb1, c1));
  psb = cadd2(psb, csc(phb1, c2));
  rhb = cadd2(rhb, csc(phb1, e1));
  rhb1 = cadd2(rhb1, csc(phb1, e1));
  // rho' = rho - h i k . jh
  rhb = cadd2(rhb, rhb1);
  for (int l = 0; l < d; ++l) jb[l] = cadd2(jb[l], csc(cik2(k[l], rhb1), h));
  // jh = P j
  if (a.project && nyq)
    for (int c = 0; c < 3; ++c) jb[c] = z;
  a.Ls[g] = phb;
  a.Ls[Ng + g] = psb;
  a.Ls[2 * Ng + g] = rhb;
  for (int c = 0; c < 3; ++c) {
    a.Ls[(3 + c) * Ng + g] = Ab[c];
    a.Ls[(6 + c) * Ng + g] = Ub[c];
    a.Lj[c * Ng + g] = jb[c];
  }
}

// Spectra of the cotangent of the field energy W = sum (|E|^2 / (2 sigma1) + |B|^2 /
// (2 sigma2)) dV with respect to the real-space state (phi, psi, rho, A, U):
// E = -i k phi - U, B = i k x A; phi-bar = (dV / sigma1) i k . E, U-bar = -(dV / sigma1) E,
// A-bar = (dV / sigma2) i k x B.
__global__ __launch_bounds__(kBlock) void k_energy_grad(Mesh M, double sigma1, double sigma2, const double2* S,
                                                        double2* out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t Ng = M.Ng;
  if (g >= Ng) return;
  double k[3];
  bool nyq;
  wavevec(M, g, k, nyq);
  const double2 ph = S[g];
  double2 E[3], A[3], B[3];
  for (int c = 0; c < 3; ++c) {
    const double2 gk = cik2(k[c], ph), U = S[(6 + c) * Ng + g];
    E[c] = make_double2(-gk.x - U.x, -gk.y - U.y);
    A[c] = S[(3 + c) * Ng + g];
  }
  for (int c = 0; c < 3; ++c) {
    const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
    const double2 a1 = cik2(k[c1], A[c2]), a2 = cik2(k[c2], A[c1]);
    B[c] = make_double2(a1.x - a2.x, a1.y - a2.y);
  }
  const double fe = M.dV / sigma1, fb = M.dV / sigma2;
  double2 phb = make_double2(0.0, 0.0);
  for (int c = 0; c < 3; ++c) phb = cadd2(phb, cik2(k[c], E[c]));
  out[g] = csc(phb, fe);
  out[Ng + g] = make_double2(0.0, 0.0);
  out[2 * Ng + g] = make_double2(0.0, 0.0);
  for (int c = 0; c < 3; ++c) {
    const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
    const double2 a1 = cik2(k[c1], B[c2]), a2 = cik2(k[c2], B[c1]);
    out[(3 + c) * Ng + g] = csc(make_double2(a1.x - a2.x, a1.y - a2.y), fb);
    out[(6 + c) * Ng + g] = csc(E[c], -fe);
  }
}

// Spectrum of the cotangent of the deposited point-shape charge at initialization:
// rho^0 = P (deposit) with the mean removed, phi^0 = sigma1 rho^0 / |k|^2 (+ terms free of
// the particles); so rho-bar_total = rho-bar + sigma1 phi-bar / |k|^2, zero at k = 0 and
// (projected) on the Nyquist planes.
__global__ __launch_bounds__(kBlock) void k_adj_init_field(Mesh M, double sigma1, int project, const double2* L,
                                                           double2* out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t Ng = M.Ng;
  if (g >= Ng) return;
  double k[3];
  bool nyq;
  wavevec(M, g, k, nyq);
  const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  double2 r = L[2 * Ng + g];
  if (k2 > 0.0) r = cadd2(r, csc(L[g], sigma1 / k2));
  if (g == 0 || (project && nyq)) r = make_double2(0.0, 0.0);
  out[g] = r;
}


// Per particle: x -> rho^0 (point shape), u -> P^0 = m kappa u + q A^0(x), q -> both
// (with m = |q|).
template <int D>
__global__ __launch_bounds__(kBlock) void k_adj_init_particle(AdjInitArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.np) return;
  const Mesh& M = a.M;
  const int64_t Ng = M.Ng;
  const int64_t li = a.id[i];
  const double q = a.q[i], m = fabs(q), mk = m * a.kappa;
  double xs[D];
  for (int l = 0; l < D; ++l) xs[l] = (a.x[l * a.ps + i] - M.lo[l]) * M.inv_h[l];
  NodeWeights<D> nw;
  nw.at(M, xs);
  double rS = 0.0, rS1[D], A[3] = {0.0, 0.0, 0.0}, A1[3][D];
  for (int j = 0; j < D; ++j) {
    rS1[j] = 0.0;
    for (int c = 0; c < 3; ++c) A1[c][j] = 0.0;
  }
  #pragma unroll
  for (int k = 0; k < kStencil<D>; ++k) {
    double S, dS[D], ddS[D][D];
    nw.vals(k, S, dS, ddS);
    const int g = nw.node(M, k);
    rS += S * a.rb[g];
    for (int j = 0; j < D; ++j) rS1[j] += dS[j] * a.rb[g];
    for (int c = 0; c < 3; ++c) {
      A[c] += S * a.A0[c * Ng + g];
      for (int j = 0; j < D; ++j) A1[c][j] += dS[j] * a.A0[c * Ng + g];
    }
  }
  double lP[3], u[3];
  for (int c = 0; c < 3; ++c) {
    lP[c] = a.lP[c * a.np + li];
    u[c] = (a.P[c * a.ps + i] - q * A[c]) / mk;
  }
  for (int j = 0; j < D; ++j) {
    double pa = 0.0;
    for (int c = 0; c < 3; ++c) pa += lP[c] * A1[c][j];
    a.gx[j * a.np + li] = a.lx[j * a.np + li] + q / M.dV * rS1[j] + q * pa;
  }
  for (int c = 0; c < 3; ++c) a.gu[c * a.np + li] = mk * lP[c];
  a.gq[li] = rS / M.dV + dot3(lP, A) + (q < 0.0 ? -1.0 : 1.0) * a.kappa * dot3(lP, u);
}

// Settle test of the adjoint current: out[0] = max |new - old|, out[1] = max |new| over
// n values (one workgroup), and old <- old + beta (new - old).
__global__ __launch_bounds__(kBlock) void k_adj_update(double* mu, const double* mnew, int64_t n, double beta,
                                                       unsigned long long* out) {
  // mu += beta (mnew - mu), and max |mnew - mu| and max |mnew| into out[0], out[1]: each
  // block reduces its share, then an integer atomic max of the bit patterns (non-negative
  // doubles order as their bits; a maximum does not depend on the order of arrival)
  __shared__ double r0[kBlock], r1[kBlock];
  double dm = 0.0, mm = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const double d = mnew[i] - mu[i];
    dm = fmax(dm, fabs(d));
    mm = fmax(mm, fabs(mnew[i]));
    mu[i] += beta * d;
  }
  r0[threadIdx.x] = dm;
  r1[threadIdx.x] = mm;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      r0[threadIdx.x] = fmax(r0[threadIdx.x], r0[threadIdx.x + w]);
      r1[threadIdx.x] = fmax(r1[threadIdx.x], r1[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    atomicMax(out, (unsigned long long)__double_as_longlong(r0[0]));
    atomicMax(out + 1, (unsigned long long)__double_as_longlong(r1[0]));
  }
}
__global__ void k_adj_update_init(unsigned long long* out) {
  if (threadIdx.x < 2) out[threadIdx.x] = 0ull;
}

// fix_scale on the device, so the scatter needs no round trip to the host: the exponent
// ceil(log2 B) from frexp (B = m 2^e with m in [1/2, 1)), exact for every B.
__global__ void k_adj_scale(const double* bound, double* fx) {
  if (threadIdx.x != 0) return;
  double B = bound[0];
  if (!(B > 0.0) || !isfinite(B)) B = 1.0;
  int e = 0;
  const double m = frexp(B, &e);
  const int eb = m == 0.5 ? e - 1 : e;
  const int sc = kFixK + 61 - eb;  // B 2^(sc-K) <= 2^61
  fx[0] = ldexp(1.0, sc - kFixK);
  fx[1] = ldexp(1.0, kFixK - sc);
  fx[2] = ldexp(1.0, -sc);
}
__global__ __launch_bounds__(kBlock) void k_adj_fix_to_double(const unsigned long long* acc, double* out, int64_t n,
                                                              const double* fx) {
  const double hi = fx[1], lo = fx[2];
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    out[i] = fix_value(acc, i, hi, lo);
}

// Fixed-order sum of n per-block values (one workgroup).
__global__ __launch_bounds__(kBlock) void k_adj_sum(const double* p, int64_t n, double* out) {
  __shared__ double r[kBlock];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += kBlock) s += p[i];
  r[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) r[threadIdx.x] += r[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = r[0];
}

namespace {
inline unsigned nblocks(int64_t n) { return (unsigned)std::max<int64_t>((n + kBlock - 1) / kBlock, 1); }
}  // namespace

template <int D>
void launch_adj_particle_d(const AdjArgs& a, hipStream_t s) {
  if (a.mode == ADJ_FINAL)
    hipLaunchKernelGGL((k_adj_particle<D, true>), dim3(nblocks(a.np)), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_adj_particle<D, false>), dim3(nblocks(a.np)), dim3(kBlock), 0, s, a);
}
hipError_t launch_adj_particle(const AdjArgs& a, hipStream_t s) {
  if (a.np == 0) return hipSuccess;
  if (a.mode != ADJ_PREP && a.mode != ADJ_FINAL) return hipErrorInvalidValue;
  if (a.M.d == 1)
    launch_adj_particle_d<1>(a, s);
  else if (a.M.d == 2)
    launch_adj_particle_d<2>(a, s);
  else
    launch_adj_particle_d<3>(a, s);
  return hipGetLastError();
}
template <int D>
void launch_adj_iter_d(const AdjArgs& a, hipStream_t s) {
  if (a.mode == ADJ_SCATTER)
    hipLaunchKernelGGL((k_adj_iter<D, true>), dim3(nblocks(a.np)), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_adj_iter<D, false>), dim3(nblocks(a.np)), dim3(kBlock), 0, s, a);
}
hipError_t launch_adj_iter(const AdjArgs& a, hipStream_t s) {
  if (a.np == 0) return hipSuccess;
  if (a.mode != ADJ_BOUND && a.mode != ADJ_SCATTER) return hipErrorInvalidValue;
  if (a.M.d == 1)
    launch_adj_iter_d<1>(a, s);
  else if (a.M.d == 2)
    launch_adj_iter_d<2>(a, s);
  else
    launch_adj_iter_d<3>(a, s);
  return hipGetLastError();
}
int64_t adj_particle_blocks(int64_t np) { return nblocks(np); }
hipError_t launch_adj_field(const AdjFieldArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_field, dim3(nblocks(a.M.Ng)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_energy_grad(const Mesh& M, double sigma1, double sigma2, const double2* S, double2* out,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_energy_grad, dim3(nblocks(M.Ng)), dim3(kBlock), 0, s, M, sigma1, sigma2, S, out);
  return hipGetLastError();
}
hipError_t launch_adj_init_field(const Mesh& M, double sigma1, int project, const double2* L, double2* out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(k_adj_init_field, dim3(nblocks(M.Ng)), dim3(kBlock), 0, s, M, sigma1, project, L, out);
  return hipGetLastError();
}
hipError_t launch_adj_init_particle(const AdjInitArgs& a, hipStream_t s) {
  if (a.np == 0) return hipSuccess;
  if (a.M.d == 1)
    hipLaunchKernelGGL(k_adj_init_particle<1>, dim3(nblocks(a.np)), dim3(kBlock), 0, s, a);
  else if (a.M.d == 2)
    hipLaunchKernelGGL(k_adj_init_particle<2>, dim3(nblocks(a.np)), dim3(kBlock), 0, s, a);
  else
    hipLaunchKernelGGL(k_adj_init_particle<3>, dim3(nblocks(a.np)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}
hipError_t launch_adj_update(double* mu, const double* mnew, int64_t n, double beta, double* out, hipStream_t s) {
  unsigned long long* o = reinterpret_cast<unsigned long long*>(out);
  hipLaunchKernelGGL(k_adj_update_init, dim3(1), dim3(64), 0, s, o);
  const unsigned blocks = (unsigned)std::min<int64_t>((n + kBlock - 1) / kBlock, 512);
  hipLaunchKernelGGL(k_adj_update, dim3(std::max(blocks, 1u)), dim3(kBlock), 0, s, mu, mnew, n, beta, o);
  return hipGetLastError();
}
hipError_t launch_adj_scale(const double* bound, double* fx, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_scale, dim3(1), dim3(64), 0, s, bound, fx);
  return hipGetLastError();
}
hipError_t launch_adj_fix_to_double(const unsigned long long* acc, double* out, int64_t n, const double* fx,
                                    hipStream_t s) {
  const unsigned blocks = (unsigned)std::max<int64_t>(std::min<int64_t>((n + kBlock - 1) / kBlock, 4096), 1);
  hipLaunchKernelGGL(k_adj_fix_to_double, dim3(blocks), dim3(kBlock), 0, s, acc, out, n, fx);
  return hipGetLastError();
}
hipError_t launch_adj_sum(const double* p, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_sum, dim3(1), dim3(kBlock), 0, s, p, n, out);
  return hipGetLastError();
}

}  // namespace gmhc
