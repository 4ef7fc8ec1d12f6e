// orbit.hip -- the orbit pass: one thread per particle runs the inner Picard loop of
// the GM-HC orbit evaluation at frozen trial fields and deposits the orbit current.
//
// Per evaluation v_out = F(v_in) (sections "Symmetric orbit-averaged maps",
// "Orbit-averaged discrete chain rule", "No-explicit-A_t GM-HC step",
// "Mechanical split and magnetic zero work"):
//   1. straight unwrapped orbit x(s) = x^n + s dt v_in, split at the knots of the
//      quadratic B-spline (half-integer node offsets), Gauss-Legendre on each piece;
//   2. orbit gathers: grad phi-bar = int sum_g (grad_h phi^{n+1/2})_g S_g ds and the
//      orbit discrete gradient D_lj = int sum_g ((1-s) A^n + s A^{n+1})_{l,g} d_j S_g ds;
//   3. endpoint interpolants A^- = A_h^n(x^n), A^+ = A_h^{n+1}(x^n + dt v_in);
//   4. p^- = P^n - q A_ep - (q dt/2) grad-phi-bar + (q dt/2) D v_in, HC rotation with
//      B_eff = axial vector of K = D^T - D, P^{n+1} = p^+ + q A_ep + the same kick;
//   5. v_out = average of the secant velocities V^dg(p^-, p^n) and V^dg(p^{n+1}, p^+).
// After the inner test passes, a second sweep over the same orbit deposits
// J_g += q v_out S-bar_g / dV and gathers U-bar for the diagnostics.
//
// Memory layout on chip.  Particles arrive sorted by cell, so a workgroup's
// particles sit in a small box of cells.  Each workgroup stages the mesh fields of
// that box plus a halo of two nodes (stencil reach one node, orbit travel below one
// cell) in LDS, and accumulates its current deposit in an LDS tile of the same box,
// flushed to HBM with one atomic per tile node and component.  Orbits whose stencil
// leaves the tile, and workgroups whose box does not fit, read and deposit through
// global memory instead.
#include <limits.h>
#include <math.h>

#include "gmhc_internal.h"

namespace gmhc {
namespace {

constexpr int kHalo = 2;               // tile halo in nodes
constexpr int kTileBytes = 40 * 1024;  // LDS per workgroup for the field and current tiles

__device__ __forceinline__ int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Quadratic B-spline weights of nodes j-1, j, j+1 at offset f = xi - j in [-1/2, 1/2]
// and their x-derivatives (inverse spacing ih).
__device__ __forceinline__ void bw(double f, double w[3]) {
  const double a = 0.5 - f, b = 0.5 + f;
  w[0] = 0.5 * a * a;
  w[1] = 0.75 - f * f;
  w[2] = 0.5 * b * b;
}
__device__ __forceinline__ void bdw(double f, double ih, double dw[3]) {
  dw[0] = (f - 0.5) * ih;
  dw[1] = -2.0 * f * ih;
  dw[2] = (0.5 + f) * ih;
}

// Weight and x-derivative of the single node c (0, 1, 2 for j-1, j, j+1) at offset f.
__device__ __forceinline__ double bw1(double f, int c) {
  const double a = 0.5 - f, b = 0.5 + f;
  return c == 0 ? 0.5 * a * a : (c == 1 ? 0.75 - f * f : 0.5 * b * b);
}
__device__ __forceinline__ double bdw1(double f, int c) { return c == 0 ? f - 0.5 : (c == 1 ? -2.0 * f : 0.5 + f); }

// Workgroup tile: box of unwrapped node coordinates [o, o + E) per axis (uniform).
struct Tile {
  int o[3];
  int E[3];
  int nodes;
  int ok;  // 1: fields staged in LDS
};

// Fields of the staged tile: 0..D-1 grad phi, D..D+2 A^n, D+3..D+5 A^{n+1},
// D+6..D+8 U^{n+1/2}; the current tile (3 components) follows the fields.
template <int D>
__device__ __forceinline__ constexpr int nfields() { return D + 9; }

template <int D>
__device__ __forceinline__ const double* gfield(const OrbitArgs& a, int f) {
  const int64_t Ng = a.M.Ng;
  if (f < D) return a.trial + (int64_t)f * Ng;
  if (f < D + 3) return a.An + (int64_t)(f - D) * Ng;
  return a.trial + (int64_t)(f - 3) * Ng;
}

// Node-index addressing of one 3^D stencil, either into the LDS tile or into HBM.
template <int D, bool LDS>
struct Stencil {
  int ix[3], iy[3], iz[3];  // per-axis contributions, summed per node
  __device__ __forceinline__ void set(const Mesh& M, const Tile& t, const int jn[3]) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (LDS) {
        ix[c] = jn[0] + c - 1 - t.o[0];
        iy[c] = D > 1 ? t.E[0] * (jn[1] + c - 1 - t.o[1]) : 0;
        iz[c] = D > 2 ? t.E[0] * t.E[1] * (jn[2] + c - 1 - t.o[2]) : 0;
      } else {
        ix[c] = wrapi(jn[0] + c - 1, M.n[0]);
        iy[c] = D > 1 ? M.n[0] * wrapi(jn[1] + c - 1, M.n[1]) : 0;
        iz[c] = D > 2 ? M.n[0] * M.n[1] * wrapi(jn[2] + c - 1, M.n[2]) : 0;
      }
    }
  }
  __device__ __forceinline__ int node(int cx, int cy, int cz) const { return ix[cx] + iy[cy] + iz[cz]; }
  // offset of stencil row (cy, cz) computed directly (no indexing by a loop variable)
  __device__ __forceinline__ int row(const Mesh& M, const Tile& t, const int jn[3], int cy, int cz) const {
    if (LDS)
      return (D > 1 ? t.E[0] * (jn[1] + cy - 1 - t.o[1]) : 0) +
             (D > 2 ? t.E[0] * t.E[1] * (jn[2] + cz - 1 - t.o[2]) : 0);
    return (D > 1 ? M.n[0] * wrapi(jn[1] + cy - 1, M.n[1]) : 0) +
           (D > 2 ? M.n[0] * M.n[1] * wrapi(jn[2] + cz - 1, M.n[2]) : 0);
  }
};

template <int D, bool LDS>
__device__ __forceinline__ double ld(const OrbitArgs& a, const Tile& t, int f, int node) {
  if (LDS) {
    HIP_DYNAMIC_SHARED(double, s_tile);
    return s_tile[f * t.nodes + node];
  } else {
    return gfield<D>(a, f)[node];
  }
}

template <int D>
__device__ __forceinline__ bool inside(const Tile& t, const int jn[3]) {
  bool r = t.ok != 0;
#pragma unroll
  for (int l = 0; l < D; ++l) r = r && (jn[l] - 1 >= t.o[l]) && (jn[l] + 1 < t.o[l] + t.E[l]);
  return r;
}

// Visit the knot-split segments [sa, sb] of the orbit xi(s) = xi0 + s dxi, s in [0,1].
// Crossings of all axes are merged on the fly (each axis' crossings are monotone in s).
template <int D, class F>
__device__ __forceinline__ void for_each_segment(const double* xi0, const double* dxi, F&& f) {
  double knot[3], next[3], stp[3];
#pragma unroll
  for (int l = 0; l < D; ++l) {
    if (dxi[l] > 0.0) {
      knot[l] = floor(xi0[l] - 0.5) + 1.5;
      stp[l] = 1.0;
      next[l] = (knot[l] - xi0[l]) / dxi[l];
    } else if (dxi[l] < 0.0) {
      knot[l] = ceil(xi0[l] - 0.5) - 0.5;
      stp[l] = -1.0;
      next[l] = (knot[l] - xi0[l]) / dxi[l];
    } else {
      knot[l] = 0.0;
      stp[l] = 0.0;
      next[l] = 2.0;
    }
  }
  double sa = 0.0;
#pragma unroll 1
  for (int it = 0; it <= D * kMaxCross; ++it) {
    double sb = 1.0;
#pragma unroll
    for (int l = 0; l < D; ++l) sb = (next[l] < sb) ? next[l] : sb;
    if (sb > sa) f(sa, sb);
    if (sb >= 1.0) break;
#pragma unroll
    for (int l = 0; l < D; ++l)
      if (next[l] == sb) {
        knot[l] += stp[l];
        next[l] = (knot[l] - xi0[l]) / dxi[l];
      }
    sa = sb;
  }
}

template <int D>
__device__ __forceinline__ void nearest(const double* xi, int jn[3]) {
#pragma unroll
  for (int l = 0; l < 3; ++l) jn[l] = (l < D) ? (int)floor(xi[l] + 0.5) : 0;
}

// Point interpolant sum_g F_g S_g(x) of A (field base fb = D: A^n, D+3: A^{n+1}).
template <int D, bool LDS>
__device__ __forceinline__ void interp3_at(const OrbitArgs& a, const Tile& t, int fb, const double* xi,
                                           const int jn[3], double out[3]) {
  double w[3][3];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if (l < D)
      bw(xi[l] - (double)jn[l], w[l]);
    else
      w[l][0] = 1.0;
  }
  Stencil<D, LDS> st;
  st.set(a.M, t, jn);
  out[0] = out[1] = out[2] = 0.0;
  constexpr int NY = D > 1 ? 3 : 1, NZ = D > 2 ? 3 : 1;
#pragma unroll
  for (int cz = 0; cz < NZ; ++cz)
#pragma unroll
    for (int cy = 0; cy < NY; ++cy) {
      const double wyz = w[1][cy] * w[2][cz];
#pragma unroll
      for (int cx = 0; cx < 3; ++cx) {
        const double S = w[0][cx] * wyz;
        const int g = st.node(cx, cy, cz);
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] += S * ld<D, LDS>(a, t, fb + c, g);
      }
    }
}

template <int D>
__device__ __forceinline__ void interp3(const OrbitArgs& a, const Tile& t, int fb, const double* xi,
                                        double out[3]) {
  int jn[3];
  nearest<D>(xi, jn);
  if (inside<D>(t, jn))
    interp3_at<D, true>(a, t, fb, xi, jn, out);
  else
    interp3_at<D, false>(a, t, fb, xi, jn, out);
}

// Quadrature of one knot segment for the gathers grad-phi-bar and D.
//
// The integrated weights of the stencil nodes of one x-row (fixed y, z offset) are
// accumulated over the Gauss points first,
//   S-bar_g = sum_q w_q S_g,  Xa_g = sum_q w_q (1-s_q) d_x S_g,  Xb_g = sum_q w_q s_q d_x S_g
// (likewise Ya, Yb for d_y and Za, Zb for d_z), then contracted once with the node
// values: grad-phi-bar += S-bar_g (grad phi)_g, D_l. += Xa_g A^n_{l,g} + Xb_g A^{n+1}_{l,g}.
// This is the same quadrature summed in a different order: each field value is read
// once per segment instead of once per Gauss point, and only one row of accumulators
// is live at a time.
template <int D, bool LDS>
__device__ __forceinline__ void eval_segment(const OrbitArgs& a, const Tile& t, const double* xi0,
                                             const double* dxi, const int jn[3], double sa, double sb,
                                             double gp[3], double Dm[3][3]) {
  const Mesh& M = a.M;
  const double len = sb - sa;
  Stencil<D, LDS> st;
  st.set(M, t, jn);
  constexpr int NR = (D > 1 ? 3 : 1) * (D > 2 ? 3 : 1);  // stencil rows
#pragma unroll 1
  for (int r = 0; r < NR; ++r) {
    const int cy = D > 1 ? r % 3 : 0, cz = D > 2 ? r / 3 : 0;
    double Sb[3] = {0, 0, 0}, Xa[3] = {0, 0, 0}, Xb[3] = {0, 0, 0};
    double Ya[3] = {0, 0, 0}, Yb[3] = {0, 0, 0}, Za[3] = {0, 0, 0}, Zb[3] = {0, 0, 0};
#pragma unroll 1
    for (int qp = 0; qp < a.ngl; ++qp) {
      const double s = sa + len * a.glx[qp];
      const double wq = len * a.glw[qp];
      const double al = wq * (1.0 - s), be = wq * s;
      double wx[3], dwx[3];
      const double fx = xi0[0] + s * dxi[0] - (double)jn[0];
      bw(fx, wx);
      bdw(fx, M.inv_h[0], dwx);
      // this row's node weight and derivative along the other axes
      double wy = 1.0, dwy = 0.0, wz = 1.0, dwz = 0.0;
      if (D > 1) {
        const double fy = xi0[1] + s * dxi[1] - (double)jn[1];
        wy = bw1(fy, cy);
        dwy = bdw1(fy, cy) * M.inv_h[1];
      }
      if (D > 2) {
        const double fz = xi0[2] + s * dxi[2] - (double)jn[2];
        wz = bw1(fz, cz);
        dwz = bdw1(fz, cz) * M.inv_h[2];
      }
      const double wyz = wy * wz;
      const double sq = wq * wyz, xa = al * wyz, xb = be * wyz;
      const double ya = al * dwy * wz, yb = be * dwy * wz;
      const double za = al * wy * dwz, zb = be * wy * dwz;
#pragma unroll
      for (int cx = 0; cx < 3; ++cx) {
        Sb[cx] += wx[cx] * sq;
        Xa[cx] += dwx[cx] * xa;
        Xb[cx] += dwx[cx] * xb;
        if (D > 1) {
          Ya[cx] += wx[cx] * ya;
          Yb[cx] += wx[cx] * yb;
        }
        if (D > 2) {
          Za[cx] += wx[cx] * za;
          Zb[cx] += wx[cx] * zb;
        }
      }
    }
    const int rowoff = st.row(M, t, jn, cy, cz);
#pragma unroll
    for (int cx = 0; cx < 3; ++cx) {
      const int g = st.ix[cx] + rowoff;
#pragma unroll
      for (int l = 0; l < D; ++l) gp[l] += Sb[cx] * ld<D, LDS>(a, t, l, g);
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const double a0 = ld<D, LDS>(a, t, D + l, g), a1 = ld<D, LDS>(a, t, D + 3 + l, g);
        Dm[l][0] += Xa[cx] * a0 + Xb[cx] * a1;
        if (D > 1) Dm[l][1] += Ya[cx] * a0 + Yb[cx] * a1;
        if (D > 2) Dm[l][2] += Za[cx] * a0 + Zb[cx] * a1;
      }
    }
  }
}

struct EvalOut {
  double vout[3];
  double Pn1[3];
  double pn1[3];
  double Ap[3];
  double gp[3];
  double Dm[3][3];
  int nseg;
};

__device__ __forceinline__ double gam(const double p[3], double inv_mk) {
  const double ux = p[0] * inv_mk, uy = p[1] * inv_mk, uz = p[2] * inv_mk;
  return sqrt(1.0 + ux * ux + uy * uy + uz * uz);
}

// One orbit evaluation of one particle.
template <int D>
__device__ void evaluate(const OrbitArgs& a, const Tile& t, const double* xi0, const double P[3], double q,
                         double m, const double Am[3], const double vin[3], EvalOut& o) {
  const Mesh& M = a.M;
  double dxi[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int l = 0; l < D; ++l) dxi[l] = a.dt * vin[l] * M.inv_h[l];
  double gp[3] = {0.0, 0.0, 0.0};
  double Dm[3][3];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int j = 0; j < 3; ++j) Dm[l][j] = 0.0;
  int nseg = 0;
  for_each_segment<D>(xi0, dxi, [&](double sa, double sb) {
    ++nseg;
    const double sm = 0.5 * (sa + sb);
    double xm[3];
#pragma unroll
    for (int l = 0; l < D; ++l) xm[l] = xi0[l] + sm * dxi[l];
    int jn[3];
    nearest<D>(xm, jn);
    if (inside<D>(t, jn))
      eval_segment<D, true>(a, t, xi0, dxi, jn, sa, sb, gp, Dm);
    else
      eval_segment<D, false>(a, t, xi0, dxi, jn, sa, sb, gp, Dm);
  });

  // endpoint interpolant A^+ = A_h^{n+1}(x^n + dt v_in)
  double xie[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int l = 0; l < D; ++l) xie[l] = xi0[l] + dxi[l];
  double Ap[3];
  interp3<D>(a, t, D + 3, xie, Ap);

  const double dt = a.dt, kappa = a.kappa;
  double Aep[3], kick[3], pm[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    Aep[c] = 0.5 * (Am[c] + Ap[c]);
    double Dv = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) Dv += Dm[c][j] * vin[j];
    kick[c] = 0.5 * q * dt * (Dv - gp[c]);
    pm[c] = P[c] - q * Aep[c] + kick[c];
  }
  // B_eff of the skew part K = D^T - D (D zero-padded to 3x3): (K23, -K13, K12)
  const double Beff[3] = {Dm[2][1] - Dm[1][2], -(Dm[2][0] - Dm[0][2]), Dm[1][0] - Dm[0][1]};
  // normalized HC map
  const double inv_mk = 1.0 / (m * kappa);
  const double um[3] = {pm[0] * inv_mk, pm[1] * inv_mk, pm[2] * inv_mk};
  const double tc = q * dt / (2.0 * m);
  const double tau[3] = {tc * Beff[0], tc * Beff[1], tc * Beff[2]};
  const double gm2 = 1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2];
  const double tau2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];
  const double ut = um[0] * tau[0] + um[1] * tau[1] + um[2] * tau[2];
  const double sig = gm2 - tau2;
  const double X = tau2 + ut * ut;
  const double R = sqrt(sig * sig + 4.0 * X);
  const double g2 = (sig >= 0.0) ? 0.5 * (sig + R) : 2.0 * X / (R - sig);
  const double ig = 1.0 / sqrt(g2);
  const double tv[3] = {tau[0] * ig, tau[1] * ig, tau[2] * ig};
  const double t2 = tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2];
  const double sf = 2.0 / (1.0 + t2);
  const double sv[3] = {sf * tv[0], sf * tv[1], sf * tv[2]};
  const double us[3] = {um[0] + (um[1] * tv[2] - um[2] * tv[1]), um[1] + (um[2] * tv[0] - um[0] * tv[2]),
                        um[2] + (um[0] * tv[1] - um[1] * tv[0])};
  const double up[3] = {um[0] + (us[1] * sv[2] - us[2] * sv[1]), um[1] + (us[2] * sv[0] - us[0] * sv[2]),
                        um[2] + (us[0] * sv[1] - us[1] * sv[0])};
  const double mk = m * kappa;
  const double pp[3] = {mk * up[0], mk * up[1], mk * up[2]};
  double pn[3], Pn1[3], pn1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    Pn1[c] = pp[c] + q * Aep[c] + kick[c];
    pn[c] = P[c] - q * Am[c];
    pn1[c] = Pn1[c] - q * Ap[c];
  }
  // secant velocities and the orbit velocity
  const double gm_ = gam(pm, inv_mk), gn = gam(pn, inv_mk), gn1 = gam(pn1, inv_mk), gp_ = gam(pp, inv_mk);
  const double d1 = 1.0 / (m * (gm_ + gn)), d2 = 1.0 / (m * (gn1 + gp_));
  o.nseg = nseg;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    o.vout[c] = 0.5 * ((pm[c] + pn[c]) * d1 + (pn1[c] + pp[c]) * d2);
    o.Pn1[c] = Pn1[c];
    o.pn1[c] = pn1[c];
    o.Ap[c] = Ap[c];
    o.gp[c] = gp[c];
#pragma unroll
    for (int j = 0; j < 3; ++j) o.Dm[c][j] = Dm[c][j];
  }
}

// Deposit sweep of one segment, one stencil row at a time: S-bar over the row, U-bar
// gather, current deposit (LDS tile or HBM atomics).
template <int D, bool LDS>
__device__ __forceinline__ void deposit_segment(const OrbitArgs& a, const Tile& t, const double* xi0,
                                                const double* dxi, const int jn[3], double sa, double sb,
                                                const double coef[3], bool do_dep, double Ub[3]) {
  const double len = sb - sa;
  Stencil<D, LDS> st;
  st.set(a.M, t, jn);
  HIP_DYNAMIC_SHARED(double, s_tile);
  double* s_J = s_tile + nfields<D>() * t.nodes;
  constexpr int NR = (D > 1 ? 3 : 1) * (D > 2 ? 3 : 1);
#pragma unroll 1
  for (int r = 0; r < NR; ++r) {
    const int cy = D > 1 ? r % 3 : 0, cz = D > 2 ? r / 3 : 0;
    double acc[3] = {0.0, 0.0, 0.0};
#pragma unroll 1
    for (int qp = 0; qp < a.ngl; ++qp) {
      const double s = sa + len * a.glx[qp];
      const double wq = len * a.glw[qp];
      double wx[3];
      bw(xi0[0] + s * dxi[0] - (double)jn[0], wx);
      double wyz = wq;
      if (D > 1) wyz *= bw1(xi0[1] + s * dxi[1] - (double)jn[1], cy);
      if (D > 2) wyz *= bw1(xi0[2] + s * dxi[2] - (double)jn[2], cz);
#pragma unroll
      for (int cx = 0; cx < 3; ++cx) acc[cx] += wx[cx] * wyz;
    }
    const int rowoff = st.row(a.M, t, jn, cy, cz);
#pragma unroll
    for (int cx = 0; cx < 3; ++cx) {
      const int g = st.ix[cx] + rowoff;
      const double Sb = acc[cx];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        Ub[c] += Sb * ld<D, LDS>(a, t, D + 6 + c, g);
        if (do_dep) {
          if (LDS)
            atomicAdd(s_J + c * t.nodes + g, coef[c] * Sb);
          else
            atomicAdd(a.J + (int64_t)c * a.M.Ng + g, coef[c] * Sb);
        }
      }
    }
  }
}

// Deposit q v_out S-bar / dV along the orbit of v_in and gather U-bar.
template <int D>
__device__ void deposit_orbit(const OrbitArgs& a, const Tile& t, const double* xi0, const double vin[3],
                              const double coef[3], bool do_dep, double Ub[3]) {
  const Mesh& M = a.M;
  double dxi[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int l = 0; l < D; ++l) dxi[l] = a.dt * vin[l] * M.inv_h[l];
  Ub[0] = Ub[1] = Ub[2] = 0.0;
  for_each_segment<D>(xi0, dxi, [&](double sa, double sb) {
    const double sm = 0.5 * (sa + sb);
    double xm[3];
#pragma unroll
    for (int l = 0; l < D; ++l) xm[l] = xi0[l] + sm * dxi[l];
    int jn[3];
    nearest<D>(xm, jn);
    if (inside<D>(t, jn))
      deposit_segment<D, true>(a, t, xi0, dxi, jn, sa, sb, coef, do_dep, Ub);
    else
      deposit_segment<D, false>(a, t, xi0, dxi, jn, sa, sb, coef, do_dep, Ub);
  });
}

// Block-wide min / max of an int (all threads participate).
__device__ __forceinline__ void block_minmax(int& lo, int& hi, int* sh) {
  for (int off = 32; off > 0; off >>= 1) {
    lo = min(lo, __shfl_xor(lo, off, 64));
    hi = max(hi, __shfl_xor(hi, off, 64));
  }
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  __syncthreads();
  if (lane == 0) {
    sh[2 * wave] = lo;
    sh[2 * wave + 1] = hi;
  }
  __syncthreads();
  lo = sh[0];
  hi = sh[1];
  for (int w = 1; w < (int)(blockDim.x / 64); ++w) {
    lo = min(lo, sh[2 * w]);
    hi = max(hi, sh[2 * w + 1]);
  }
}

template <int D>
__device__ __forceinline__ int tile_to_global(const Mesh& M, const Tile& t, int nd) {
  const int ux = nd % t.E[0] + t.o[0];
  const int uy = D > 1 ? (nd / t.E[0]) % t.E[1] + t.o[1] : 0;
  const int uz = D > 2 ? nd / (t.E[0] * t.E[1]) + t.o[2] : 0;
  return wrapi(ux, M.n[0]) + M.n[0] * ((D > 1 ? wrapi(uy, M.n[1]) : 0) + M.n[1] * (D > 2 ? wrapi(uz, M.n[2]) : 0));
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_orbit(OrbitArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const Mesh& M = a.M;
  const int64_t ps = a.ps;
  HIP_DYNAMIC_SHARED(double, s_tile);
  __shared__ int s_mm[2 * (kBlock / 64)];
  constexpr int NF = nfields<D>();

  // ---- particle position and the workgroup's tile box
  double x[3] = {0.0, 0.0, 0.0}, xi0[3] = {0.0, 0.0, 0.0};
  bool valid = i < a.np;
  if (valid) {
#pragma unroll
    for (int l = 0; l < D; ++l) {
      x[l] = a.x[l * ps + i];
      xi0[l] = (x[l] - M.lo[l]) * M.inv_h[l];
      valid = valid && isfinite(xi0[l]) && fabs(xi0[l]) < 1.0e8;
    }
  }
  Tile t;
  int nodes = 1, ok = 1;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    t.o[l] = 0;
    t.E[l] = 1;
  }
#pragma unroll
  for (int l = 0; l < D; ++l) {
    int lo = valid ? (int)floor(xi0[l] + 0.5) : INT_MAX;
    int hi = valid ? (int)floor(xi0[l] + 0.5) : INT_MIN;
    block_minmax(lo, hi, s_mm);
    if (lo > hi) {  // no valid particle in this workgroup
      ok = 0;
    } else {
      t.o[l] = uni(lo - kHalo);
      const int e = hi - lo + 1 + 2 * kHalo;
      t.E[l] = uni(e);
      nodes = (e > 4096) ? (1 << 30) : nodes * e;
    }
  }
  if (ok && (int64_t)nodes * (NF + 3) * (int64_t)sizeof(double) > kTileBytes) ok = 0;
  t.nodes = uni(nodes);
  t.ok = uni(ok);
  if (t.ok) {
    // stage the fields and clear the current tile
    double* s_J = s_tile + NF * t.nodes;
    for (int k = threadIdx.x; k < NF * t.nodes; k += blockDim.x) {
      const int f = k / t.nodes, nd = k - f * t.nodes;
      s_tile[k] = gfield<D>(a, f)[tile_to_global<D>(M, t, nd)];
    }
    for (int k = threadIdx.x; k < 3 * t.nodes; k += blockDim.x) s_J[k] = 0.0;
  }
  __syncthreads();

  double part[kOrbitParts];
#pragma unroll
  for (int v = 0; v < kOrbitParts; ++v) part[v] = 0.0;
  if (i < a.np) {
    const double q = a.q[i];
    const double m = fabs(q);
    double vin[3] = {a.v[i], a.v[ps + i], a.v[2 * ps + i]};
    double Am[3] = {0.0, 0.0, 0.0};
    if (valid) interp3<D>(a, t, D, xi0, Am);
    int it = 0, segs = 0;
    bool conv = false;
    double kin = 0.0, work = 0.0, ra2 = 0.0;
    const int maxit = a.iterate ? a.max_inner : 1;
    for (it = 1; it <= maxit; ++it) {
      // the orbit must stay finite and within the supported knot-crossing range
      const double vnin = sqrt(vin[0] * vin[0] + vin[1] * vin[1] + vin[2] * vin[2]);
      bool okv = valid && isfinite(vnin);
#pragma unroll
      for (int l = 0; l < D; ++l) okv = okv && fabs(a.dt * vin[l] * M.inv_h[l]) < (double)(kMaxCross - 1);
      if (!okv) break;
      const double P[3] = {a.P[i], a.P[ps + i], a.P[2 * ps + i]};
      EvalOut o;
      evaluate<D>(a, t, xi0, P, q, m, Am, vin, o);
      segs += o.nseg;
      const double vn = sqrt(o.vout[0] * o.vout[0] + o.vout[1] * o.vout[1] + o.vout[2] * o.vout[2]);
      if (!isfinite(vn) || !(vn < a.kappa)) break;  // finite and subluminal
      double dmax = 0.0, vmax = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        dmax = fmax(dmax, fabs(o.vout[c] - vin[c]));
        vmax = fmax(vmax, fabs(o.vout[c]));
      }
      if (!a.iterate || dmax <= a.tol_abs + a.tol_rel * vmax) {
        // converged: deposit along the evaluated orbit, accept-pass diagnostics, store
        conv = true;
        double coef[3];
        const double qv = q / M.dV;
#pragma unroll
        for (int c = 0; c < 3; ++c) coef[c] = qv * o.vout[c];
        double Ub[3];
        deposit_orbit<D>(a, t, xi0, vin, coef, a.deposit != 0, Ub);
        double wk = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double Dv = 0.0;
#pragma unroll
          for (int j = 0; j < D; ++j) Dv += o.Dm[c][j] * vin[j];
          const double r = o.Ap[c] - Am[c] - a.dt * (Ub[c] + Dv);
          ra2 += r * r;
          wk += o.vout[c] * (-o.gp[c] - Ub[c]);
        }
        const double inv_mk = 1.0 / (m * a.kappa);
        const double p2 = o.pn1[0] * o.pn1[0] + o.pn1[1] * o.pn1[1] + o.pn1[2] * o.pn1[2];
        kin = p2 / (m * (gam(o.pn1, inv_mk) + 1.0));
        work = q * wk;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          a.v[c * ps + i] = o.vout[c];
          a.Pn[c * ps + i] = o.Pn1[c];
        }
#pragma unroll
        for (int l = 0; l < D; ++l) {
          double xv = x[l] + a.dt * vin[l];
          const double top = M.lo[l] + M.len[l];
          if (xv >= top) xv -= M.len[l];
          if (xv < M.lo[l]) xv += M.len[l];
          if (xv >= top) xv -= M.len[l];
          a.xn[l * ps + i] = xv;
        }
        break;
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) vin[c] = o.vout[c];
    }
    if (it > maxit) it = maxit;
    a.iters[i] = it;
    part[OP_FAIL] = conv ? 0.0 : 1.0;
    part[OP_ITERS] = (double)it;
    part[OP_ITMAX] = (double)it;
    part[OP_KIN] = kin;
    part[OP_WORK] = work;
    part[OP_RA2] = ra2;
    part[OP_SEGS] = (double)segs;
  }
  __syncthreads();
  // flush the current tile: one atomic per nonzero tile node and component
  if (t.ok && a.deposit) {
    const double* s_J = s_tile + NF * t.nodes;
    for (int k = threadIdx.x; k < 3 * t.nodes; k += blockDim.x) {
      const double v = s_J[k];
      if (v == 0.0) continue;
      const int c = k / t.nodes, nd = k - c * t.nodes;
      atomicAdd(a.J + (int64_t)c * M.Ng + tile_to_global<D>(M, t, nd), v);
    }
  }
  // block reduction in a fixed order: butterfly within each wave, then waves in order
#pragma unroll
  for (int v = 0; v < kOrbitParts; ++v) {
    for (int off = 32; off > 0; off >>= 1) {
      const double o2 = __shfl_xor(part[v], off, 64);
      part[v] = (v == OP_ITMAX) ? fmax(part[v], o2) : part[v] + o2;
    }
  }
  __shared__ double sh[kBlock / 64][kOrbitParts];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0)
#pragma unroll
    for (int v = 0; v < kOrbitParts; ++v) sh[wave][v] = part[v];
  __syncthreads();
  if (threadIdx.x < kOrbitParts) {
    const int v = threadIdx.x;
    double acc = sh[0][v];
    for (int w = 1; w < (int)(blockDim.x / 64); ++w) acc = (v == OP_ITMAX) ? fmax(acc, sh[w][v]) : acc + sh[w][v];
    a.partials[(int64_t)blockIdx.x * kOrbitParts + v] = acc;
  }
}

}  // namespace

hipError_t launch_orbit(const OrbitArgs& a, int ngl, hipStream_t s) {
  (void)ngl;
  if (a.np <= 0) return hipSuccess;
  const unsigned blocks = (unsigned)((a.np + kBlock - 1) / kBlock);
  switch (a.M.d) {
    case 1: hipLaunchKernelGGL(k_orbit<1>, dim3(blocks), dim3(kBlock), kTileBytes, s, a); break;
    case 2: hipLaunchKernelGGL(k_orbit<2>, dim3(blocks), dim3(kBlock), kTileBytes, s, a); break;
    case 3: hipLaunchKernelGGL(k_orbit<3>, dim3(blocks), dim3(kBlock), kTileBytes, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gmhc
