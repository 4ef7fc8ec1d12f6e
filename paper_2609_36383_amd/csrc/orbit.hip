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
// J_g += q v_out S-bar_g / dV (FP64 atomics) and gathers U-bar for the diagnostics.
#include <math.h>

#include "gmhc_internal.h"

namespace gmhc {
namespace {

__device__ __forceinline__ int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

// Quadratic B-spline weights of nodes j-1, j, j+1 at offset f = xi - j in [-1/2, 1/2]
// and their x-derivatives (inverse spacing ih).
__device__ __forceinline__ void bw(double f, double w[3]) {
  double a = 0.5 - f, b = 0.5 + f;
  w[0] = 0.5 * a * a;
  w[1] = 0.75 - f * f;
  w[2] = 0.5 * b * b;
}
__device__ __forceinline__ void bdw(double f, double ih, double dw[3]) {
  dw[0] = (f - 0.5) * ih;
  dw[1] = -2.0 * f * ih;
  dw[2] = (0.5 + f) * ih;
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

// Point interpolant sum_g F_g S_g(x) of a 3-component mesh array at normalized xi.
template <int D>
__device__ __forceinline__ void interp3(const Mesh& M, const double* const* F, const double* xi,
                                        double out[3]) {
  int gi[3][3];
  double w[3][3];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if (l < D) {
      int j = (int)floor(xi[l] + 0.5);
      bw(xi[l] - (double)j, w[l]);
#pragma unroll
      for (int c = 0; c < 3; ++c) gi[l][c] = wrapi(j + c - 1, M.n[l]);
    } else {
      w[l][0] = 1.0;
      gi[l][0] = 0;
    }
  }
  out[0] = out[1] = out[2] = 0.0;
  constexpr int NY = D > 1 ? 3 : 1, NZ = D > 2 ? 3 : 1;
#pragma unroll
  for (int cz = 0; cz < NZ; ++cz)
#pragma unroll
    for (int cy = 0; cy < NY; ++cy) {
      double wyz = w[1][cy] * w[2][cz];
      int64_t row = (int64_t)M.n[0] * (gi[1][cy] + (int64_t)M.n[1] * gi[2][cz]);
#pragma unroll
      for (int cx = 0; cx < 3; ++cx) {
        double S = w[0][cx] * wyz;
        int64_t g = gi[0][cx] + row;
        out[0] += S * F[0][g];
        out[1] += S * F[1][g];
        out[2] += S * F[2][g];
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
  double ux = p[0] * inv_mk, uy = p[1] * inv_mk, uz = p[2] * inv_mk;
  return sqrt(1.0 + ux * ux + uy * uy + uz * uz);
}

// One orbit evaluation of one particle.
template <int D>
__device__ void evaluate(const OrbitArgs& a, const double* x, const double* xi0, const double P[3],
                         double q, double m, const double Am[3], const double vin[3], EvalOut& o) {
  const Mesh& M = a.M;
  double dxi[3];
#pragma unroll
  for (int l = 0; l < D; ++l) dxi[l] = a.dt * vin[l] * M.inv_h[l];
  double gp[3] = {0.0, 0.0, 0.0};
  double Dm[3][3];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int j = 0; j < 3; ++j) Dm[l][j] = 0.0;

  constexpr int NY = D > 1 ? 3 : 1, NZ = D > 2 ? 3 : 1;
  int nseg = 0;
  for_each_segment<D>(xi0, dxi, [&](double sa, double sb) {
    double len = sb - sa, sm = 0.5 * (sa + sb);
    ++nseg;
    int gi[3][3];
    int jn[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      if (l < D) {
        jn[l] = (int)floor(xi0[l] + sm * dxi[l] + 0.5);
#pragma unroll
        for (int c = 0; c < 3; ++c) gi[l][c] = wrapi(jn[l] + c - 1, M.n[l]);
      } else {
        jn[l] = 0;
        gi[l][0] = gi[l][1] = gi[l][2] = 0;
      }
    }
    for (int qp = 0; qp < a.ngl; ++qp) {
      double s = sa + len * a.glx[qp];
      double wq = len * a.glw[qp];
      double w[3][3], dw[3][3];
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        if (l < D) {
          double f = xi0[l] + s * dxi[l] - (double)jn[l];
          bw(f, w[l]);
          bdw(f, M.inv_h[l], dw[l]);
        } else {
          w[l][0] = 1.0;
          dw[l][0] = 0.0;
        }
      }
      double al = wq * (1.0 - s), be = wq * s;
#pragma unroll
      for (int cz = 0; cz < NZ; ++cz)
#pragma unroll
        for (int cy = 0; cy < NY; ++cy) {
          int64_t row = (int64_t)M.n[0] * (gi[1][cy] + (int64_t)M.n[1] * gi[2][cz]);
#pragma unroll
          for (int cx = 0; cx < 3; ++cx) {
            int64_t g = gi[0][cx] + row;
            double S = w[0][cx] * w[1][cy] * w[2][cz];
            double dS[3];
            dS[0] = dw[0][cx] * w[1][cy] * w[2][cz];
            if (D > 1) dS[1] = w[0][cx] * dw[1][cy] * w[2][cz];
            if (D > 2) dS[2] = w[0][cx] * w[1][cy] * dw[2][cz];
            double wS = wq * S;
#pragma unroll
            for (int l = 0; l < D; ++l) gp[l] += wS * a.gphi[l][g];
#pragma unroll
            for (int l = 0; l < 3; ++l) {
              double t = al * a.An[l][g] + be * a.Anp1[l][g];
#pragma unroll
              for (int j = 0; j < D; ++j) Dm[l][j] += t * dS[j];
            }
          }
        }
    }
  });

  // endpoint interpolant A^+ = A_h^{n+1}(x^n + dt v_in)
  double xie[3];
#pragma unroll
  for (int l = 0; l < D; ++l) xie[l] = xi0[l] + dxi[l];
  double Ap[3];
  interp3<D>(M, a.Anp1, xie, Ap);

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
  double Beff[3] = {Dm[2][1] - Dm[1][2], -(Dm[2][0] - Dm[0][2]), Dm[1][0] - Dm[0][1]};
  // normalized HC map
  const double inv_mk = 1.0 / (m * kappa);
  double um[3] = {pm[0] * inv_mk, pm[1] * inv_mk, pm[2] * inv_mk};
  const double tc = q * dt / (2.0 * m);
  double tau[3] = {tc * Beff[0], tc * Beff[1], tc * Beff[2]};
  double gm2 = 1.0 + um[0] * um[0] + um[1] * um[1] + um[2] * um[2];
  double tau2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];
  double ut = um[0] * tau[0] + um[1] * tau[1] + um[2] * tau[2];
  double sig = gm2 - tau2;
  double X = tau2 + ut * ut;
  double R = sqrt(sig * sig + 4.0 * X);
  double g2 = (sig >= 0.0) ? 0.5 * (sig + R) : 2.0 * X / (R - sig);
  double ig = 1.0 / sqrt(g2);
  double t[3] = {tau[0] * ig, tau[1] * ig, tau[2] * ig};
  double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
  double sf = 2.0 / (1.0 + t2);
  double sv[3] = {sf * t[0], sf * t[1], sf * t[2]};
  double us[3] = {um[0] + (um[1] * t[2] - um[2] * t[1]), um[1] + (um[2] * t[0] - um[0] * t[2]),
                  um[2] + (um[0] * t[1] - um[1] * t[0])};
  double up[3] = {um[0] + (us[1] * sv[2] - us[2] * sv[1]), um[1] + (us[2] * sv[0] - us[0] * sv[2]),
                  um[2] + (us[0] * sv[1] - us[1] * sv[0])};
  const double mk = m * kappa;
  double pp[3] = {mk * up[0], mk * up[1], mk * up[2]};
  double pn[3], Pn1[3], pn1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    Pn1[c] = pp[c] + q * Aep[c] + kick[c];
    pn[c] = P[c] - q * Am[c];
    pn1[c] = Pn1[c] - q * Ap[c];
  }
  // secant velocities and the orbit velocity
  double gm_ = gam(pm, inv_mk), gn = gam(pn, inv_mk), gn1 = gam(pn1, inv_mk), gp_ = gam(pp, inv_mk);
  double d1 = 1.0 / (m * (gm_ + gn)), d2 = 1.0 / (m * (gn1 + gp_));
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

// Deposit q v_out S-bar / dV along the orbit of v_in and gather U-bar.
template <int D>
__device__ void deposit_orbit(const OrbitArgs& a, const double* xi0, const double vin[3],
                              const double coef[3], bool do_dep, double Ub[3]) {
  const Mesh& M = a.M;
  double dxi[3];
#pragma unroll
  for (int l = 0; l < D; ++l) dxi[l] = a.dt * vin[l] * M.inv_h[l];
  Ub[0] = Ub[1] = Ub[2] = 0.0;
  constexpr int NY = D > 1 ? 3 : 1, NZ = D > 2 ? 3 : 1;
  for_each_segment<D>(xi0, dxi, [&](double sa, double sb) {
    double len = sb - sa, sm = 0.5 * (sa + sb);
    int gi[3][3];
    int jn[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      if (l < D) {
        jn[l] = (int)floor(xi0[l] + sm * dxi[l] + 0.5);
#pragma unroll
        for (int c = 0; c < 3; ++c) gi[l][c] = wrapi(jn[l] + c - 1, M.n[l]);
      } else {
        jn[l] = 0;
        gi[l][0] = gi[l][1] = gi[l][2] = 0;
      }
    }
    double acc[NZ][NY][3];
#pragma unroll
    for (int cz = 0; cz < NZ; ++cz)
#pragma unroll
      for (int cy = 0; cy < NY; ++cy)
#pragma unroll
        for (int cx = 0; cx < 3; ++cx) acc[cz][cy][cx] = 0.0;
    for (int qp = 0; qp < a.ngl; ++qp) {
      double s = sa + len * a.glx[qp];
      double wq = len * a.glw[qp];
      double w[3][3];
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        if (l < D)
          bw(xi0[l] + s * dxi[l] - (double)jn[l], w[l]);
        else
          w[l][0] = 1.0;
      }
#pragma unroll
      for (int cz = 0; cz < NZ; ++cz)
#pragma unroll
        for (int cy = 0; cy < NY; ++cy) {
          double wyz = wq * w[1][cy] * w[2][cz];
#pragma unroll
          for (int cx = 0; cx < 3; ++cx) acc[cz][cy][cx] += w[0][cx] * wyz;
        }
    }
#pragma unroll
    for (int cz = 0; cz < NZ; ++cz)
#pragma unroll
      for (int cy = 0; cy < NY; ++cy) {
        int64_t row = (int64_t)M.n[0] * (gi[1][cy] + (int64_t)M.n[1] * gi[2][cz]);
#pragma unroll
        for (int cx = 0; cx < 3; ++cx) {
          int64_t g = gi[0][cx] + row;
          double Sb = acc[cz][cy][cx];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            Ub[c] += Sb * a.Uh[c][g];
            if (do_dep) atomicAdd(a.J[c] + g, coef[c] * Sb);
          }
        }
      }
  });
}

template <int D>
__global__ __launch_bounds__(kBlock) void k_orbit(OrbitArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double part[kOrbitParts];
#pragma unroll
  for (int v = 0; v < kOrbitParts; ++v) part[v] = 0.0;
  if (i < a.np) {
    const Mesh& M = a.M;
    double x[3] = {0.0, 0.0, 0.0}, xi0[3] = {0.0, 0.0, 0.0};
    bool valid = true;
#pragma unroll
    for (int l = 0; l < D; ++l) {
      x[l] = a.x[l][i];
      xi0[l] = (x[l] - M.lo[l]) * M.inv_h[l];
      valid = valid && isfinite(xi0[l]) && fabs(xi0[l]) < 1.0e8;
    }
    double P[3] = {a.P[0][i], a.P[1][i], a.P[2][i]};
    double vin[3] = {a.v[0][i], a.v[1][i], a.v[2][i]};
    const double q = a.q[i];
    const double m = fabs(q);
    double Am[3] = {0.0, 0.0, 0.0};
    if (valid) interp3<D>(M, a.An, xi0, Am);
    EvalOut o;
    int it = 0;
    bool conv = false;
    const int maxit = a.iterate ? a.max_inner : 1;
    for (it = 1; it <= maxit; ++it) {
      // the orbit must stay finite and within the supported knot-crossing range
      double vnin = sqrt(vin[0] * vin[0] + vin[1] * vin[1] + vin[2] * vin[2]);
      bool ok = valid && isfinite(vnin);
#pragma unroll
      for (int l = 0; l < D; ++l) ok = ok && fabs(a.dt * vin[l] * M.inv_h[l]) < (double)(kMaxCross - 1);
      if (!ok) {
        valid = false;
        break;
      }
      evaluate<D>(a, x, xi0, P, q, m, Am, vin, o);
      part[OP_SEGS] += (double)o.nseg;
      if (!a.iterate) {
        conv = true;
        break;
      }
      double vn = sqrt(o.vout[0] * o.vout[0] + o.vout[1] * o.vout[1] + o.vout[2] * o.vout[2]);
      if (!isfinite(vn) || !(vn < a.kappa)) break;  // finite and subluminal
      double dmax = 0.0, vmax = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        dmax = fmax(dmax, fabs(o.vout[c] - vin[c]));
        vmax = fmax(vmax, fabs(o.vout[c]));
      }
      if (dmax <= a.tol_abs + a.tol_rel * vmax) {
        conv = true;
        break;
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) vin[c] = o.vout[c];
    }
    if (it > maxit) it = maxit;
    part[OP_FAIL] = conv ? 0.0 : 1.0;
    part[OP_ITERS] = (double)it;
    part[OP_ITMAX] = (double)it;
    if (conv) {
      double coef[3];
      const double qv = q / M.dV;
#pragma unroll
      for (int c = 0; c < 3; ++c) coef[c] = qv * o.vout[c];
      double Ub[3];
      deposit_orbit<D>(a, xi0, vin, coef, a.deposit != 0, Ub);
      // accept-pass diagnostics of this evaluation
      double ra2 = 0.0, wk = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double Dv = 0.0;
#pragma unroll
        for (int j = 0; j < D; ++j) Dv += o.Dm[c][j] * vin[j];
        double r = o.Ap[c] - Am[c] - a.dt * (Ub[c] + Dv);
        ra2 += r * r;
        wk += o.vout[c] * (-o.gp[c] - Ub[c]);
      }
      const double inv_mk = 1.0 / (m * a.kappa);
      double p2 = o.pn1[0] * o.pn1[0] + o.pn1[1] * o.pn1[1] + o.pn1[2] * o.pn1[2];
      part[OP_KIN] = p2 / (m * (gam(o.pn1, inv_mk) + 1.0));
      part[OP_WORK] = q * wk;
      part[OP_RA2] = ra2;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        a.v[c][i] = o.vout[c];
        a.Pn[c][i] = o.Pn1[c];
      }
#pragma unroll
      for (int l = 0; l < D; ++l) {
        double xv = x[l] + a.dt * vin[l];
        const double top = M.lo[l] + M.len[l];
        if (xv >= top) xv -= M.len[l];
        if (xv < M.lo[l]) xv += M.len[l];
        if (xv >= top) xv -= M.len[l];
        a.xn[l][i] = xv;
      }
    }
    a.iters[i] = it;
  }
  // block reduction in a fixed order: butterfly within each wave, then waves in order
#pragma unroll
  for (int v = 0; v < kOrbitParts; ++v) {
    for (int off = 32; off > 0; off >>= 1) {
      double o2 = __shfl_xor(part[v], off, 64);
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
    case 1: hipLaunchKernelGGL(k_orbit<1>, dim3(blocks), dim3(kBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_orbit<2>, dim3(blocks), dim3(kBlock), 0, s, a); break;
    case 3: hipLaunchKernelGGL(k_orbit<3>, dim3(blocks), dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace gmhc
