// orbit.hip -- the orbit pass: one thread per particle runs the inner Picard loop of
// the GM-HC orbit evaluation at frozen trial fields and deposits the orbit current.
//
// Per evaluation v_out = F(v_in) (sections "Symmetric orbit-averaged maps",
// "Orbit-averaged discrete chain rule", "No-explicit-A_t GM-HC step",
// "Mechanical split and magnetic zero work"):
//   1. straight unwrapped orbit x(s) = x^n + s dt v_in, split at the knots of the
//      B-spline shape (quadratic: half-integer node offsets; linear: the nodes),
//      Gauss-Legendre on each piece;
//   2. orbit gathers: grad phi-bar = int sum_g (grad_h phi^{n+1/2})_g S_g ds and the
//      orbit discrete gradient D_lj = int sum_g ((1-s) A^n + s A^{n+1})_{l,g} d_j S_g ds;
//   3. endpoint interpolants A^- = A_h^n(x^n), A^+ = A_h^{n+1}(x^n + dt v_in);
//   4. p^- = P^n - q A_ep - (q dt/2) grad-phi-bar + (q dt/2) D v_in, HC rotation with
//      B_eff = axial vector of K = D^T - D, P^{n+1} = p^+ + q A_ep + the same kick;
//   5. v_out = average of the secant velocities V^dg(p^-, p^n) and V^dg(p^{n+1}, p^+).
// After the inner test passes, a second sweep over the same orbit deposits
// J_g += q v_out S-bar_g / dV and gathers U-bar for the diagnostics.
//
// Memory layout on chip.  Particles arrive sorted by cell and a workgroup is one
// wave, so its particles sit in a small box of cells.  Each workgroup stages in LDS the
// mesh fields of the box spanned by its particles' nodes and their warm-start orbit
// endpoints, plus the stencil reach of one node, and accumulates its current deposit
// in an FP64 LDS tile of the same box, summed in a fixed order within the wave.  The
// tile is flushed to HBM as fixed-point integers (fixsum.h), one pair of integer atomics
// per tile node and component, so the current is the same whatever the order in which
// workgroups finish.  Orbit segments whose stencil leaves the tile, and workgroups whose
// box does not fit, read and deposit (fixed-point) through global memory instead.
//
// Arithmetic.  The bulk type R (double, or float in the FP32-bulk mode) carries the
// particle state, the staged fields, the quadrature and the push; positions stay
// FP64 and the orbit geometry is taken relative to the particle's nearest node, so
// FP32 keeps sub-cell resolution.  The deposit tile, the current and every
// reduction (kinetic energy, work, chain-rule residual) are FP64.
#include <hip/hip_ext.h>
#include <limits.h>
#include <math.h>

#include "gmhc_internal.h"
#include "wave.h"

namespace gmhc {
namespace {

constexpr int kHalo = 1;               // tile halo in nodes (the stencil reach)
// LDS per workgroup for the field and current tiles.  A one-wave workgroup of sorted
// particles spans one or two cells; the budgets let eight workgroups share a CU's
// 160 KB in every dimension, with the park block below where there is one (3D: a
// 5 x 5 x 5 box of 12 FP64 values per node; a larger box takes the global path).
template <int D>
constexpr int tile_bytes() { return D == 3 ? 16 * 1024 : 8 * 1024; }

// The particle constants wait in LDS (PARK) instead of registers across the segment
// quadrature where registers are short: FP64 2D quadratic at its default Gauss order,
// which keeps the row-independent quadrature values of each segment (Gauss point offsets
// and factors, hence its x weights) across the stencil rows, and FP64 3D quadratic at its
// default order, whose 27-node quadrature otherwise spills.
template <int D, int SH, int NGL, class R>
constexpr bool orbit_park() {
  return SH == 2 && sizeof(R) == 8 && ((D == 2 && NGL == 3) || (D == 3 && NGL == 4));
}

// i mod n for a mesh size n (a power of two; two's complement makes this the
// non-negative residue for negative i too)
__device__ __forceinline__ int wrapi(int i, int n) { return i & (n - 1); }

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

// A position less than one period outside [lo, lo + len) brought back into it.
__device__ __forceinline__ double wrap_pos(double xv, double lo, double len) {
  const double top = lo + len;
  if (xv >= top) xv -= len;
  if (xv < lo) xv += len;
  if (xv >= top) xv -= len;
  return xv;
}

// Reciprocal and square roots: hardware estimates refined by Newton / Goldschmidt
// steps to full FP64 precision; single hardware instructions in FP32.
__device__ __forceinline__ double rcp_(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ float rcp_(float x) { return __builtin_amdgcn_rcpf(x); }

// sqrt(a) and 1/sqrt(a) for a >= 1e-300 (normal, positive).
__device__ __forceinline__ void sqrt_rsq(double a, double& s, double& rs) {
  const double y = __builtin_amdgcn_rsq(a);
  double g = a * y, h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  const double d = fma(-g, g, a);
  s = fma(d, h, g);
  rs = 2.0 * h;
}
__device__ __forceinline__ void sqrt_rsq(float a, float& s, float& rs) {
  s = __builtin_amdgcn_sqrtf(a);
  rs = __builtin_amdgcn_rsqf(a);
}
template <class R>
__device__ __forceinline__ R sqrt_(R a) {
  R s, rs;
  sqrt_rsq(a, s, rs);
  return s;
}

// Workgroup tile: box of unwrapped node coordinates [o, o + E) per axis (uniform).
struct Tile {
  int o[3];
  int E[3];
  int nodes;
  int ok;     // 1: fields staged in LDS
  int joff;   // double offset of the current tile in the dynamic LDS block
  int goff;   // int offset of the tile nodes' mesh indices in the dynamic LDS block
};

// Fields of the staged tile: 0..D-1 grad phi, D..D+2 A^n, D+3..D+5 A^{n+1},
// D+6..D+8 U^{n+1/2}; the FP64 current tile (3 components) follows the fields.
template <int D>
__device__ __forceinline__ constexpr int nfields() { return D + 9; }

template <int D>
__device__ __forceinline__ const double* gfield(const OrbitArgs& a, int f) {
  const int64_t Ng = a.M.Ng;
  if (f < D) return a.gphi + (int64_t)f * Ng;
  if (f < D + 3) return a.An + (int64_t)(f - D) * Ng;
  if (f < D + 6) return a.Anp1 + (int64_t)(f - D - 3) * Ng;
  return a.Uh + (int64_t)(f - D - 6) * Ng;
}

template <int D, class R, bool LDS>
__device__ __forceinline__ R ld(const OrbitArgs& a, const Tile& t, int f, int node) {
  if (LDS) {
    HIP_DYNAMIC_SHARED(double, s_dyn);
    const R* s_tile = reinterpret_cast<const R*>(s_dyn);
    return s_tile[f * t.nodes + node];
  } else {
    return (R)gfield<D>(a, f)[node];
  }
}

// Node index of stencil offsets (cx, cy, cz) around the absolute node jn: into the LDS
// tile or into the periodic mesh.
template <int D, bool LDS>
struct Stencil {
  int ix[3];
  int base_y, base_z;  // unwrapped or tile-relative row coordinates of offset 0
  const Mesh* M;
  const Tile* t;
  __device__ __forceinline__ Stencil(const Mesh& m, const Tile& tt, const int jn[3]) : M(&m), t(&tt) {
#pragma unroll
    for (int c = 0; c < 3; ++c) ix[c] = LDS ? jn[0] + c - 1 - tt.o[0] : wrapi(jn[0] + c - 1, m.n[0]);
    base_y = LDS ? jn[1] - 1 - tt.o[1] : jn[1] - 1;
    base_z = LDS ? jn[2] - 1 - tt.o[2] : jn[2] - 1;
  }
  __device__ __forceinline__ int row(int cy, int cz) const {
    if (LDS)
      return (D > 1 ? t->E[0] * (base_y + cy) : 0) + (D > 2 ? t->E[0] * t->E[1] * (base_z + cz) : 0);
    return (D > 1 ? M->n[0] * wrapi(base_y + cy, M->n[1]) : 0) +
           (D > 2 ? M->n[0] * M->n[1] * wrapi(base_z + cz, M->n[2]) : 0);
  }
};

template <int D>
__device__ __forceinline__ bool inside(const Tile& t, const int jn[3]) {
  bool r = t.ok != 0;
#pragma unroll
  for (int l = 0; l < D; ++l) r = r && (jn[l] - 1 >= t.o[l]) && (jn[l] + 1 < t.o[l] + t.E[l]);
  return r;
}

// B-spline weights of nodes j-1, j, j+1 at local offset f from node j, and their
// derivatives with respect to xi (times h they are d/dx).  SH = 2: the quadratic S_2,
// j the nearest node, f in [-1/2, 1/2].  SH = 1: the linear S_1 = (1-|xi|)_+ (the
// degree the paper raises to two), j = floor(xi), f in [0, 1]: only nodes j and j+1
// (stencil columns 1 and 2) carry weight, and the derivatives are those of the knot
// segment [j, j+1] the point lies in.
template <int SH, class R>
__device__ __forceinline__ void bw(R f, R w[3], R dw[3]) {
  if constexpr (SH == 1) {
    w[0] = R(0);
    w[1] = R(1) - f;
    w[2] = f;
    dw[0] = R(0);
    dw[1] = R(-1);
    dw[2] = R(1);
  } else {
    // w2 - w0 = f: one addition instead of a square
    const R a = R(0.5) - f;
    w[0] = R(0.5) * a * a;
    w[1] = R(0.75) - f * f;
    w[2] = w[0] + f;
    dw[0] = -a;
    dw[1] = R(-2.0) * f;
    dw[2] = R(0.5) + f;
  }
}
// weight and derivative of the single stencil node c (0, 1, 2).  SHORT (for stencil rows
// known at compile time): the S_2 outer nodes take their pieces directly, since f lies
// within half a node of the base node (|f| <= 1/2 up to rounding) and so the offsets
// f + 1 and f - 1 of nodes 0 and 2 are positive and negative.  Otherwise the piece is
// chosen by |offset|, which costs fewer registers when c is a run-time value.
template <int SH, bool SHORT, class R>
__device__ __forceinline__ void bw1(R f, int c, R& w, R& dw) {
  if constexpr (SH == 1) {
    w = c == 0 ? R(0) : (c == 1 ? R(1) - f : f);
    dw = c == 0 ? R(0) : (c == 1 ? R(-1) : R(1));
  } else if constexpr (SHORT) {
    if (c == 1) {
      w = R(0.75) - f * f;
      dw = R(-2.0) * f;
    } else {
      const R g = c == 0 ? R(0.5) - f : R(0.5) + f;
      w = R(0.5) * g * g;
      dw = c == 0 ? -g : g;
    }
  } else {
    const R t = f - R(c - 1);  // offset from node j + c - 1
    const R at = fabs(t);
    const R o = R(1.5) - at;
    const R sg = t > R(0) ? R(1) : R(-1);
    w = c == 1 ? R(0.75) - t * t : R(0.5) * o * o;
    dw = c == 1 ? R(-2.0) * t : -sg * o;
  }
}

// The short form where it does not raise register use: FP64 with rows unrolled (d < 3).
template <int D, class R>
constexpr bool kShortW = D < 3 && sizeof(R) == 8;

// Stencil rows and columns that carry weight: all three per axis for S_2, the upper two
// (nodes j and j+1) for S_1.  Rows of the 3^(d-1) row layout are visited as
// cy = RB + row % RW, cz = RB + row / RW.
template <int SH>
constexpr int kC0 = SH == 1 ? 1 : 0;
template <int D, int SH>
constexpr int kRows = D == 1 ? 1 : (SH == 1 ? (D == 2 ? 2 : 4) : (D == 2 ? 3 : 9));

// Knot offset from the nodes of the B-spline of degree SH: half-integer for S_2, the
// nodes themselves for S_1.
template <int SH, class R>
__device__ __forceinline__ constexpr R knot_off() { return SH == 1 ? R(0) : R(0.5); }

// Orbit geometry relative to the particle's node j0: xi(s) = j0 + f0 + s del.
// Visits the knot-split segments [sa, sb] of s in [0, 1]; each axis' crossings of the
// half-integer knots are monotone in s and are merged on the fly.
template <int D, int SH, class R, class F>
__device__ __forceinline__ void for_each_segment(const R* f0, const R* del, F&& f) {
  R knot[3], next[3], stp[3], rd[3];
#pragma unroll
  for (int l = 0; l < D; ++l) {
    rd[l] = del[l] != R(0) ? rcp_(del[l]) : R(0);
    if (del[l] > R(0)) {
      knot[l] = floor(f0[l] - knot_off<SH, R>()) + R(1) + knot_off<SH, R>();
      stp[l] = R(1);
      next[l] = (knot[l] - f0[l]) * rd[l];
    } else if (del[l] < R(0)) {
      knot[l] = ceil(f0[l] - knot_off<SH, R>()) - R(1) + knot_off<SH, R>();
      stp[l] = R(-1);
      next[l] = (knot[l] - f0[l]) * rd[l];
    } else {
      knot[l] = R(0);
      stp[l] = R(0);
      next[l] = R(2);
    }
  }
  R sa = R(0);
#pragma unroll 1
  for (int it = 0; it <= D * kMaxCross; ++it) {
    R sb = R(1);
#pragma unroll
    for (int l = 0; l < D; ++l) sb = (next[l] < sb) ? next[l] : sb;
    if (sb > sa) f(sa, sb);
    if (sb >= R(1)) break;
#pragma unroll
    for (int l = 0; l < D; ++l)
      if (next[l] == sb) {
        knot[l] += stp[l];
        next[l] = (knot[l] - f0[l]) * rd[l];
      }
    sa = sb;
  }
}

// Base node of the segment point s (nearest node for S_2, the node below for S_1):
// relative offsets k and local offset at s = 0.
template <int D, int SH, class R>
__device__ __forceinline__ void seg_base(const int j0[3], const R* f0, const R* del, R sm, int jn[3], R fs[3]) {
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if (l < D) {
      const R xm = f0[l] + sm * del[l];
      const int k = SH == 1 ? (int)floor(xm) : (int)floor(xm + R(0.5));
      jn[l] = j0[l] + k;
      fs[l] = f0[l] - R(k);
    } else {
      jn[l] = 0;
      fs[l] = R(0);
    }
  }
}

template <int NGL>
struct GL {
  // compile-time point count; NGL == 0 runs the runtime count
  __device__ static constexpr int n(int runtime) { return NGL > 0 ? NGL : runtime; }
};

// Point interpolant sum_g F_g S_g at node jn with local offsets f (field base fb).
template <int D, int SH, class R, bool LDS>
__device__ __forceinline__ void interp3_at(const OrbitArgs& a, const Tile& t, int fb, const int jn[3],
                                           const R f[3], R out[3]) {
  R w[3][3], dw[3][3];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if (l < D) {
      bw<SH>(f[l], w[l], dw[l]);
    } else {
      w[l][0] = R(1);
    }
  }
  Stencil<D, LDS> st(a.M, t, jn);
  out[0] = out[1] = out[2] = R(0);
  constexpr int NY = D > 1 ? 3 : 1, NZ = D > 2 ? 3 : 1;
  constexpr int Y0 = D > 1 ? kC0<SH> : 0, Z0 = D > 2 ? kC0<SH> : 0;
#pragma unroll
  for (int cz = Z0; cz < NZ; ++cz)
#pragma unroll
    for (int cy = Y0; cy < NY; ++cy) {
      const R wyz = w[1][cy] * w[2][cz];
      const int rowoff = st.row(cy, cz);
#pragma unroll
      for (int cx = kC0<SH>; cx < 3; ++cx) {
        const R S = w[0][cx] * wyz;
        const int g = st.ix[cx] + rowoff;
#pragma unroll
        for (int c = 0; c < 3; ++c) out[c] += S * ld<D, R, LDS>(a, t, fb + c, g);
      }
    }
}

template <int D, int SH, class R>
__device__ __forceinline__ void interp3(const OrbitArgs& a, const Tile& t, int fb, const int j0[3], const R* fr,
                                        R out[3]) {
  int jn[3];
  R f[3];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if (l < D) {
      const int k = SH == 1 ? (int)floor(fr[l]) : (int)floor(fr[l] + R(0.5));
      jn[l] = j0[l] + k;
      f[l] = fr[l] - R(k);
    } else {
      jn[l] = 0;
      f[l] = R(0);
    }
  }
  if (inside<D>(t, jn))
    interp3_at<D, SH, R, true>(a, t, fb, jn, f, out);
  else
    interp3_at<D, SH, R, false>(a, t, fb, jn, f, out);
}

// Quadrature of one knot segment for the gathers grad-phi-bar and D.
//
// The stencil is visited one x-row at a time (3^(d-1) rows of three nodes).  For the
// row, the integrated weights of its three nodes are accumulated over the Gauss
// points first,
//   S_c = sum_q w_q S_c(s_q),  X0_c = sum_q w_q (1-s_q) dS_c/dxi,  X1_c = sum_q w_q s_q dS_c/dxi
// (likewise Y0, Y1 and Z0, Z1), then contracted once with the row's node values:
//   grad-phi-bar += S_c (grad phi)_c,  D_l. += X0_c A^n_{l,c} + X1_c A^{n+1}_{l,c}.
// This is the same quadrature summed in a different order; each field value is read
// once per segment and only one row of weights is live at a time.  D is left in xi
// units and scaled by 1/h afterwards.
template <int D, int SH, int NGL, class R, bool LDS>
__device__ __forceinline__ void eval_segment(const OrbitArgs& a, const Tile& t, const R* gx, const R* gw,
                                             const int jn[3], const R fs[3], const R* del, R sa, R sb,
                                             R gp[3], R Dm[3][3]) {
  const R len = sb - sa;
  Stencil<D, LDS> st(a.M, t, jn);
  constexpr int NROW = kRows<D, SH>;
  constexpr int RW = SH == 1 ? 2 : 3, RB = kC0<SH>;
  // 1D and 2D rows at a compile-time GL order are unrolled (the y weights specialise
  // per row); 3D and the runtime order keep a loop
  constexpr int kRowUnroll = (D < 3 && NGL > 0) ? NROW : 1;
  // FP64 2D has registers for the row-independent quadrature factors w_q, w_q (1 - s_q)
  // and w_q s_q of its unrolled rows; elsewhere they are recomputed per row
  constexpr bool kHoist = D == 2 && orbit_park<D, SH, NGL, R>();
  constexpr int NH = kHoist ? NGL : 1;
  R hw[NH], ha[NH], hb[NH], hx[NH], hy[NH];
  if (kHoist) {
#pragma unroll
    for (int q = 0; q < NH; ++q) {
      const R s = sa + len * gx[q];
      hw[q] = len * gw[q];
      hb[q] = hw[q] * s;
      ha[q] = hw[q] - hb[q];
      hx[q] = fs[0] + s * del[0];
      hy[q] = fs[1] + s * del[1];
    }
  }
#pragma unroll kRowUnroll
  for (int row = 0; row < NROW; ++row) {
    const int cy = D > 1 ? RB + row % RW : 0, cz = D > 2 ? RB + row / RW : 0;
    const int rowoff = st.row(cy, cz);
    // FP32 has registers to spare: read the row's field values before the weight
    // arithmetic so their latency overlaps it.  FP64 reads them node by node below.
    constexpr bool kEarly = sizeof(R) == 4;
    R F[3][D + 6];
    if (kEarly) {
#pragma unroll
      for (int c = kC0<SH>; c < 3; ++c)
#pragma unroll
        for (int f = 0; f < D + 6; ++f) F[c][f] = ld<D, R, LDS>(a, t, f, st.ix[c] + rowoff);
    }
    R S[3], X0[3], X1[3], Y0[3], Y1[3], Z0[3], Z1[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) S[c] = X0[c] = X1[c] = Y0[c] = Y1[c] = Z0[c] = Z1[c] = R(0);
    // recompute the x weights per row rather than keep them live across rows
    R sar = sa;
    asm volatile("" : "+v"(sar));
    const int nq = GL<NGL>::n(a.ngl);
#pragma unroll
    for (int q = 0; q < nq; ++q) {
      const R s = sar + len * gx[q];
      R wq, b1, a1;  // w_q, w_q s and w_q (1 - s)
      if (kHoist) {
        wq = hw[q];
        b1 = hb[q];
        a1 = ha[q];
      } else {
        wq = len * gw[q];
        b1 = wq * s;
        a1 = wq - b1;
      }
      R wx[3], dwx[3];
      bw<SH>(kHoist ? hx[q] : fs[0] + s * del[0], wx, dwx);
      R wy = R(1), dwy = R(0), wz = R(1), dwz = R(0);
      if (D > 1) bw1<SH, kShortW<D, R>>(kHoist ? hy[q] : fs[1] + s * del[1], cy, wy, dwy);
      if (D > 2) bw1<SH, kShortW<D, R>>(fs[2] + s * del[2], cz, wz, dwz);
      const R wyz = wy * wz;
      const R sw = wq * wyz, xw0 = a1 * wyz, xw1 = b1 * wyz;
      const R yz = dwy * wz, zy = wy * dwz;
      const R yw0 = a1 * yz, yw1 = b1 * yz, zw0 = a1 * zy, zw1 = b1 * zy;
#pragma unroll
      for (int c = kC0<SH>; c < 3; ++c) {
        S[c] += sw * wx[c];
        X0[c] += xw0 * dwx[c];
        X1[c] += xw1 * dwx[c];
        if (D > 1) {
          Y0[c] += yw0 * wx[c];
          Y1[c] += yw1 * wx[c];
        }
        if (D > 2) {
          Z0[c] += zw0 * wx[c];
          Z1[c] += zw1 * wx[c];
        }
      }
    }
#pragma unroll
    for (int c = kC0<SH>; c < 3; ++c) {
      const int g = st.ix[c] + rowoff;
      if (!kEarly) {
#pragma unroll
        for (int f = 0; f < D + 6; ++f) F[c][f] = ld<D, R, LDS>(a, t, f, g);
      }
#pragma unroll
      for (int l = 0; l < D; ++l) gp[l] += S[c] * F[c][l];
#pragma unroll
      for (int l = 0; l < 3; ++l) {
        const R a0 = F[c][D + l], a1v = F[c][D + 3 + l];
        Dm[l][0] += X0[c] * a0 + X1[c] * a1v;
        if (D > 1) Dm[l][1] += Y0[c] * a0 + Y1[c] * a1v;
        if (D > 2) Dm[l][2] += Z0[c] * a0 + Z1[c] * a1v;
      }
    }
  }
}

template <class R>
struct EvalOut {
  R vout[3];
  R Pn1[3];
  R pn1[3];
  R Ap[3];
  R dA[3];  // A^+ - A^-
  R gp[3];
  R Dm[3][3];
  int nseg;
};

// Constants of one particle: its charge (m = |q|) and the gamma of p^n = P^n - q A^-
// (fixed over the inner iterations).  The other per-particle factors are recomputed from q
// after the segment quadrature, where fewer registers are live.
template <class R>
struct PConst {
  R q;
  R gpn;
};

// Particle constants parked in LDS (PARK): P^n, A^-, q and the gamma of p^n, value k of
// lane l at s_dyn[park + 64 k] with park = (LDS offset of the block) + l.  They are read
// back after the segment quadrature, so no registers hold them across it.
constexpr int kParkVals = 8;

template <class R>
__device__ __forceinline__ void park_store(int park, const R P[3], const R Am[3], const PConst<R>& pc) {
  HIP_DYNAMIC_SHARED(double, s_dyn);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    s_dyn[park + 64 * c] = (double)P[c];
    s_dyn[park + 64 * (3 + c)] = (double)Am[c];
  }
  s_dyn[park + 64 * 6] = (double)pc.q;
  s_dyn[park + 64 * 7] = (double)pc.gpn;
}

// One orbit evaluation of one particle.
template <int D, int SH, int NGL, class R, bool PARK = false>
__device__ void evaluate(const OrbitArgs& a, const Tile& t, const R* gx, const R* gw, const int j0[3], const R* f0,
                         const R Pa[3], const PConst<R>& pca, const R Ama[3], const R vin[3], EvalOut<R>& o,
                         int park = 0) {
  const Mesh& M = a.M;
  R del[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int l = 0; l < D; ++l) del[l] = R(a.dt) * vin[l] * R(M.inv_h[l]);
  R gp[3] = {R(0), R(0), R(0)};
  R Dm[3][3];
#pragma unroll
  for (int l = 0; l < 3; ++l)
#pragma unroll
    for (int j = 0; j < 3; ++j) Dm[l][j] = R(0);
  int nseg = 0;
  for_each_segment<D, SH, R>(f0, del, [&](R sa, R sb) {
    ++nseg;
    int jn[3];
    R fs[3];
    seg_base<D, SH, R>(j0, f0, del, R(0.5) * (sa + sb), jn, fs);
    if (inside<D>(t, jn))
      eval_segment<D, SH, NGL, R, true>(a, t, gx, gw, jn, fs, del, sa, sb, gp, Dm);
    else
      eval_segment<D, SH, NGL, R, false>(a, t, gx, gw, jn, fs, del, sa, sb, gp, Dm);
  });
#pragma unroll
  for (int j = 0; j < D; ++j) {
    const R ih = R(M.inv_h[j]);
#pragma unroll
    for (int l = 0; l < 3; ++l) Dm[l][j] *= ih;
  }

  // the particle constants, from LDS when parked (the opaque offset keeps the reads here)
  R P[3], Am[3];
  PConst<R> pc;
  if constexpr (PARK) {
    HIP_DYNAMIC_SHARED(double, s_dyn);
    int off = park;
    asm volatile("" : "+v"(off));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      P[c] = (R)s_dyn[off + 64 * c];
      Am[c] = (R)s_dyn[off + 64 * (3 + c)];
    }
    pc.q = (R)s_dyn[off + 64 * 6];
    pc.gpn = (R)s_dyn[off + 64 * 7];
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      P[c] = Pa[c];
      Am[c] = Ama[c];
    }
    pc = pca;
  }

  // endpoint interpolant A^+ = A_h^{n+1}(x^n + dt v_in)
  R fe[3] = {R(0), R(0), R(0)};
#pragma unroll
  for (int l = 0; l < D; ++l) fe[l] = f0[l] + del[l];
  R Ap[3];
  interp3<D, SH, R>(a, t, D + 3, j0, fe, Ap);

  const R q = pc.q;
  const R m = fabs(q);
  const R inv_mk = rcp_(m * R(a.kappa));
  const R tc = q * R(a.dt) * rcp_(R(2) * m);
  const R half_qdt = R(0.5) * q * R(a.dt);
  R Aep[3], kick[3], pm[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    Aep[c] = R(0.5) * (Am[c] + Ap[c]);
    R Dv = R(0);
#pragma unroll
    for (int j = 0; j < D; ++j) Dv += Dm[c][j] * vin[j];
    kick[c] = half_qdt * (Dv - gp[c]);
    pm[c] = P[c] - q * Aep[c] + kick[c];
  }
  // B_eff of the skew part K = D^T - D (D zero-padded to 3x3): (K23, -K13, K12)
  const R Beff[3] = {Dm[2][1] - Dm[1][2], -(Dm[2][0] - Dm[0][2]), Dm[1][0] - Dm[0][1]};
  // normalized HC map.  The rotation is linear in u = p / (m kappa), so it is applied
  // to p directly; u enters only through |u|^2 and u . tau in gamma_HC.  (Scaling p
  // down and back up would bias every momentum by the same rounding in FP32.)
  const R tau[3] = {tc * Beff[0], tc * Beff[1], tc * Beff[2]};
  const R um2 = (pm[0] * pm[0] + pm[1] * pm[1] + pm[2] * pm[2]) * inv_mk * inv_mk;
  const R tau2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];
  const R ut = (pm[0] * tau[0] + pm[1] * tau[1] + pm[2] * tau[2]) * inv_mk;
  const R sig = R(1) + um2 - tau2;
  const R X = tau2 + ut * ut;
  R tv[3];
  if (X > R(0)) {
    const R Rr = sqrt_(sig * sig + R(4) * X);
    const R g2 = (sig >= R(0)) ? R(0.5) * (sig + Rr) : R(2) * X * rcp_(Rr - sig);
    R gh, ig;
    sqrt_rsq(g2, gh, ig);
    tv[0] = tau[0] * ig;
    tv[1] = tau[1] * ig;
    tv[2] = tau[2] * ig;
  } else {
    tv[0] = tv[1] = tv[2] = R(0);  // no magnetic generator: the rotation is the identity
  }
  const R t2 = tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2];
  const R sf = R(2) * rcp_(R(1) + t2);
  const R sv[3] = {sf * tv[0], sf * tv[1], sf * tv[2]};
  const R ps[3] = {pm[0] + (pm[1] * tv[2] - pm[2] * tv[1]), pm[1] + (pm[2] * tv[0] - pm[0] * tv[2]),
                   pm[2] + (pm[0] * tv[1] - pm[1] * tv[0])};
  const R pp[3] = {pm[0] + (ps[1] * sv[2] - ps[2] * sv[1]), pm[1] + (ps[2] * sv[0] - ps[0] * sv[2]),
                   pm[2] + (ps[0] * sv[1] - ps[1] * sv[0])};
  R pn[3], Pn1[3], pn1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    Pn1[c] = pp[c] + q * Aep[c] + kick[c];
    pn[c] = P[c] - q * Am[c];
    pn1[c] = Pn1[c] - q * Ap[c];
  }
  // secant velocities V^dg and the orbit velocity
  auto gam = [&](const R p[3]) {
    const R ux = p[0] * inv_mk, uy = p[1] * inv_mk, uz = p[2] * inv_mk;
    return sqrt_(R(1) + ux * ux + uy * uy + uz * uz);
  };
  const R d1 = rcp_(m * (gam(pm) + pc.gpn));
  const R d2 = rcp_(m * (gam(pn1) + gam(pp)));
  o.nseg = nseg;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    o.vout[c] = R(0.5) * ((pm[c] + pn[c]) * d1 + (pn1[c] + pp[c]) * d2);
    o.Pn1[c] = Pn1[c];
    o.pn1[c] = pn1[c];
    o.Ap[c] = Ap[c];
    o.dA[c] = Ap[c] - Am[c];
    o.gp[c] = gp[c];
#pragma unroll
    for (int j = 0; j < 3; ++j) o.Dm[c][j] = Dm[c][j];
  }
}

// Per-lane iterator over the same knot-split segments as for_each_segment (same
// arithmetic, so the deposit sees exactly the segments the gathers saw); lets a whole
// wave step through its particles' segments in lockstep.
template <int D, int SH, class R>
struct SegIter {
  R knot[3], next[3], stp[3], rd[3];
  R sa;
  int steps;
  bool live;
  __device__ __forceinline__ void init(const R* f0, const R* del, bool on) {
#pragma unroll
    for (int l = 0; l < D; ++l) {
      rd[l] = del[l] != R(0) ? rcp_(del[l]) : R(0);
      if (del[l] > R(0)) {
        knot[l] = floor(f0[l] - knot_off<SH, R>()) + R(1) + knot_off<SH, R>();
        stp[l] = R(1);
        next[l] = (knot[l] - f0[l]) * rd[l];
      } else if (del[l] < R(0)) {
        knot[l] = ceil(f0[l] - knot_off<SH, R>()) - R(1) + knot_off<SH, R>();
        stp[l] = R(-1);
        next[l] = (knot[l] - f0[l]) * rd[l];
      } else {
        knot[l] = R(0);
        stp[l] = R(0);
        next[l] = R(2);
      }
    }
#pragma unroll
    for (int l = 0; l < 3; ++l) f0s[l] = l < D ? f0[l] : R(0);
    sa = R(0);
    steps = 0;
    live = on;
  }
  // next segment [s0, s1] of nonzero length; false once the orbit is exhausted
  __device__ __forceinline__ bool advance(R& s0, R& s1) {
    while (live) {
      R sb = R(1);
#pragma unroll
      for (int l = 0; l < D; ++l) sb = (next[l] < sb) ? next[l] : sb;
      const R a0 = sa;
      ++steps;
      if (sb >= R(1) || steps > D * kMaxCross) {
        live = false;
      } else {
#pragma unroll
        for (int l = 0; l < D; ++l)
          if (next[l] == sb) {
            knot[l] += stp[l];
            next[l] = (knot[l] - f0s[l]) * rd[l];
          }
      }
      sa = sb;
      if (sb > a0) {
        s0 = a0;
        s1 = sb;
        return true;
      }
    }
    return false;
  }
  R f0s[3];
};

// ---- wave-wide reduce-scatter (all 64 lanes active)
//
// The deposit of a wave is summed across the wave before it reaches LDS: NP2 values
// per lane (NP2 = 16, 32 or 64) are reduced so that every lane ends with the wave total
// of one value.  Exchange partners per step: lane ^ 32 and lane ^ 16 (gfx950 permlane
// swaps), lane ^ 8 (row rotation by 8), lane ^ 7 (half-row mirror), lane ^ 2 and
// lane ^ 1 (quad permutations).  The six masks span all 64 lanes, so each total covers
// the whole wave.  Each step halves the values a lane holds; once a lane holds one
// value, the remaining steps add the partner's copy instead.

// (A, B) -> lower rows keep A and receive the partner's A; upper rows keep B and
// receive the partner's B (partner lane ^ 32, or lane ^ 16 for ROW16).
template <bool ROW16>
__device__ __forceinline__ double swap_sum(double A, double B) {
  const uint64_t a = as_u64(A), b = as_u64(B);
  uint32_t alo, blo, ahi, bhi;
  if (ROW16) {
    const auto lo = __builtin_amdgcn_permlane16_swap((uint32_t)a, (uint32_t)b, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false);
    alo = lo[0]; blo = lo[1]; ahi = hi[0]; bhi = hi[1];
  } else {
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)a, (uint32_t)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(a >> 32), (uint32_t)(b >> 32), false, false);
    alo = lo[0]; blo = lo[1]; ahi = hi[0]; bhi = hi[1];
  }
  return as_f64(alo, ahi) + as_f64(blo, bhi);
}

template <int CTRL>
__device__ __forceinline__ double dpp_f64(double x) {
  const uint64_t u = as_u64(x);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)u, CTRL, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(u >> 32), CTRL, 0xF, 0xF, false);
  return as_f64(lo, hi);
}
constexpr int kDppRor8 = 0x128;        // row_ror:8  -> lane ^ 8
constexpr int kDppHalfMirror = 0x141;  // row_half_mirror -> lane ^ 7
constexpr int kDppXor2 = 0x4E;         // quad_perm [2,3,0,1]
constexpr int kDppXor1 = 0xB1;         // quad_perm [1,0,3,2]

// one scatter step through a DPP exchange: the lane keeps the lower half of v if its
// bit `kb` is clear, the upper half otherwise, and adds the partner's copy of it
template <int H, int CTRL>
__device__ __forceinline__ void dpp_step(double* v, bool up) {
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const double send = up ? v[j] : v[j + H];
    const double keep = up ? v[j + H] : v[j];
    v[j] = keep + dpp_f64<CTRL>(send);
  }
}

// Reduce-scatter of v[NP2]; returns the wave total of value wave_slot<NP2>(lane).
template <int NP2>
__device__ __forceinline__ double wave_reduce_scatter(double* v, int lane) {
  static_assert(NP2 == 16 || NP2 == 32 || NP2 == 64, "NP2");
  constexpr int H1 = NP2 / 2, H2 = NP2 / 4, H3 = NP2 / 8, H4 = NP2 / 16, H5 = NP2 / 32, H6 = NP2 / 64;
#pragma unroll
  for (int j = 0; j < H1; ++j) v[j] = swap_sum<false>(v[j], v[j + H1]);
#pragma unroll
  for (int j = 0; j < H2; ++j) v[j] = swap_sum<true>(v[j], v[j + H2]);
  dpp_step<H3, kDppRor8>(v, (lane & 8) != 0);
  dpp_step<H4, kDppHalfMirror>(v, (lane & 4) != 0);
  if constexpr (H5 > 0) {
    dpp_step<H5, kDppXor2>(v, (lane & 2) != 0);
  } else {
    v[0] += dpp_f64<kDppXor2>(v[0]);
  }
  if constexpr (H6 > 0) {
    dpp_step<H6, kDppXor1>(v, (lane & 1) != 0);
  } else {
    v[0] += dpp_f64<kDppXor1>(v[0]);
  }
  return v[0];
}
// value index a lane holds after wave_reduce_scatter (lane bit b stands for the half
// NP2 / 2^(6-b) kept at its step); owner() picks one copy of each
template <int NP2>
__device__ __forceinline__ int wave_slot(int lane) {
  const int b5 = (lane >> 5) & 1, b4 = (lane >> 4) & 1, b3 = (lane >> 3) & 1, b2 = (lane >> 2) & 1;
  if (NP2 == 64) return lane;
  return NP2 == 32 ? 16 * b5 + 8 * b4 + 4 * b3 + 2 * b2 + ((lane >> 1) & 1) : 8 * b5 + 4 * b4 + 2 * b3 + b2;
}
template <int NP2>
__device__ __forceinline__ bool wave_owner(int lane) {
  return NP2 == 64 ? true : (NP2 == 32 ? (lane & 1) == 0 : (lane & 3) == 0);
}

// Rows Y0 .. Y0+NR-1 of a window WX nodes wide: the lanes' values cf[k] W[y][x] are summed
// over the wave by one reduce-scatter, and each total is added to its tile node by the lane
// holding it (window node (x, y) is tile node b - 1 + (x, y, zp)).
template <int D, int WX, int Y0, int NR, class R>
__device__ __forceinline__ void window_rows(const Tile& t, const R (&W)[4][4], const double cf[3], const int b[3],
                                            int zp, int lane, double* s_J) {
  constexpr int NN = WX * NR, NV = 3 * NN, NP2 = NV <= 16 ? 16 : 32;
  double v[NP2];
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int nd = 0; nd < NN; ++nd) v[k * NN + nd] = cf[k] * (double)W[Y0 + nd / WX][nd % WX];
#pragma unroll
  for (int j = NV; j < NP2; ++j) v[j] = 0.0;
  const double tot = wave_reduce_scatter<NP2>(v, lane);
  const int idx = wave_slot<NP2>(lane);
  if (wave_owner<NP2>(lane) && idx < NV && tot != 0.0) {
    const int k = idx / NN, nd = idx - k * NN;
    const int gx = b[0] - 1 + (nd % WX) - t.o[0];
    const int gy = D > 1 ? b[1] - 1 + Y0 + nd / WX - t.o[1] : 0;
    const int gz = D > 2 ? b[2] - 1 + zp - t.o[2] : 0;
    // a nonzero total comes from stencils inside the tile; the test is a guard
    if (gx >= 0 && gx < t.E[0] && gy >= 0 && gy < t.E[1] && gz >= 0 && gz < t.E[2])
      atomicAdd(s_J + k * t.nodes + gx + t.E[0] * (gy + t.E[1] * gz), tot);
  }
}

// Window deposit with a window of WX x WY nodes per z-plane (WX, WY = 3 when no lane's
// base sits one node above b on that axis, else 4) and nz z-planes.
template <int D, class R, int NR, int WX, int WY>
__device__ void window_deposit(const Tile& t, const R (&S)[NR][3], const int o[3], const int b[3], const double cf[3],
                               int nz, int lane, double* s_J) {
  const bool sx = WX == 4 && o[0] != 0, sy = WY == 4 && o[1] != 0;
#pragma unroll 1
  for (int zp = 0; zp < nz; ++zp) {
    // the lane's stencil plane for window plane zp (zero when it has none there)
    R P[3][3];
#pragma unroll
    for (int cy = 0; cy < 3; ++cy)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (D == 3) {
          const int cz = zp - o[2];
          P[cy][c] = cz == 0 ? S[cy % NR][c] : (cz == 1 ? S[(3 + cy) % NR][c] : (cz == 2 ? S[(6 + cy) % NR][c] : R(0)));
        } else if (D == 2) {
          P[cy][c] = S[cy % NR][c];
        } else {
          P[cy][c] = cy == 0 ? S[0][c] : R(0);
        }
      }
    // shift along x, then along y, into the window
    R Wx[3][4];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      if (WX == 4) {
        Wx[r][0] = sx ? R(0) : P[r][0];
        Wx[r][1] = sx ? P[r][0] : P[r][1];
        Wx[r][2] = sx ? P[r][1] : P[r][2];
        Wx[r][3] = sx ? P[r][2] : R(0);
      } else {
        Wx[r][0] = P[r][0];
        Wx[r][1] = P[r][1];
        Wx[r][2] = P[r][2];
        Wx[r][3] = R(0);
      }
    }
    R W[4][4];
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      if (WY == 4) {
        W[0][x] = sy ? R(0) : Wx[0][x];
        W[1][x] = sy ? Wx[0][x] : Wx[1][x];
        W[2][x] = sy ? Wx[1][x] : Wx[2][x];
        W[3][x] = sy ? Wx[2][x] : R(0);
      } else {
        W[0][x] = Wx[0][x];
        W[1][x] = Wx[1][x];
        W[2][x] = Wx[2][x];
        W[3][x] = R(0);
      }
    }
    // reduce-scatters of at most 32 values: two or three rows at a time
    if (D == 1) {
      window_rows<D, WX, 0, 1>(t, W, cf, b, zp, lane, s_J);
    } else if (WX == 4) {
      window_rows<D, 4, 0, 2>(t, W, cf, b, zp, lane, s_J);
      if (WY == 4)
        window_rows<D, 4, 2, 2>(t, W, cf, b, zp, lane, s_J);
      else
        window_rows<D, 4, 2, 1>(t, W, cf, b, zp, lane, s_J);
    } else {
      window_rows<D, 3, 0, 3>(t, W, cf, b, zp, lane, s_J);
      if (WY == 4) window_rows<D, 3, 3, 1>(t, W, cf, b, zp, lane, s_J);
    }
  }
}

// Current deposit of one segment into the LDS tile.  S[row][c] holds the lane's
// integrated weights of its stencil (row = cy + 3 cz, node c along x).
//
// The lanes whose stencil lies in the tile share a window anchored one node below the
// lowest stencil base b of their cluster: three nodes per axis when every lane of the
// cluster has its base at b, four when some have it at b + 1.  The window lanes place
// q v_out S / dV into the window (shifted by their offset from b); reduce-scatters over
// the wave then leave each window value on one lane, which adds it to the tile.  In 2D and 3D the window is taken one
// z-plane at a time, two or three y-rows (at most 32 values) per reduction.
template <int D, class R, int NR>
__device__ __forceinline__ void deposit_window(const Tile& t, const int jn[3], const R (&S)[NR][3],
                                               const double coef[3], bool in, int lane) {
  HIP_DYNAMIC_SHARED(double, s_dyn);
  double* s_J = s_dyn + t.joff;
  // The lanes are taken in clusters.  Each pass takes the lanes whose base lies within one
  // node, on every axis, of the lowest remaining lane's base, and deposits them through
  // one window anchored at their lowest base (a fixed-order wave reduction, so every tile
  // value is summed in the same order on every run).  A sorted wave needs one pass; a wave
  // whose particles have drifted apart (counter-streaming beams) needs one per cluster.
  bool todo = in;
#pragma unroll 1
  for (uint64_t m = __ballot(todo); m != 0; m = __ballot(todo)) {
    const int lead = __ffsll((long long)m) - 1;  // wave-uniform
    bool near = todo;
#pragma unroll
    for (int l = 0; l < D; ++l) near = near && abs(jn[l] - __builtin_amdgcn_readlane(jn[l], lead)) <= 1;
    int b[3] = {0, 0, 0}, o[3] = {0, 0, 0};
    bool win = near;
#pragma unroll
    for (int l = 0; l < D; ++l) {
      b[l] = wave_min_i32(near ? jn[l] : INT_MAX);
      o[l] = jn[l] - b[l];
      win = win && o[l] <= 1;
    }
    const double cf[3] = {win ? coef[0] : 0.0, win ? coef[1] : 0.0, win ? coef[2] : 0.0};
    // window extent: wave-uniform choices
    const bool wx4 = uni(__ballot(win && o[0] != 0) != 0 ? 1 : 0) != 0;
    const bool wy4 = D > 1 && uni(__ballot(win && o[1] != 0) != 0 ? 1 : 0) != 0;
    const int nz = D > 2 ? (uni(__ballot(win && o[2] != 0) != 0 ? 1 : 0) ? 4 : 3) : 1;
    if (wx4) {
      if (wy4)
        window_deposit<D, R, NR, 4, 4>(t, S, o, b, cf, nz, lane, s_J);
      else
        window_deposit<D, R, NR, 4, 3>(t, S, o, b, cf, nz, lane, s_J);
    } else {
      if (wy4)
        window_deposit<D, R, NR, 3, 4>(t, S, o, b, cf, nz, lane, s_J);
      else
        window_deposit<D, R, NR, 3, 3>(t, S, o, b, cf, nz, lane, s_J);
    }
    todo = todo && !win;
  }
}

// Deposit phase of the pass, run by every lane of the workgroup: the lanes whose
// particle converged walk the segments of their accepted orbit (v_in) in lockstep;
// per segment they take the integrated weights of every stencil row, gather U-bar and
// deposit J_g += q v_out S-bar_g / dV into the tile through the window deposit.
// Stencils outside the tile read and add through global memory per lane.
template <int D, int SH, int NGL, class R>
__device__ void deposit_phase(const OrbitArgs& a, const Tile& t, const R* gx, const R* gw, const int j0[3],
                              const R* f0, const R del[3], bool dep, const double coef[3], R Ub[3]) {
  const int lane = threadIdx.x & 63;
  const bool do_dep = a.deposit != 0;
  SegIter<D, SH, R> sit;
  sit.init(f0, del, dep);
  Ub[0] = Ub[1] = Ub[2] = R(0);
#pragma unroll 1
  for (int guard = 0; guard <= D * kMaxCross; ++guard) {
    R sa = R(0), sb = R(0);
    const bool has = sit.advance(sa, sb);
    if (__ballot(has) == 0) break;
    int jn[3] = {0, 0, 0};
    R fs[3] = {R(0), R(0), R(0)};
    if (has) seg_base<D, SH, R>(j0, f0, del, R(0.5) * (sa + sb), jn, fs);
    const bool in = has && inside<D>(t, jn);
    const R len = sb - sa;  // zero for lanes without a segment: all weights vanish
    constexpr int NROW = D == 1 ? 1 : (D == 2 ? 3 : 9);
    R Sr[NROW][3];
#pragma unroll
    for (int row = 0; row < NROW; ++row) {
      const int cy = D > 1 ? row % 3 : 0, cz = D > 2 ? row / 3 : 0;
      R* S = Sr[row];
      S[0] = S[1] = S[2] = R(0);
      if (SH == 1 && ((D > 1 && cy == 0) || (D > 2 && cz == 0))) continue;  // S_1: no weight here
      const int nq = GL<NGL>::n(a.ngl);
#pragma unroll
      for (int q = 0; q < nq; ++q) {
        const R s = sa + len * gx[q];
        const R wq = len * gw[q];
        R wx[3], dwx[3];
        bw<SH>(fs[0] + s * del[0], wx, dwx);
        R wy = R(1), dwy, wz = R(1), dwz;
        if (D > 1) bw1<SH, kShortW<D, R>>(fs[1] + s * del[1], cy, wy, dwy);
        if (D > 2) bw1<SH, kShortW<D, R>>(fs[2] + s * del[2], cz, wz, dwz);
        const R sw = wq * wy * wz;
#pragma unroll
        for (int c = kC0<SH>; c < 3; ++c) S[c] += sw * wx[c];
      }
      if (in) {
        Stencil<D, true> st(a.M, t, jn);
        const int rowoff = st.row(cy, cz);
#pragma unroll
        for (int c = kC0<SH>; c < 3; ++c)
#pragma unroll
          for (int k = 0; k < 3; ++k) Ub[k] += S[c] * ld<D, R, true>(a, t, D + 6 + k, st.ix[c] + rowoff);
      } else if (has) {
        Stencil<D, false> st(a.M, t, jn);
        const int rowoff = st.row(cy, cz);
#pragma unroll
        for (int c = kC0<SH>; c < 3; ++c) {
          const int g = st.ix[c] + rowoff;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            Ub[k] += S[c] * ld<D, R, false>(a, t, D + 6 + k, g);
            if (do_dep) fix_add(a.J, (int64_t)k * a.M.Ng + g, coef[k] * (double)S[c], a.M.fx.up);
          }
        }
      }
    }
    if (do_dep && t.ok) deposit_window<D, R, NROW>(t, jn, Sr, coef, in, lane);
  }
}

// Workgroup-wide (one wave) min / max of D ints per thread (all threads participate).
template <int D>
__device__ __forceinline__ void block_minmax(int lo[3], int hi[3]) {
  static_assert(kOrbitBlock == 64, "the orbit workgroup is one wave");
#pragma unroll
  for (int l = 0; l < D; ++l) {
    lo[l] = wave_min_i32(lo[l]);
    hi[l] = wave_max_i32(hi[l]);
  }
}

template <int D>
__device__ __forceinline__ int tile_to_global(const Mesh& M, const Tile& t, int nd) {
  const int ux = nd % t.E[0] + t.o[0];
  const int uy = D > 1 ? (nd / t.E[0]) % t.E[1] + t.o[1] : 0;
  const int uz = D > 2 ? nd / (t.E[0] * t.E[1]) + t.o[2] : 0;
  return wrapi(ux, M.n[0]) + M.n[0] * ((D > 1 ? wrapi(uy, M.n[1]) : 0) + M.n[1] * (D > 2 ? wrapi(uz, M.n[2]) : 0));
}

// Occupancy target (waves per SIMD) the register allocator works to, chosen per
// instantiation by measurement: 1D at its least exact Gauss-Legendre order runs short
// launches whose time is latency, and fits three waves in FP64 and four in FP32 without
// spilling; the other FP32 kernels of 1D and 2D fit three with little spilling; 2D FP64,
// 3D and the other 1D FP64 kernels run best at two.
template <int D, int SH, int NGL, class R>
constexpr int orbit_waves() {
  const bool fp32 = sizeof(R) == 4;
  if (D == 1 && NGL == (SH == 1 ? 1 : 2)) return fp32 ? 4 : 3;
  return (fp32 && D <= 2) ? 3 : 2;
}

// dynamic LDS of one orbit-pass workgroup: the tile, then the park block
template <int D, int SH, int NGL, class R>
constexpr int orbit_lds() {
  return tile_bytes<D>() + (orbit_park<D, SH, NGL, R>() ? kParkVals * 64 * 8 : 0);
}

// REF: refinement is on (a.rstate set); the kernel then hands the particles whose
// full-step solve fails, and those refined earlier in the step, to the refinement pass.
template <int D, int SH, int NGL, class R, bool REF>
__global__ __launch_bounds__(kOrbitBlock)
__attribute__((amdgpu_waves_per_eu(orbit_waves<D, SH, NGL, R>()))) void k_orbit(OrbitArgs a) {
  if (a.stop && *a.stop) return;  // the outer iteration this pass belongs to is done
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const Mesh& M = a.M;
  const int64_t ps = a.ps;
  HIP_DYNAMIC_SHARED(double, s_dyn);
  constexpr int NF = nfields<D>();
  constexpr bool kPark = orbit_park<D, SH, NGL, R>();
  constexpr int kParkBase = tile_bytes<D>() / 8;  // the park block follows the tile
  const R* Pp = static_cast<const R*>(a.P);
  const R* qp = static_cast<const R*>(a.q);
  const R* vinp = static_cast<const R*>(a.vin);
  R* vp = static_cast<R*>(a.v);
  R* Pnp = static_cast<R*>(a.Pn);

  // ---- particle position: nearest node j0 (wrapped into [0, n)) and offset f0
  double x[3] = {0.0, 0.0, 0.0};
  int j0[3] = {0, 0, 0};
  R f0[3] = {R(0), R(0), R(0)};
  bool valid = i < a.np;
  if (valid) {
#pragma unroll
    for (int l = 0; l < D; ++l) {
      x[l] = a.x[l * ps + i];
      const double xi = (x[l] - M.lo[l]) * M.inv_h[l];
      valid = valid && isfinite(xi) && fabs(xi) < 1.0e8;
      const double jr = valid ? floor(xi + 0.5) : 0.0;
      j0[l] = valid ? wrapi((int)jr, M.n[l]) : 0;
      f0[l] = valid ? (R)(xi - jr) : R(0);
    }
  }
  // the particle's own inputs are read up front, so their latency overlaps the setup
  const bool live = i < a.np;
  R qv = R(0), vin0[3] = {R(0), R(0), R(0)}, P0[3] = {R(0), R(0), R(0)};
  if (live) {
    qv = qp[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      vin0[c] = vinp[c * ps + i];
      P0[c] = Pp[c * ps + i];
    }
  }
  // ---- the workgroup's tile box, taken periodically: on an axis whose nodes spread
  // over more than half the mesh, the low side moves up by one period, so particles
  // on either side of the periodic seam become neighbours
  Tile t;
  int nodes = 1, ok = 1;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    t.o[l] = 0;
    t.E[l] = 1;
  }
  int lo[3], hi[3];
#pragma unroll
  for (int l = 0; l < D; ++l) {
    lo[l] = valid ? j0[l] : INT_MAX;
    hi[l] = valid ? j0[l] : INT_MIN;
  }
  block_minmax<D>(lo, hi);
  int shift = 0;
#pragma unroll
  for (int l = 0; l < D; ++l)
    if (lo[l] <= hi[l] && hi[l] - lo[l] > M.n[l] / 2) shift |= 1 << l;
  if (uni(shift)) {
#pragma unroll
    for (int l = 0; l < D; ++l) {
      if (((shift >> l) & 1) && valid && j0[l] < M.n[l] / 2) j0[l] += M.n[l];
      lo[l] = valid ? j0[l] : INT_MAX;
      hi[l] = valid ? j0[l] : INT_MIN;
    }
    block_minmax<D>(lo, hi);
  }
  // The box covers every particle's node and the node of its orbit endpoint under the
  // warm-start velocity, plus the stencil reach.  Later inner iterates move the orbit
  // little; a segment whose stencil still leaves the box takes the global path.
  const bool any_valid = uni(lo[0] <= hi[0] ? 1 : 0) != 0;
  if (any_valid) {
#pragma unroll
    for (int l = 0; l < D; ++l) {
      int je = j0[l];
      const double del = a.dt * (double)vin0[l] * M.inv_h[l];
      if (valid && fabs(del) < (double)kMaxCross) je = j0[l] + (int)floor((double)f0[l] + del + 0.5);
      lo[l] = valid ? min(j0[l], je) : INT_MAX;
      hi[l] = valid ? max(j0[l], je) : INT_MIN;
    }
    block_minmax<D>(lo, hi);
  }
#pragma unroll
  for (int l = 0; l < D; ++l) {
    if (lo[l] > hi[l]) {  // no valid particle in this workgroup
      ok = 0;
    } else {
      // S_1 bases its stencil on the node below the point, which can lie one node
      // under the nearest: the box reaches one node further down
      t.o[l] = uni(lo[l] - kHalo - (SH == 1 ? 1 : 0));
      const int e = hi[l] - lo[l] + 1 + 2 * kHalo + (SH == 1 ? 1 : 0);
      t.E[l] = uni(e);
      nodes = (e > 4096 || nodes > 4096) ? (1 << 30) : nodes * e;  // no overflow: 4096^2 < 2^30
    }
  }
  // field tile in R, then the FP64 current tile at an 8-byte boundary, then the tile
  // nodes' mesh indices (int32; the mesh has at most 2^30 nodes)
  const int64_t fbytes = ((int64_t)nodes * NF * (int64_t)sizeof(R) + 7) / 8 * 8;
  if (ok && fbytes + (int64_t)nodes * (3 * 8 + 4) > tile_bytes<D>()) ok = 0;
  t.nodes = uni(nodes);
  t.ok = uni(ok);
  t.joff = uni((int)(fbytes / 8));
  t.goff = uni((int)(fbytes / 4) + 6 * nodes);
  if (t.ok) {
    // one tile node per lane at a time: its mesh index is computed once for all fields
    // and kept for the flush
    R* s_tile = reinterpret_cast<R*>(s_dyn);
    double* s_J = s_dyn + t.joff;
    int* s_g = reinterpret_cast<int*>(s_dyn) + t.goff;
    for (int nd = threadIdx.x; nd < t.nodes; nd += blockDim.x) {
      const int g = tile_to_global<D>(M, t, nd);
      s_g[nd] = g;
#pragma unroll
      for (int f = 0; f < NF; ++f) s_tile[f * t.nodes + nd] = (R)gfield<D>(a, f)[g];
#pragma unroll
      for (int c = 0; c < 3; ++c) s_J[c * t.nodes + nd] = 0.0;
    }
  }
  __syncthreads();

  // Gauss-Legendre nodes and weights on [0, 1]
  constexpr int NQ = NGL > 0 ? NGL : kMaxGL;
  R gx[NQ], gw[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    gx[k] = (R)a.glx[k];
    gw[k] = (R)a.glw[k];
  }

  double part[kOrbitParts];
#pragma unroll
  for (int v = 0; v < kOrbitParts; ++v) part[v] = 0.0;
  // state the deposit phase needs from the accepted evaluation
  bool conv = false;
  R vin[3] = {R(0), R(0), R(0)};
  R q = R(0);
  // of the accepted evaluation: v_out, the chain-rule part w = (A^+ - A^-) - dt D v_in
  // (the residual R_A once dt U-bar is subtracted), the work part -v_out . grad-phi-bar and
  // the kinetic energy of p^{n+1}
  double vout[3] = {0.0, 0.0, 0.0}, wra[3] = {0.0, 0.0, 0.0};
  double wgp = 0.0, kin = 0.0;
  // with refinement, a particle already refined earlier in the step skips the full step
  const bool solve = live && !(REF && (a.rstate[i] & 0xff) != 0);
  if (solve) {
    PConst<R> pc;
    pc.q = qv;
    q = pc.q;
    vin[0] = vin0[0];
    vin[1] = vin0[1];
    vin[2] = vin0[2];
    R Am[3] = {R(0), R(0), R(0)};
    if (valid) interp3<D, SH, R>(a, t, D, j0, f0, Am);
    {
      R u2 = R(0);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const R u = (P0[c] - pc.q * Am[c]) * rcp_(fabs(pc.q) * R(a.kappa));
        u2 += u * u;
      }
      pc.gpn = sqrt_(R(1) + u2);
    }
    if (kPark) park_store<R>(kParkBase + (int)threadIdx.x, P0, Am, pc);
    int it = 0, segs = 0;
    bool xlim = false;  // the orbit reached the supported knot-crossing range
    const int maxit = a.iterate ? a.max_inner : 1;
    const R kap2 = R(a.kappa) * R(a.kappa);
    const R P[3] = {P0[0], P0[1], P0[2]};
    for (it = 1; it <= maxit; ++it) {
      // the orbit must stay finite and within the supported knot-crossing range
      const R vn2 = vin[0] * vin[0] + vin[1] * vin[1] + vin[2] * vin[2];
      bool okv = valid && isfinite(vn2);
      bool inr = true;
#pragma unroll
      for (int l = 0; l < D; ++l) inr = inr && fabs(R(a.dt) * vin[l] * R(M.inv_h[l])) < R(kMaxCross - 1);
      xlim = okv && !inr;
      if (!okv || !inr) break;
      EvalOut<R> o;
      evaluate<D, SH, NGL, R, kPark>(a, t, gx, gw, j0, f0, P, pc, Am, vin, o, kParkBase + (int)threadIdx.x);
      segs += o.nseg;
      const R vo2 = o.vout[0] * o.vout[0] + o.vout[1] * o.vout[1] + o.vout[2] * o.vout[2];
      if (!isfinite(vo2) || !(vo2 < kap2)) break;  // finite and subluminal
      R dmax = R(0), vmax = R(0);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        dmax = fmax(dmax, fabs(o.vout[c] - vin[c]));
        vmax = fmax(vmax, fabs(o.vout[c]));
      }
      if (!a.iterate || dmax <= R(a.tol_abs) + R(a.tol_rel) * vmax) {
        // converged: store the new state; the orbit of this v_in is deposited below
        conv = true;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          double d = 0.0;
#pragma unroll
          for (int j = 0; j < D; ++j) d += (double)o.Dm[c][j] * (double)vin[j];
          wra[c] = (kPark ? (double)o.dA[c] : (double)o.Ap[c] - (double)Am[c]) - a.dt * d;
          vout[c] = (double)o.vout[c];
          wgp -= vout[c] * (double)o.gp[c];
        }
        const double m = fabs(kPark ? s_dyn[kParkBase + threadIdx.x + 64 * 6] : (double)pc.q);
        const double p2 = (double)o.pn1[0] * o.pn1[0] + (double)o.pn1[1] * o.pn1[1] + (double)o.pn1[2] * o.pn1[2];
        const double gmm = sqrt(1.0 + p2 / (m * m * a.kappa * a.kappa));
        kin = p2 / (m * (gmm + 1.0));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          vp[c * ps + i] = o.vout[c];
          Pnp[c * ps + i] = o.Pn1[c];
        }
#pragma unroll
        for (int l = 0; l < D; ++l) a.xn[l * ps + i] = wrap_pos(a.x[l * ps + i] + a.dt * (double)vin[l], M.lo[l], M.len[l]);
        break;
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) vin[c] = o.vout[c];
    }
    if (it > maxit) it = maxit;
    if (a.iters) a.iters[i] = it;
    // with refinement a failed full step is handed to the refinement pass, with the
    // evaluations it took
    const bool refine = REF && !conv;
    if (refine) a.rstate[i] = (it << 8) | 1;
    part[OP_FAIL] = (conv || refine) ? 0.0 : 1.0;
    part[OP_ITERS] = (double)it;
    part[OP_ITMAX] = (double)it;
    part[OP_SEGS] = (double)segs;
    part[OP_XLIM] = (!conv && !refine && xlim) ? 1.0 : 0.0;
  }
  if (REF) {  // flag the workgroup for the refinement pass (its skipped and failed particles)
    const uint64_t need = __ballot(live && !conv);
    if (threadIdx.x == 0) a.rblock[blockIdx.x] = need != 0 ? 1 : 0;
  }

  // ---- deposit phase (every lane of the workgroup, converged particles contribute)
  {
    R del[3] = {R(0), R(0), R(0)};
    double coef[3] = {0.0, 0.0, 0.0};
    if (conv) {
#pragma unroll
      for (int l = 0; l < D; ++l) del[l] = R(a.dt) * vin[l] * R(M.inv_h[l]);
      const double qv = (double)q / M.dV;
#pragma unroll
      for (int c = 0; c < 3; ++c) coef[c] = qv * vout[c];
    }
    R Ub[3];
    deposit_phase<D, SH, NGL, R>(a, t, gx, gw, j0, f0, del, conv, coef, Ub);
    if (conv) {
      double wk = 0.0, ra2 = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double r = wra[c] - a.dt * (double)Ub[c];
        ra2 += r * r;
        wk -= vout[c] * (double)Ub[c];
      }
      wk += wgp;
      part[OP_KIN] = kin;
      part[OP_WORK] = (double)q * wk;
      part[OP_RA2] = ra2;
    }
  }
  __syncthreads();
  // flush the current tile: one fixed-point addition (two integer atomics) per nonzero
  // tile node and component, so the sum over workgroups does not depend on their order
  if (t.ok && a.deposit) {
    const double* s_J = s_dyn + t.joff;
    const int* s_g = reinterpret_cast<const int*>(s_dyn) + t.goff;
    for (int nd = threadIdx.x; nd < t.nodes; nd += blockDim.x) {
      const double v[3] = {s_J[nd], s_J[t.nodes + nd], s_J[2 * t.nodes + nd]};
      if (v[0] == 0.0 && v[1] == 0.0 && v[2] == 0.0) continue;
      const int64_t g = s_g[nd];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (v[c] != 0.0) fix_add(a.J, (int64_t)c * M.Ng + g, v[c], M.fx.up);
    }
  }
  // workgroup (one wave) reduction in a fixed order: the sums by one reduce-scatter (the
  // lane that ends up holding a total stores it), the maximum by a DPP maximum
  static_assert(kOrbitParts <= 16 && kOrbitBlock == 64, "one reduce-scatter of 16 over one wave");
  double v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = (k < kOrbitParts && k != OP_ITMAX) ? part[k] : 0.0;
  const int lane = threadIdx.x;
  const double tot = wave_reduce_scatter<16>(v, lane);
  const double itmax = wave_reduce_f64<true>(part[OP_ITMAX]);
  const int idx = wave_slot<16>(lane);
  if (wave_owner<16>(lane) && idx < kOrbitParts)
    a.partials[(int64_t)idx * a.pstride + blockIdx.x] = idx == OP_ITMAX ? itmax : tot;
}

// ---- refinement pass (convergence-triggered particle refinement of the spline-degree
// comparison in the results section)
//
// A particle whose full-step solve failed, in this pass or earlier in the step, is solved
// with K = 2^L equal particle sub-steps of dt/K, for L = its level, ... refine_levels (the
// level rises when a sub-step solve fails).  Sub-step k is the full-step map with dt/K and
// the vector potential of the step at the fractions k/K and (k+1)/K of it,
// A(s) = (1 - s) A^n + s A^{n+1} (the interpolant the orbit discrete gradient uses),
// grad phi^{n+1/2} and U^{n+1/2} unchanged; it starts where the previous one ended, from
// the previous v_out.  The particle deposits the mean of its sub-step orbit currents,
// (1/K) sum_k q v_out,k S-bar_k / dV, which keeps the particle work of the sub-steps equal
// to the mesh work of the deposit; its accepted orbit velocity is the mean of the sub-step
// v_out.  Rare work: one wave per flagged workgroup of the main pass (one lane per
// particle), fields from global memory, fixed-point deposits straight to the accumulator.

// Nearest node j0 (wrapped into [0, n)) and offset f0 of position x, as the main pass
// takes them; false for a non-finite or far-off position.
template <int D, class R>
__device__ __forceinline__ bool locate(const Mesh& M, const double x[3], int j0[3], R f0[3]) {
  bool ok = true;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    j0[l] = 0;
    f0[l] = R(0);
  }
#pragma unroll
  for (int l = 0; l < D; ++l) {
    const double xi = (x[l] - M.lo[l]) * M.inv_h[l];
    ok = ok && isfinite(xi) && fabs(xi) < 1.0e8;
    const double jr = ok ? floor(xi + 0.5) : 0.0;
    j0[l] = ok ? wrapi((int)jr, M.n[l]) : 0;
    f0[l] = ok ? (R)(xi - jr) : R(0);
  }
  return ok;
}

// A(j / 2^refine_levels): A^n, A^{n+1}, or an interpolant of the potentials pass.
__device__ __forceinline__ const double* sub_potential(const OrbitArgs& a, int j) {
  if (j == 0) return a.An;
  if (j == (1 << a.refine_levels)) return a.Anp1;
  return a.Ab + (int64_t)(j - 1) * 3 * a.M.Ng;
}

// The refinement of the particles of main-pass workgroup b (all 64 lanes call it).
template <int D, int SH, int NGL, class R>
__device__ void refine_block(const OrbitArgs& a, int64_t b, int lane, const R* gx, const R* gw) {
  const Mesh& M = a.M;
  const int64_t ps = a.ps;
  const int64_t i = b * kOrbitBlock + lane;
  const int st = i < a.np ? a.rstate[i] : 0;
  int lv = st & 0xff;
  const int ev0 = st >> 8;  // evaluations of a failed full-step attempt in this pass
  const bool act = lv > 0;
  const R* Pp = static_cast<const R*>(a.P);
  const R* qp = static_cast<const R*>(a.q);
  const R* vinp = static_cast<const R*>(a.vin);
  R q = R(0), P0[3] = {R(0), R(0), R(0)}, w0[3] = {R(0), R(0), R(0)};
  double x0[3] = {0.0, 0.0, 0.0};
  if (act) {
    q = qp[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      P0[c] = Pp[c * ps + i];
      w0[c] = vinp[c * ps + i];
    }
#pragma unroll
    for (int l = 0; l < D; ++l) x0[l] = a.x[l * ps + i];
  }
  Tile t;  // no LDS tile: every gather and deposit goes through global memory
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    t.o[l] = 0;
    t.E[l] = 1;
  }
  t.nodes = 0;
  t.ok = 0;
  t.joff = 0;
  t.goff = 0;

  // per sub-step of the accepted level: v_in, v_out, the chain-rule part
  // (A^+ - A^-) - dt_k D v_in and -v_out . grad-phi-bar
  constexpr int KM = 1 << kMaxRefine;
  R svin[KM][3];
  double svout[KM][3], swra[KM][3], swgp[KM];
  bool ok = false, xlim = false;
  int evals = 0, segs = 0, K = 1;
  double kin = 0.0, xend[3] = {0.0, 0.0, 0.0};
  R Pend[3] = {R(0), R(0), R(0)};
  const R kap2 = R(a.kappa) * R(a.kappa);
  for (int L = 1; L <= a.refine_levels; ++L) {
    const bool run = act && !ok && lv <= L;
    if (__ballot(run) == 0) continue;
    const int KL = 1 << L;
    const int stride = (1 << a.refine_levels) >> L;
    OrbitArgs as = a;
    as.dt = a.dt / KL;
    double xk[3] = {x0[0], x0[1], x0[2]};
    R Pk[3] = {P0[0], P0[1], P0[2]}, warm[3] = {w0[0], w0[1], w0[2]};
    bool okL = run;
    xlim = false;
    for (int k = 0; k < KL; ++k) {
      as.An = sub_potential(a, k * stride);
      as.Anp1 = sub_potential(a, (k + 1) * stride);
      if (!okL) continue;
      int j0[3];
      R f0[3];
      const bool valid = locate<D, R>(M, xk, j0, f0);
      R Am[3] = {R(0), R(0), R(0)};
      if (valid) interp3<D, SH, R>(as, t, D, j0, f0, Am);
      PConst<R> pc;
      pc.q = q;
      {
        R u2 = R(0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const R u = (Pk[c] - q * Am[c]) * rcp_(fabs(q) * R(a.kappa));
          u2 += u * u;
        }
        pc.gpn = sqrt_(R(1) + u2);
      }
      R vin[3] = {warm[0], warm[1], warm[2]};
      bool conv = false;
      for (int it = 1; it <= a.max_inner; ++it) {
        const R vn2 = vin[0] * vin[0] + vin[1] * vin[1] + vin[2] * vin[2];
        const bool okv = valid && isfinite(vn2);
        bool inr = true;
#pragma unroll
        for (int l = 0; l < D; ++l) inr = inr && fabs(R(as.dt) * vin[l] * R(M.inv_h[l])) < R(kMaxCross - 1);
        xlim = okv && !inr;
        if (!okv || !inr) break;
        EvalOut<R> o;
        evaluate<D, SH, NGL, R>(as, t, gx, gw, j0, f0, Pk, pc, Am, vin, o);
        ++evals;
        segs += o.nseg;
        const R vo2 = o.vout[0] * o.vout[0] + o.vout[1] * o.vout[1] + o.vout[2] * o.vout[2];
        if (!isfinite(vo2) || !(vo2 < kap2)) break;  // finite and subluminal
        R dmax = R(0), vmax = R(0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          dmax = fmax(dmax, fabs(o.vout[c] - vin[c]));
          vmax = fmax(vmax, fabs(o.vout[c]));
        }
        if (dmax <= R(a.tol_abs) + R(a.tol_rel) * vmax) {
          conv = true;
          double wg = 0.0;
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            double d = 0.0;
#pragma unroll
            for (int j = 0; j < D; ++j) d += (double)o.Dm[c][j] * (double)vin[j];
            svin[k][c] = vin[c];
            svout[k][c] = (double)o.vout[c];
            swra[k][c] = ((double)o.Ap[c] - (double)Am[c]) - as.dt * d;
            wg -= svout[k][c] * (double)o.gp[c];
            Pk[c] = o.Pn1[c];
            warm[c] = o.vout[c];
          }
          swgp[k] = wg;
#pragma unroll
          for (int l = 0; l < D; ++l) xk[l] = xk[l] + as.dt * (double)vin[l];
          if (k == KL - 1) {
            const double m = fabs((double)q);
            const double p2 =
                (double)o.pn1[0] * o.pn1[0] + (double)o.pn1[1] * o.pn1[1] + (double)o.pn1[2] * o.pn1[2];
            const double gmm = sqrt(1.0 + p2 / (m * m * a.kappa * a.kappa));
            kin = p2 / (m * (gmm + 1.0));
          }
          break;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) vin[c] = o.vout[c];
      }
      okL = conv;
    }
    if (run && okL) {
      ok = true;
      K = KL;
      lv = L;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        xend[c] = xk[c];
        Pend[c] = Pk[c];
      }
    } else if (run) {
      lv = L + 1;
    }
  }

  // deposit of the accepted sub-steps, with the U-bar gathers of the diagnostics
  double ra2 = 0.0, wk = 0.0;
  {
    double xd[3] = {x0[0], x0[1], x0[2]};
    const double dtK = a.dt / K;
    for (int k = 0; k < (1 << a.refine_levels); ++k) {
      const bool dep = ok && k < K;
      if (__ballot(dep) == 0) break;
      int j0[3] = {0, 0, 0};
      R f0[3] = {R(0), R(0), R(0)}, del[3] = {R(0), R(0), R(0)};
      double coef[3] = {0.0, 0.0, 0.0};
      if (dep) {
        locate<D, R>(M, xd, j0, f0);
#pragma unroll
        for (int l = 0; l < D; ++l) del[l] = R(dtK) * svin[k][l] * R(M.inv_h[l]);
        const double qv = (double)q / (M.dV * K);
#pragma unroll
        for (int c = 0; c < 3; ++c) coef[c] = qv * svout[k][c];
      }
      R Ub[3];
      deposit_phase<D, SH, NGL, R>(a, t, gx, gw, j0, f0, del, dep, coef, Ub);
      if (dep) {
        double w = swgp[k];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double r = swra[k][c] - dtK * (double)Ub[c];
          ra2 += r * r;
          w -= svout[k][c] * (double)Ub[c];
        }
        wk += w / K;
#pragma unroll
        for (int l = 0; l < D; ++l) xd[l] = xd[l] + dtK * (double)svin[k][l];
      }
    }
  }
  if (act) {
    if (ok) {
      R* vp = static_cast<R*>(a.v);
      R* Pnp = static_cast<R*>(a.Pn);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double vs = 0.0;
        for (int k = 0; k < K; ++k) vs += svout[k][c];
        vp[c * ps + i] = (R)(vs / K);
        Pnp[c * ps + i] = Pend[c];
      }
#pragma unroll
      for (int l = 0; l < D; ++l) a.xn[l * ps + i] = wrap_pos(xend[l], M.lo[l], M.len[l]);
    }
    a.rstate[i] = lv;  // the settled level (refine_levels + 1 after a failure)
    if (a.iters) a.iters[i] = ev0 + evals;
  }
  // the wave's sums join the main pass's partials of workgroup b, in a fixed order
  double part[kOrbitParts];
#pragma unroll
  for (int v = 0; v < kOrbitParts; ++v) part[v] = 0.0;
  if (act) {
    part[OP_FAIL] = ok ? 0.0 : 1.0;
    part[OP_ITERS] = (double)evals;
    part[OP_ITMAX] = (double)(ev0 + evals);
    part[OP_SEGS] = (double)segs;
    part[OP_XLIM] = (!ok && xlim) ? 1.0 : 0.0;
    part[OP_REFINED] = ok ? 1.0 : 0.0;
    if (ok) {
      part[OP_KIN] = kin;
      part[OP_WORK] = (double)q * wk;
      part[OP_RA2] = ra2;
    }
  }
  double v[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) v[k] = (k < kOrbitParts && k != OP_ITMAX) ? part[k] : 0.0;
  const double tot = wave_reduce_scatter<16>(v, lane);
  const double itmax = wave_reduce_f64<true>(part[OP_ITMAX]);
  const int idx = wave_slot<16>(lane);
  if (wave_owner<16>(lane) && idx < kOrbitParts) {
    double* p = a.partials + (int64_t)idx * a.pstride + b;
    *p = idx == OP_ITMAX ? fmax(*p, itmax) : *p + tot;
  }
}

// One wave per workgroup; each takes 64 block flags of the main pass at a time and
// refines the flagged blocks one after another.
template <int D, int SH, int NGL, class R>
__global__ __launch_bounds__(kOrbitBlock) void k_refine(OrbitArgs a, int64_t nblocks) {
  if (a.stop && *a.stop) return;
  const int lane = threadIdx.x;
  constexpr int NQ = NGL > 0 ? NGL : kMaxGL;
  R gx[NQ], gw[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    gx[k] = (R)a.glx[k];
    gw[k] = (R)a.glw[k];
  }
  for (int64_t c0 = (int64_t)blockIdx.x * 64; c0 < nblocks; c0 += (int64_t)gridDim.x * 64) {
    const int64_t bb = c0 + lane;
    uint64_t m = __ballot(bb < nblocks && a.rblock[bb] != 0);
    while (m != 0) {
      const int bit = __ffsll((long long)m) - 1;
      m &= m - 1;
      refine_block<D, SH, NGL, R>(a, c0 + bit, lane, gx, gw);
    }
  }
}

// A(j / kmax) = (1 - s) A^n + s A^{n+1} at the interior fractions j = 1 .. kmax - 1.
__global__ void k_refine_potentials(const double* An, const double* Anp1, double* Ab, int64_t n3, int kmax,
                                    const int32_t* stop) {
  if (stop && *stop) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n3) return;
  const double a0 = An[e], a1 = Anp1[e];
  for (int j = 1; j < kmax; ++j) {
    const double s = (double)j / (double)kmax;
    Ab[(int64_t)(j - 1) * n3 + e] = (1.0 - s) * a0 + s * a1;
  }
}

__global__ void k_refine_reset(int32_t* rstate, int64_t np) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) rstate[i] = 0;
}

template <int D, int SH, int NGL, class R>
hipError_t launch_k(const OrbitArgs& a, unsigned blocks, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  constexpr unsigned kLds = orbit_lds<D, SH, NGL, R>();
  if (!a.rstate) {
    if (e0 || e1)
      hipExtLaunchKernelGGL((k_orbit<D, SH, NGL, R, false>), dim3(blocks), dim3(kOrbitBlock), kLds, s, e0,
                            e1, 0u, a);
    else
      hipLaunchKernelGGL((k_orbit<D, SH, NGL, R, false>), dim3(blocks), dim3(kOrbitBlock), kLds, s, a);
    return hipGetLastError();
  }
  // with refinement: the main pass, the interpolated potentials, the refinement pass (a
  // timed launch spans all three)
  if (e0)
    hipExtLaunchKernelGGL((k_orbit<D, SH, NGL, R, true>), dim3(blocks), dim3(kOrbitBlock), kLds, s, e0,
                          nullptr, 0u, a);
  else
    hipLaunchKernelGGL((k_orbit<D, SH, NGL, R, true>), dim3(blocks), dim3(kOrbitBlock), kLds, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int kmax = 1 << a.refine_levels;
  if (kmax > 1) {
    const int64_t n3 = 3 * a.M.Ng;
    hipLaunchKernelGGL(k_refine_potentials, dim3((unsigned)((n3 + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, a.An,
                       a.Anp1, a.Ab, n3, kmax, a.stop);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int64_t chunks = ((int64_t)blocks + 63) / 64;
  const unsigned rg = (unsigned)(chunks < 2048 ? chunks : 2048);
  if (e1)
    hipExtLaunchKernelGGL((k_refine<D, SH, NGL, R>), dim3(rg), dim3(kOrbitBlock), 0, s, nullptr, e1, 0u, a,
                          (int64_t)blocks);
  else
    hipLaunchKernelGGL((k_refine<D, SH, NGL, R>), dim3(rg), dim3(kOrbitBlock), 0, s, a, (int64_t)blocks);
  return hipGetLastError();
}

template <int D, class R>
hipError_t launch_d(const OrbitArgs& a, unsigned blocks, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  // compile-time Gauss-Legendre orders: the least exact for the per-segment polynomials
  // (d+1 for S_2, ceil((d+1)/2) for S_1) and, for S_2, the paper's 8; any other order
  // runs the runtime loop
  if (a.M.shape == 1) {
    if (a.ngl == (D + 2) / 2) return launch_k<D, 1, (D + 2) / 2, R>(a, blocks, s, e0, e1);
    return launch_k<D, 1, 0, R>(a, blocks, s, e0, e1);
  }
  if (a.ngl == D + 1) return launch_k<D, 2, D + 1, R>(a, blocks, s, e0, e1);
  if (a.ngl == 8) return launch_k<D, 2, 8, R>(a, blocks, s, e0, e1);
  return launch_k<D, 2, 0, R>(a, blocks, s, e0, e1);
}

}  // namespace

hipError_t launch_refine_reset(int32_t* rstate, int64_t np, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_refine_reset, dim3((unsigned)((np + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, rstate, np);
  return hipGetLastError();
}

hipError_t launch_orbit(const OrbitArgs& a, int ngl, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  (void)ngl;
  if (a.np <= 0) {
    hipError_t e = hipSuccess;
    if (e0) e = hipEventRecord(e0, s);
    if (e1 && e == hipSuccess) e = hipEventRecord(e1, s);
    return e;
  }
  const unsigned blocks = (unsigned)((a.np + kOrbitBlock - 1) / kOrbitBlock);
  const bool f32 = a.precision == 1;
  switch (a.M.d) {
    case 1: return f32 ? launch_d<1, float>(a, blocks, s, e0, e1) : launch_d<1, double>(a, blocks, s, e0, e1);
    case 2: return f32 ? launch_d<2, float>(a, blocks, s, e0, e1) : launch_d<2, double>(a, blocks, s, e0, e1);
    case 3: return f32 ? launch_d<3, float>(a, blocks, s, e0, e1) : launch_d<3, double>(a, blocks, s, e0, e1);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace gmhc
