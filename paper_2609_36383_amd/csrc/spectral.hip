// spectral.hip -- periodic spectral field step on the mesh: batched radix-2 FFTs in
// LDS, the mode-by-mode Crank-Nicolson solve of the potential system with continuity
// and the Nyquist projector, the outer residual norms, initialization and the
// spectral diagnostics (section "Mesh-based field values and the Crank-Nicolson
// potential update", the Nyquist-projection paragraph and the constraint diagnostics).
#include <math.h>

#include <algorithm>

#include "gmhc_internal.h"

namespace gmhc {
namespace {

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// i k * a
__device__ __forceinline__ double2 cik(double k, double2 a) { return make_double2(-k * a.y, k * a.x); }

// Signed-index derivative symbol k_l of unshifted index m (zero at the even-grid
// Nyquist index, as the spectral operators of the paper use).
__device__ __forceinline__ double ksym(const Mesh& M, int l, int64_t m) {
  const int n = M.n[l];
  if (l >= M.d) return 0.0;
  if ((n & 1) == 0 && m == n / 2) return 0.0;
  const int64_t ms = (m <= n / 2) ? m : m - n;
  return 2.0 * M_PI * (double)ms / M.len[l];
}

__device__ __forceinline__ void mode_index(const Mesh& M, int64_t g, int64_t idx[3]) {
  idx[0] = g % M.n[0];
  idx[1] = (g / M.n[0]) % M.n[1];
  idx[2] = g / ((int64_t)M.n[0] * M.n[1]);
}

__device__ __forceinline__ bool on_nyquist(const Mesh& M, const int64_t idx[3]) {
  bool r = false;
  for (int l = 0; l < M.d; ++l) r = r || (((M.n[l] & 1) == 0) && idx[l] == M.n[l] / 2);
  return r;
}

// One axis pass of a batched complex FFT.  A workgroup loads T lines of length N
// into LDS in bit-reversed order, runs log2 N radix-2 butterfly stages and writes
// the lines back.  blockIdx.y selects the component.
template <bool IN_REAL, bool OUT_REAL>
__global__ __launch_bounds__(kBlock) void k_fft_axis(const double* src_r, const double2* src_c,
                                                     double2* dst_c, double* dst_r, int64_t Ng,
                                                     FftPlanAxis ax, int inverse, int project,
                                                     Mesh M, const int32_t* stop) {
  if (stop && *stop) return;
  extern __shared__ double2 lds[];
  const int N = ax.N, T = ax.T, logN = ax.logN;  // N and T are powers of two
  const int logT = 31 - __clz(T);
  const int64_t comp = blockIdx.y;
  const int64_t line0 = (int64_t)blockIdx.x * T;
  const int64_t total = (int64_t)T * N;
  const int shift = 32 - logN;
  // twiddles exp(-2 pi i m / N), m < N/2, staged once after the T lines when they fit
  double2* twl = lds + (int64_t)T * N;
  if (ax.lds_tw)
    for (int m = threadIdx.x; m < N / 2; m += blockDim.x) twl[m] = ax.tw[m];
  const double2* tws = ax.lds_tw ? twl : ax.tw;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    int lt, k;
    if (ax.stride == 1) {
      lt = (int)(e >> logN);
      k = (int)(e & (N - 1));
    } else {
      lt = (int)(e & (T - 1));
      k = (int)(e >> logT);
    }
    const int64_t line = line0 + lt;
    double2 v = make_double2(0.0, 0.0);
    if (line < ax.nlines) {
      const int64_t iin = line % ax.stride, iout = line / ax.stride;
      const int64_t addr = comp * Ng + iin + ax.stride * ((int64_t)k + (int64_t)N * iout);
      if (IN_REAL)
        v = make_double2(src_r[addr], 0.0);
      else
        v = src_c[addr];
    }
    const int rk = (N > 1) ? (int)(__brev((unsigned)k) >> shift) : 0;
    lds[lt * N + rk] = v;
  }
  __syncthreads();
  for (int st = 1; st <= logN; ++st) {
    const int half = 1 << (st - 1);
    const int twstep = N >> st;
    for (int b = threadIdx.x; b < T * (N / 2); b += blockDim.x) {
      const int lt = b >> (logN - 1), j = b & (N / 2 - 1);
      const int grp = j >> (st - 1), pos = j & (half - 1);
      const int i1 = lt * N + grp * (2 * half) + pos, i2 = i1 + half;
      double2 w = tws[pos * twstep];
      if (inverse) w.y = -w.y;
      const double2 u = lds[i1];
      const double2 t = cmul(lds[i2], w);
      lds[i1] = cadd(u, t);
      lds[i2] = csub(u, t);
    }
    __syncthreads();
  }
  const double sc = inverse ? 1.0 / (double)N : 1.0;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    int lt, k;
    if (ax.stride == 1) {
      lt = (int)(e >> logN);
      k = (int)(e & (N - 1));
    } else {
      lt = (int)(e & (T - 1));
      k = (int)(e >> logT);
    }
    const int64_t line = line0 + lt;
    if (line >= ax.nlines) continue;
    const int64_t iin = line % ax.stride, iout = line / ax.stride;
    const int64_t g = iin + ax.stride * ((int64_t)k + (int64_t)N * iout);
    double2 v = cscale(lds[lt * N + k], sc);
    if (project) {
      int64_t idx[3];
      mode_index(M, g, idx);
      if (on_nyquist(M, idx)) v = make_double2(0.0, 0.0);
    }
    if (OUT_REAL)
      dst_r[comp * Ng + g] = v.x;
    else
      dst_c[comp * Ng + g] = v;
  }
}

__global__ __launch_bounds__(kBlock) void k_cn(CNArgs a) {
  if (a.stop && *a.stop) return;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const Mesh& M = a.M;
  if (g >= M.Ng) return;
  int64_t idx[3];
  mode_index(M, g, idx);
  const double k[3] = {ksym(M, 0, idx[0]), ksym(M, 1, idx[1]), ksym(M, 2, idx[2])};
  const int64_t Ng = M.Ng;
  const double2 j0 = a.jh[g], j1 = a.jh[Ng + g], j2 = a.jh[2 * Ng + g];
  // continuity: rho^{n+1} = rho^n - dt div_h J^{n+1/2}
  double2 divj = cadd(cadd(cik(k[0], j0), cik(k[1], j1)), cik(k[2], j2));
  const double h = a.dt;
  const double2 rho0 = a.rho[g];
  const double2 rho1 = csub(rho0, cscale(divj, h));
  const double2 rhoh = cscale(cadd(rho0, rho1), 0.5);
  const double av = a.kappa2 * (k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
  const double q4 = 0.25 * h * h * av;
  const double inv_den = 1.0 / (1.0 + q4);
  const double c1 = 1.0 - q4;
  const double src1 = 0.5 * h * h * a.kappa2 * a.sigma1;
  const double src2 = 0.5 * h * h * a.kappa2 * a.sigma2;
  // (phi, psi): phi^{n+1} from the CN pair with psi eliminated
  const double2 ph0 = a.phi[g], ps0 = a.psi[g];
  const double2 ph1 = cscale(cadd(cadd(cscale(ph0, c1), cscale(ps0, h)), cscale(rhoh, src1)), inv_den);
  const double2 ps1 = csub(cscale(csub(ph1, ph0), 2.0 / h), ps0);
  a.rho1[g] = rho1;
  a.phi1[g] = ph1;
  a.psi1[g] = ps1;
  const double2 phh = cscale(cadd(ph0, ph1), 0.5);
  int o = 0;
  for (int l = 0; l < M.d; ++l) a.out[(int64_t)(o++) * Ng + g] = cik(k[l], phh);
  const double2 jj[3] = {j0, j1, j2};
  for (int c = 0; c < 3; ++c) {
    const double2 A0 = a.A[c * Ng + g], U0 = a.U[c * Ng + g];
    const double2 A1 = cscale(cadd(cadd(cscale(A0, c1), cscale(U0, h)), cscale(jj[c], src2)), inv_den);
    const double2 U1 = csub(cscale(csub(A1, A0), 2.0 / h), U0);
    a.A1[c * Ng + g] = A1;
    a.U1[c * Ng + g] = U1;
    a.out[(int64_t)(M.d + c) * Ng + g] = A1;
    a.out[(int64_t)(M.d + 3 + c) * Ng + g] = cscale(cadd(U0, U1), 0.5);
  }
}

template <int NV>
__device__ __forceinline__ void block_store(double (&part)[NV], uint32_t max_mask, double* out) {
#pragma unroll
  for (int v = 0; v < NV; ++v)
    for (int off = 32; off > 0; off >>= 1) {
      const double o2 = __shfl_xor(part[v], off, 64);
      part[v] = ((max_mask >> v) & 1u) ? fmax(part[v], o2) : part[v] + o2;
    }
  __shared__ double sh[kBlock / 64][NV];
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0)
#pragma unroll
    for (int v = 0; v < NV; ++v) sh[wave][v] = part[v];
  __syncthreads();
  if (threadIdx.x < NV) {
    const int v = threadIdx.x;
    double acc = sh[0][v];
    for (int w = 1; w < (int)(blockDim.x / 64); ++w)
      acc = ((max_mask >> v) & 1u) ? fmax(acc, sh[w][v]) : acc + sh[w][v];
    out[(int64_t)blockIdx.x * NV + v] = acc;
  }
}

// Outer residual r = H(j) - j: sums of |r|^2, |H|^2, |j|^2, the max-node test ratio,
// and the mesh work sum_g H . E^{n+1/2} (E^{n+1/2} = -grad phi^{n+1/2} - U^{n+1/2}).
__global__ __launch_bounds__(kBlock) void k_residual(ResidualArgs a) {
  if (a.stop && *a.stop) return;
  double part[kResParts];
#pragma unroll
  for (int v = 0; v < kResParts; ++v) part[v] = 0.0;
  const int64_t Ng = a.M.Ng;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < Ng;
       g += (int64_t)gridDim.x * blockDim.x) {
    double r2 = 0.0, h2 = 0.0, j2 = 0.0, w = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double H = a.H[c * Ng + g], j = a.j[c * Ng + g];
      const double r = H - j;
      r2 += r * r;
      h2 += H * H;
      j2 += j * j;
      const double gp = (c < a.M.d) ? a.gphi[c * Ng + g] : 0.0;
      w += H * (-gp - a.Uh[c * Ng + g]);
    }
    part[0] += r2;
    part[1] += h2;
    part[2] += j2;
    part[3] = fmax(part[3], sqrt(r2) / (a.tol_abs + 0.5 * a.tol_rel * (sqrt(h2) + sqrt(j2))));
    part[4] += w;
  }
  block_store<kResParts>(part, 1u << 3, a.partials);
}

__global__ __launch_bounds__(kBlock) void k_reduce(const double* partials, int nblocks, int64_t bstride,
                                                   int64_t vstride, int nvals, uint32_t max_mask, double* out,
                                                   const int32_t* stop) {
  if (stop && *stop) return;
  // One workgroup per value.  Thread t folds blocks t, t + 256, ... into eight
  // independent accumulators (so eight loads are in flight), combines them in a fixed
  // order, then a fixed pairwise tree combines the threads: the result depends only
  // on nblocks.
  const int v = blockIdx.x;
  if (v >= nvals) return;
  const bool mx = (max_mask >> v) & 1u;
  const double id = mx ? -INFINITY : 0.0;
  const double* p = partials + (int64_t)v * vstride;
  double a8[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a8[k] = id;
  const int step = (int)blockDim.x;
  int b = threadIdx.x;
  for (; b + 7 * step < nblocks; b += 8 * step) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const double x = p[(int64_t)(b + k * step) * bstride];
      a8[k] = mx ? fmax(a8[k], x) : a8[k] + x;
    }
  }
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const int bb = b + k * step;
    if (bb < nblocks) {
      const double x = p[(int64_t)bb * bstride];
      a8[k] = mx ? fmax(a8[k], x) : a8[k] + x;
    }
  }
  double acc = a8[0];
#pragma unroll
  for (int k = 1; k < 8; ++k) acc = mx ? fmax(acc, a8[k]) : acc + a8[k];
  __shared__ double sh[kBlock];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kBlock / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      const double o = sh[threadIdx.x + h];
      sh[threadIdx.x] = mx ? fmax(sh[threadIdx.x], o) : sh[threadIdx.x] + o;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = sh[0];
}

__global__ __launch_bounds__(kBlock) void k_zero(double* y, int64_t n, const int32_t* stop) {
  if (stop && *stop) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = 0.0;
}

__global__ void k_outer_test(const double* res, int koff, int32_t* ctl, double* acc, int k, double n3,
                             double tol_abs, double tol_rel) {
  if (threadIdx.x != 0 || ctl[0]) return;
  const double* h = res;
  const double* r = res + koff;
  acc[0] += h[OP_ITERS];
  acc[1] += h[OP_SEGS];
  acc[2] = h[OP_ITMAX];
  acc[3] += 1.0;
  acc[10] = h[OP_ITERS];
  if (h[OP_FAIL] > 0.0) {
    acc[4] = h[OP_FAIL];
    ctl[1] = 1;
    ctl[2] = k;
    ctl[0] = 1;
    return;
  }
  const double rr = sqrt(r[0] / n3) / (tol_abs + 0.5 * tol_rel * (sqrt(r[1] / n3) + sqrt(r[2] / n3)));
  const double mr = r[3];
  acc[5] = rr;
  acc[6] = mr;
  if (rr <= 1.0 && mr <= 1.0) {
    acc[7] = h[OP_RA2];
    acc[8] = h[OP_WORK];
    acc[9] = r[4];
    ctl[2] = k;
    ctl[0] = 1;
  }
}

// y = a x + b z over n values (outer-solver vector updates).
__global__ __launch_bounds__(kBlock) void k_axpbz(double* y, double a, const double* x, double b, const double* z,
                                                  int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + (z ? b * z[i] : 0.0);
}

// Pairwise dot products of K <= kMaxDotVecs vectors of length n: partial sums per block
// of the upper triangle (a <= b) in row order, for the fixed-order reduction.
__global__ __launch_bounds__(kBlock) void k_dots(DotArgs a) {
  double part[kMaxDots];
#pragma unroll
  for (int v = 0; v < kMaxDots; ++v) part[v] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * blockDim.x) {
    double x[kMaxDotVecs];
#pragma unroll
    for (int k = 0; k < kMaxDotVecs; ++k) x[k] = k < a.K ? a.v[k][i] : 0.0;
    int p = 0;
#pragma unroll
    for (int k1 = 0; k1 < kMaxDotVecs; ++k1)
#pragma unroll
      for (int k2 = k1; k2 < kMaxDotVecs; ++k2) part[p++] += x[k1] * x[k2];
  }
  block_store<kMaxDots>(part, 0u, a.partials);
}

__global__ void k_axpy2(double* y, const double* x, double2* yc, const double2* xc, double beta,
                        int64_t nreal, int64_t ncplx, const int32_t* stop) {
  if (stop && *stop) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nreal) y[i] += beta * (x[i] - y[i]);
  if (i < ncplx) {
    double2 a = yc[i], b = xc[i];
    yc[i] = make_double2(a.x + beta * (b.x - a.x), a.y + beta * (b.y - a.y));
  }
}

// ---- initialization --------------------------------------------------------------

__device__ __forceinline__ int wrapi(int i, int n) {
  int r = i % n;
  return r < 0 ? r + n : r;
}

__device__ __forceinline__ void pw(double xi, int n, int gi[3], double w[3]) {
  if (!(xi > -1.0e9 && xi < 1.0e9)) xi = 0.0;  // non-finite positions map to a valid node
  const int j = (int)floor(xi + 0.5);
  const double f = xi - (double)j;
  const double a = 0.5 - f, b = 0.5 + f;
  w[0] = 0.5 * a * a;
  w[1] = 0.75 - f * f;
  w[2] = 0.5 * b * b;
  for (int c = 0; c < 3; ++c) gi[c] = wrapi(j + c - 1, n);
}

// Point-shape stencil of a particle: up to 27 (node, weight) pairs.
__device__ __forceinline__ int point_stencil(const Mesh& M, const double* const* x, int64_t i,
                                             int64_t* nodes, double* wts) {
  int gi[3][3];
  double w[3][3];
  for (int l = 0; l < 3; ++l) {
    if (l < M.d) {
      pw((x[l][i] - M.lo[l]) * M.inv_h[l], M.n[l], gi[l], w[l]);
    } else {
      gi[l][0] = 0;
      w[l][0] = 1.0;
    }
  }
  const int NX = 3, NY = M.d > 1 ? 3 : 1, NZ = M.d > 2 ? 3 : 1;
  int cnt = 0;
  for (int cz = 0; cz < NZ; ++cz)
    for (int cy = 0; cy < NY; ++cy)
      for (int cx = 0; cx < NX; ++cx) {
        nodes[cnt] = gi[0][cx] + (int64_t)M.n[0] * (gi[1][cy] + (int64_t)M.n[1] * gi[2][cz]);
        wts[cnt] = w[0][cx] * w[1][cy] * w[2][cz];
        ++cnt;
      }
  return cnt;
}

__global__ __launch_bounds__(kBlock) void k_init_deposit(InitArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.np) return;
  const double q = ld_bulk(a.q, i, a.prec), m = fabs(q);
  const double p[3] = {ld_bulk(a.P[0], i, a.prec), ld_bulk(a.P[1], i, a.prec), ld_bulk(a.P[2], i, a.prec)};
  const double imk = 1.0 / (m * a.kappa);
  const double g = sqrt(1.0 + (p[0] * p[0] + p[1] * p[1] + p[2] * p[2]) * imk * imk);
  double v[3];
  for (int c = 0; c < 3; ++c) {
    v[c] = p[c] / (m * g);
    st_bulk(a.v[c], i, v[c], a.prec);
  }
  int64_t nodes[27];
  double wts[27];
  const int cnt = point_stencil(a.M, a.x, i, nodes, wts);
  const double qd = q / a.M.dV;
  for (int k = 0; k < cnt; ++k) {
    atomicAdd(a.rho + nodes[k], qd * wts[k]);
    for (int c = 0; c < 3; ++c) atomicAdd(a.J[c] + nodes[k], qd * v[c] * wts[k]);
  }
}

// Spectral initialization: neutralizing background (k = 0 charge removed), Nyquist
// projection, phi from Gauss's law |k|^2 phi = sigma1 rho + i k . U, psi = -kappa^2 i k . A.
__global__ __launch_bounds__(kBlock) void k_init_spectral(InitSpecArgs a) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const Mesh& M = a.M;
  if (g >= M.Ng) return;
  const int64_t Ng = M.Ng;
  int64_t idx[3];
  mode_index(M, g, idx);
  const bool kill = a.project && on_nyquist(M, idx);
  if (g == 0) a.rho[0] = make_double2(0.0, 0.0);
  if (kill) {
    a.rho[g] = make_double2(0.0, 0.0);
    for (int c = 0; c < 3; ++c) {
      a.A[c * Ng + g] = make_double2(0.0, 0.0);
      a.U[c * Ng + g] = make_double2(0.0, 0.0);
      a.J[c * Ng + g] = make_double2(0.0, 0.0);
    }
  }
  const double k[3] = {ksym(M, 0, idx[0]), ksym(M, 1, idx[1]), ksym(M, 2, idx[2])};
  double2 divU = make_double2(0.0, 0.0), divA = make_double2(0.0, 0.0);
  for (int c = 0; c < 3; ++c) {
    divU = cadd(divU, cik(k[c], a.U[c * Ng + g]));
    divA = cadd(divA, cik(k[c], a.A[c * Ng + g]));
  }
  const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
  const double2 rho = a.rho[g];
  a.phi[g] = (k2 > 0.0) ? cscale(cadd(cscale(rho, a.sigma1), divU), 1.0 / k2) : make_double2(0.0, 0.0);
  a.psi[g] = cscale(divA, -a.kappa2);
}

__global__ __launch_bounds__(kBlock) void k_canonical(CanonArgs a) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.np) return;
  int64_t nodes[27];
  double wts[27];
  const int cnt = point_stencil(a.M, a.x, i, nodes, wts);
  double Ah[3] = {0.0, 0.0, 0.0};
  for (int k = 0; k < cnt; ++k)
    for (int c = 0; c < 3; ++c) Ah[c] += wts[k] * a.A[c][nodes[k]];
  const double q = ld_bulk(a.q, i, a.prec);
  for (int c = 0; c < 3; ++c) st_bulk(a.P[c], i, ld_bulk(a.P[c], i, a.prec) + a.sign * q * Ah[c], a.prec);
}

// Kinetic energy and transverse velocity moments of the accepted state.
__global__ __launch_bounds__(kBlock) void k_kinetic(KinArgs a) {
  double part[kDiagParts];
  for (int v = 0; v < kDiagParts; ++v) part[v] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.np;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t nodes[27];
    double wts[27];
    const int cnt = point_stencil(a.M, a.x, i, nodes, wts);
    double Ah[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < cnt; ++k)
      for (int c = 0; c < 3; ++c) Ah[c] += wts[k] * a.A[c][nodes[k]];
    const double q = ld_bulk(a.q, i, a.prec), m = fabs(q);
    double p[3];
    for (int c = 0; c < 3; ++c) p[c] = ld_bulk(a.P[c], i, a.prec) - q * Ah[c];
    const double imk = 1.0 / (m * a.kappa);
    const double p2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
    const double g = sqrt(1.0 + p2 * imk * imk);
    part[0] += p2 / (m * (g + 1.0));
    const double vy = p[1] / (m * g), vz = p[2] / (m * g);
    part[1] += m * (vy * vy + vz * vz);
    part[2] += m;
  }
  block_store<kDiagParts>(part, 0u, a.partials);
}

// Parseval sums over modes: |E_hat|^2, |B_hat|^2, |R_G hat|^2, |R_L hat|^2.
__global__ __launch_bounds__(kBlock) void k_spec_diag(SpecDiagArgs a) {
  double part[kDiagParts];
  for (int v = 0; v < kDiagParts; ++v) part[v] = 0.0;
  const Mesh& M = a.M;
  const int64_t Ng = M.Ng;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < Ng;
       g += (int64_t)gridDim.x * blockDim.x) {
    int64_t idx[3];
    mode_index(M, g, idx);
    const double k[3] = {ksym(M, 0, idx[0]), ksym(M, 1, idx[1]), ksym(M, 2, idx[2])};
    const double2 ph = a.phi[g];
    double2 E[3], A[3];
    double2 divE = make_double2(0.0, 0.0), divA = make_double2(0.0, 0.0);
    for (int c = 0; c < 3; ++c) {
      A[c] = a.A[c * Ng + g];
      E[c] = csub(make_double2(-cik(k[c], ph).x, -cik(k[c], ph).y), a.U[c * Ng + g]);
      divE = cadd(divE, cik(k[c], E[c]));
      divA = cadd(divA, cik(k[c], A[c]));
    }
    // B = i k x A
    const double2 B0 = csub(cik(k[1], A[2]), cik(k[2], A[1]));
    const double2 B1 = csub(cik(k[2], A[0]), cik(k[0], A[2]));
    const double2 B2 = csub(cik(k[0], A[1]), cik(k[1], A[0]));
    double e2 = 0.0;
    for (int c = 0; c < 3; ++c) e2 += E[c].x * E[c].x + E[c].y * E[c].y;
    const double b2 = B0.x * B0.x + B0.y * B0.y + B1.x * B1.x + B1.y * B1.y + B2.x * B2.x + B2.y * B2.y;
    const double2 RG = csub(divE, cscale(a.rho[g], a.sigma1));
    const double2 RL = cadd(cscale(a.psi[g], 1.0 / a.kappa2), divA);
    part[0] += e2;
    part[1] += b2;
    part[2] += RG.x * RG.x + RG.y * RG.y;
    part[3] += RL.x * RL.x + RL.y * RL.y;
  }
  block_store<kDiagParts>(part, 0u, a.partials);
}

__global__ __launch_bounds__(kBlock) void k_spec_field(Mesh M, int which_e, const double2* phi,
                                                       const double2* A, const double2* U,
                                                       double2* out) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t Ng = M.Ng;
  if (g >= Ng) return;
  int64_t idx[3];
  mode_index(M, g, idx);
  const double k[3] = {ksym(M, 0, idx[0]), ksym(M, 1, idx[1]), ksym(M, 2, idx[2])};
  if (which_e) {
    const double2 ph = phi[g];
    for (int c = 0; c < 3; ++c) {
      const double2 gk = cik(k[c], ph);
      out[c * Ng + g] = csub(make_double2(-gk.x, -gk.y), U[c * Ng + g]);
    }
  } else {
    const double2 A0 = A[g], A1 = A[Ng + g], A2 = A[2 * Ng + g];
    out[g] = csub(cik(k[1], A2), cik(k[2], A1));
    out[Ng + g] = csub(cik(k[2], A0), cik(k[0], A2));
    out[2 * Ng + g] = csub(cik(k[0], A1), cik(k[1], A0));
  }
}

struct PermArgs {
  const void* src[12];
  void* dst[12];
};

// inverse = 0: scatter sorted data (type prec) back to load order (FP64);
// inverse = 1: gather load-order data (FP64) into sorted order (type prec).
__global__ __launch_bounds__(kBlock) void k_unpermute(PermArgs p, int ncomp, const int32_t* id,
                                                      int64_t np, int inverse, int prec) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  const int64_t k = id[i];
  for (int c = 0; c < ncomp; ++c) {
    if (inverse)
      st_bulk(p.dst[c], i, static_cast<const double*>(p.src[c])[k], prec);
    else
      static_cast<double*>(p.dst[c])[k] = ld_bulk(p.src[c], i, prec);
  }
}

__global__ __launch_bounds__(kBlock) void k_load_state(const double* u0, const double* u1, const double* u2,
                                                       const double* qd, void* P0, void* P1, void* P2, void* q,
                                                       int prec, double kappa, int64_t np) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  st_bulk(q, i, qd[i], prec);
  const double mk = fabs(ld_bulk(q, i, prec)) * kappa;  // m = |q| as stored
  st_bulk(P0, i, mk * u0[i], prec);
  st_bulk(P1, i, mk * u1[i], prec);
  st_bulk(P2, i, mk * u2[i], prec);
}

__global__ __launch_bounds__(kBlock) void k_iota(int32_t* id, int64_t np) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) id[i] = (int32_t)i;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_load_state(double* const u[3], const double* qd, void* const P[3], void* q, int prec,
                             double kappa, int64_t np, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_load_state, dim3(nblk(np)), dim3(kBlock), 0, s, u[0], u[1], u[2], qd, P[0], P[1], P[2], q,
                     prec, kappa, np);
  return hipGetLastError();
}

hipError_t launch_iota(int32_t* id, int64_t np, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3(nblk(np)), dim3(kBlock), 0, s, id, np);
  return hipGetLastError();
}

hipError_t fft_nd(const Mesh& M, const FftPlanAxis* axes, int ncomp, const double* src_r,
                  const double2* src_c, double2* dst_c, double* dst_r, double2* scratch_c,
                  bool inverse, bool project, hipStream_t s, const int32_t* stop) {
  // passes: axis 0 .. d-1 (forward) or the same order (inverse; axes commute)
  double2* work = dst_c ? dst_c : scratch_c;
  for (int l = 0; l < M.d; ++l) {
    // lines per workgroup: enough workgroups to cover the chip (>= 512 when the mesh
    // allows), at most 4096 elements (64 KiB of LDS) per workgroup
    FftPlanAxis ax = axes[l];
    int64_t T = (ax.nlines * ncomp) / 512;
    T = std::max<int64_t>(1, std::min<int64_t>(T, std::max(1, 4096 / ax.N)));
    T = std::min<int64_t>(T, ax.nlines);
    while (T & (T - 1)) T &= T - 1;  // a power of two (nlines is one)
    // lines plus staged twiddles within 4096 complex values (64 KiB of LDS)
    while (T > 1 && T * ax.N + ax.N / 2 > 4096) T >>= 1;
    ax.lds_tw = (T * ax.N + ax.N / 2 <= 4096) ? 1 : 0;
    ax.T = (int)T;
    const int threads = (int)std::min<int64_t>(kBlock, std::max<int64_t>(64, (T * ax.N / 2 + 63) / 64 * 64));
    const bool first = (l == 0), last = (l == M.d - 1);
    const bool in_real = first && src_r != nullptr;
    const bool out_real = last && dst_r != nullptr;
    const double2* in_c = first ? src_c : work;
    const unsigned gx = (unsigned)((ax.nlines + ax.T - 1) / ax.T);
    const size_t lds = sizeof(double2) * ((size_t)ax.T * ax.N + (ax.lds_tw ? (size_t)std::max(ax.N / 2, 1) : 0));
    const int proj = (last && project && !inverse) ? 1 : 0;
    dim3 grid(gx, (unsigned)ncomp);
    if (in_real && out_real)
      hipLaunchKernelGGL((k_fft_axis<true, true>), grid, dim3(threads), lds, s, src_r, nullptr, nullptr,
                         dst_r, M.Ng, ax, inverse ? 1 : 0, proj, M, stop);
    else if (in_real)
      hipLaunchKernelGGL((k_fft_axis<true, false>), grid, dim3(threads), lds, s, src_r, nullptr, work,
                         nullptr, M.Ng, ax, inverse ? 1 : 0, proj, M, stop);
    else if (out_real)
      hipLaunchKernelGGL((k_fft_axis<false, true>), grid, dim3(threads), lds, s, nullptr, in_c, nullptr,
                         dst_r, M.Ng, ax, inverse ? 1 : 0, proj, M, stop);
    else
      hipLaunchKernelGGL((k_fft_axis<false, false>), grid, dim3(threads), lds, s, nullptr, in_c, work,
                         nullptr, M.Ng, ax, inverse ? 1 : 0, proj, M, stop);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_cn(const CNArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_cn, dim3(nblk(a.M.Ng)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_residual(const ResidualArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_reduce(const double* partials, int nblocks, int64_t bstride, int64_t vstride, int nvals,
                         uint32_t max_mask, double* out, hipStream_t s, const int32_t* stop) {
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)nvals), dim3(kBlock), 0, s, partials, nblocks, bstride, vstride, nvals,
                     max_mask, out, stop);
  return hipGetLastError();
}

hipError_t launch_zero(double* y, int64_t n, hipStream_t s, const int32_t* stop) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(nblk(n)), dim3(kBlock), 0, s, y, n, stop);
  return hipGetLastError();
}

hipError_t launch_outer_test(const double* res, int koff, int32_t* ctl, double* acc, int k, double n3,
                             double tol_abs, double tol_rel, hipStream_t s) {
  hipLaunchKernelGGL(k_outer_test, dim3(1), dim3(64), 0, s, res, koff, ctl, acc, k, n3, tol_abs, tol_rel);
  return hipGetLastError();
}

hipError_t launch_axpbz(double* y, double a, const double* x, double b, const double* z, int64_t n,
                        hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpbz, dim3(nblk(n)), dim3(kBlock), 0, s, y, a, x, b, z, n);
  return hipGetLastError();
}

hipError_t launch_dots(const DotArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_dots, dim3(blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_axpy2(double* y, const double* x, double2* yc, const double2* xc, double beta,
                        int64_t nreal, int64_t ncplx, hipStream_t s, const int32_t* stop) {
  const int64_t n = nreal > ncplx ? nreal : ncplx;
  hipLaunchKernelGGL(k_axpy2, dim3(nblk(n)), dim3(kBlock), 0, s, y, x, yc, xc, beta, nreal, ncplx, stop);
  return hipGetLastError();
}

hipError_t launch_init_deposit(const InitArgs& a, hipStream_t s) {
  if (a.np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_init_deposit, dim3(nblk(a.np)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_init_spectral(const InitSpecArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_init_spectral, dim3(nblk(a.M.Ng)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_canonical(const CanonArgs& a, hipStream_t s) {
  if (a.np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_canonical, dim3(nblk(a.np)), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_kinetic(const KinArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_kinetic, dim3(blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_spec_diag(const SpecDiagArgs& a, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_spec_diag, dim3(blocks), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_spec_field(const Mesh& M, int which_e, const double2* phi, const double2* A,
                             const double2* U, double2* out, hipStream_t s) {
  hipLaunchKernelGGL(k_spec_field, dim3(nblk(M.Ng)), dim3(kBlock), 0, s, M, which_e, phi, A, U, out);
  return hipGetLastError();
}

hipError_t launch_unpermute(const void* const* src, int src_prec, double* const* dst, int ncomp,
                            const int32_t* id, int64_t np, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  if (ncomp > 12) return hipErrorInvalidValue;
  PermArgs p;
  for (int c = 0; c < ncomp; ++c) {
    p.src[c] = src[c];
    p.dst[c] = dst[c];
  }
  hipLaunchKernelGGL(k_unpermute, dim3(nblk(np)), dim3(kBlock), 0, s, p, ncomp, id, np, 0, src_prec);
  return hipGetLastError();
}

hipError_t launch_permute_in(const double* const* src, void* const* dst, int dst_prec, int ncomp,
                             const int32_t* id, int64_t np, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  if (ncomp > 12) return hipErrorInvalidValue;
  PermArgs p;
  for (int c = 0; c < ncomp; ++c) {
    p.src[c] = src[c];
    p.dst[c] = dst[c];
  }
  hipLaunchKernelGGL(k_unpermute, dim3(nblk(np)), dim3(kBlock), 0, s, p, ncomp, id, np, 1, dst_prec);
  return hipGetLastError();
}

}  // namespace gmhc
