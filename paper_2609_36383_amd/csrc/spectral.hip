// spectral.hip -- periodic spectral field step on the mesh: batched radix-2 FFTs in
// LDS, the mode-by-mode Crank-Nicolson solve of the potential system with continuity
// and the Nyquist projector, the outer residual norms, initialization and the
// spectral diagnostics (section "Mesh-based field values and the Crank-Nicolson
// potential update", the Nyquist-projection paragraph and the constraint diagnostics).
#include <math.h>

#include <algorithm>

#include "gmhc_internal.h"
#include "wave.h"

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
  return M.kf[l] * (double)ms;
}

// per-axis mode index of node g (mesh sizes are powers of two)
__device__ __forceinline__ void mode_index(const Mesh& M, int64_t g, int64_t idx[3]) {
  idx[0] = g & (M.n[0] - 1);
  idx[1] = (g >> M.ln[0]) & (M.n[1] - 1);
  idx[2] = g >> (M.ln[0] + M.ln[1]);
}

__device__ __forceinline__ bool on_nyquist(const Mesh& M, const int64_t idx[3]) {
  bool r = false;
  for (int l = 0; l < M.d; ++l) r = r || (((M.n[l] & 1) == 0) && idx[l] == M.n[l] / 2);
  return r;
}

// Crank-Nicolson solve of mode g at the trial current: returns component `comp` of the
// trial-field spectrum [d+6]: i k phi^{n+1/2} (d), A^{n+1} (3), U^{n+1/2} (3).  With
// `side`, the new state the component belongs to is stored as well (rho, phi, psi with
// component 0; A and U of axis c with component d + c).
__device__ __forceinline__ double2 cn_point(const CNArgs& a, int64_t g, int comp, bool side) {
  const Mesh& M = a.M;
  const int64_t Ng = M.Ng;
  const int d = M.d;
  int64_t idx[3];
  mode_index(M, g, idx);
  const double k[3] = {ksym(M, 0, idx[0]), ksym(M, 1, idx[1]), ksym(M, 2, idx[2])};
  const double h = a.dt;
  const double av = a.kappa2 * (k[0] * k[0] + k[1] * k[1] + k[2] * k[2]);
  const double q4 = 0.25 * h * h * av;
  const double inv_den = 1.0 / (1.0 + q4);
  const double c1 = 1.0 - q4;
  if (comp < d) {
    const double2 j0 = a.jh[g], j1 = a.jh[Ng + g], j2 = a.jh[2 * Ng + g];
    // continuity: rho^{n+1} = rho^n - dt div_h J^{n+1/2}
    const double2 divj = cadd(cadd(cik(k[0], j0), cik(k[1], j1)), cik(k[2], j2));
    const double2 rho0 = a.rho[g];
    const double2 rho1 = csub(rho0, cscale(divj, h));
    const double2 rhoh = cscale(cadd(rho0, rho1), 0.5);
    const double src1 = 0.5 * h * h * a.kappa2 * a.sigma1;
    // (phi, psi): phi^{n+1} from the CN pair with psi eliminated
    const double2 ph0 = a.phi[g], ps0 = a.psi[g];
    const double2 ph1 = cscale(cadd(cadd(cscale(ph0, c1), cscale(ps0, h)), cscale(rhoh, src1)), inv_den);
    if (side && comp == 0) {
      a.rho1[g] = rho1;
      a.phi1[g] = ph1;
      a.psi1[g] = csub(cscale(csub(ph1, ph0), 2.0 / h), ps0);
    }
    return cik(k[comp], cscale(cadd(ph0, ph1), 0.5));
  }
  const int c = (comp - d) % 3;
  const double src2 = 0.5 * h * h * a.kappa2 * a.sigma2;
  const double2 A0 = a.A[c * Ng + g], U0 = a.U[c * Ng + g], jc = a.jh[c * Ng + g];
  const double2 A1 = cscale(cadd(cadd(cscale(A0, c1), cscale(U0, h)), cscale(jc, src2)), inv_den);
  if (comp < d + 3) {
    if (side) {
      a.A1[c * Ng + g] = A1;
      a.U1[c * Ng + g] = csub(cscale(csub(A1, A0), 2.0 / h), U0);
    }
    return A1;
  }
  const double2 U1 = csub(cscale(csub(A1, A0), 2.0 / h), U0);
  return cscale(cadd(U0, U1), 0.5);
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

// Outer residual r = H(j) - j at node g, folded into part: sums of |r|^2, |H|^2, |j|^2,
// the max-node test ratio, and the mesh work sum_g H . E^{n+1/2}
// (E^{n+1/2} = -grad phi^{n+1/2} - U^{n+1/2}).
__device__ __forceinline__ void residual_node(const ResidualArgs& a, int64_t g, const double H[3],
                                              double (&part)[kResParts]) {
  const int64_t Ng = a.M.Ng;
  double r2 = 0.0, h2 = 0.0, j2 = 0.0, w = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double j = a.j[c * Ng + g];
    const double r = H[c] - j;
    r2 += r * r;
    h2 += H[c] * H[c];
    j2 += j * j;
    const double gp = (c < a.M.d) ? a.gphi[c * Ng + g] : 0.0;
    w += H[c] * (-gp - a.Uh[c * Ng + g]);
  }
  part[0] += r2;
  part[1] += h2;
  part[2] += j2;
  part[3] = fmax(part[3], sqrt(r2) / (a.tol_abs + 0.5 * a.tol_rel * (sqrt(h2) + sqrt(j2))));
  part[4] += w;
}

__global__ __launch_bounds__(kBlock) void k_residual(ResidualArgs a) {
  if (a.stop && *a.stop) return;
  double part[kResParts];
#pragma unroll
  for (int v = 0; v < kResParts; ++v) part[v] = 0.0;
  const int64_t Ng = a.M.Ng;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < Ng;
       g += (int64_t)gridDim.x * blockDim.x) {
    const double H[3] = {a.H[g], a.H[Ng + g], a.H[2 * Ng + g]};
    residual_node(a, g, H, part);
  }
  block_store<kResParts>(part, 1u << 3, a.partials);
}

// ---- batched line FFTs along one axis
//
// A workgroup loads T lines of length N of cpb components into LDS and runs radix-2
// butterfly stages on them (all lines at once, one barrier per stage).  The first
// transform is decimation in time (bit-reversed load, natural-order result).  A pass
// with both transforms (the last forward axis of H = P J) then zeroes the even-grid
// Nyquist modes, stores the projected spectrum and runs the inverse by decimation in
// frequency (natural order in, bit-reversed out), so the spectrum is never reordered.
// The load can compute the Crank-Nicolson solve of the trial current instead of reading
// (the first inverse pass of the trial fields); the store can zero a deposit buffer and,
// with the three current components in one workgroup, fold the outer residual.
struct FftTask {
  FftPlanAxis ax;
  int cpb;              // components per workgroup
  int fwd, inv;         // transforms of the pass (forward first when both)
  int project;          // zero the even-grid Nyquist modes after the forward transform
  const double* src_r;  // real input, or
  const unsigned long long* src_fx;  // real input as fixed-point pairs (fixsum.h), or
  const double2* src_c; // complex input (unless the load computes the CN solve)
  double2* dst_c;       // complex output, or
  double* dst_r;        // real part of the output
  double2* spec;        // fwd && inv: the projected spectrum is stored here
  unsigned long long* zero;  // fixed-point pair c Ng + g cleared at the output positions
                             // of components c < 3
  int res;              // fold the outer residual of H = output (cpb == 3)
  ResidualArgs ra;
};

__device__ __forceinline__ int brev_n(int k, int logN) {
  return logN > 0 ? (int)(__brev((unsigned)k) >> (32 - logN)) : 0;
}

// IN: 0 complex input, 1 real input, 2 CN solve at load
constexpr int kFftThreads = 1024;  // threads per FFT workgroup at most

// One pass as workgroup (bx, by) of its grid: lines bx T .. bx T + T - 1, components
// by cpb .. by cpb + cpb - 1.
template <int IN, bool OUT_REAL>
__device__ __forceinline__ void fft_body(const FftTask& t, const CNArgs& cn, const Mesh& M, int bx, int by,
                                         double2* lds) {
  const FftPlanAxis& ax = t.ax;
  const int N = ax.N, T = ax.T, logN = ax.logN;  // N and T are powers of two
  const int logT = 31 - __clz(T);
  const int64_t Ng = M.Ng;
  const int64_t comp0 = (int64_t)by * t.cpb;
  const int64_t line0 = (int64_t)bx * T;
  const int per = T * N, total = per * t.cpb;
  // twiddles exp(-2 pi i m / N), m < N/2, staged once after the lines when they fit
  double2* twl = lds + total;
  if (ax.lds_tw)
    for (int m = threadIdx.x; m < N / 2; m += blockDim.x) twl[m] = ax.tw[m];
  const double2* tws = ax.lds_tw ? twl : ax.tw;
  // element e -> (component c, line lt, index k), coalesced in the axis' memory order
  const int logPer = logT + logN;
  auto split = [&](int e, int& c, int& lt, int& k) {
    c = e >> logPer;
    const int r = e & (per - 1);
    if (ax.stride == 1) {
      lt = r >> logN;
      k = r & (N - 1);
    } else {
      lt = r & (T - 1);
      k = r >> logT;
    }
  };
  auto node = [&](int64_t line, int k) {
    const int64_t iin = line & (ax.stride - 1), iout = line >> ax.lstride;
    return iin + (((int64_t)k + (iout << logN)) << ax.lstride);
  };
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int c, lt, k;
    split(e, c, lt, k);
    const int64_t line = line0 + lt;
    double2 v = make_double2(0.0, 0.0);
    if (line < ax.nlines) {
      const int64_t g = node(line, k);
      const int64_t comp = comp0 + c;
      if (IN == 2)
        v = cn_point(cn, g, (int)comp, true);
      else if (IN == 1)
        v = make_double2(t.src_fx ? fix_value(t.src_fx, comp * Ng + g, M.fx.hi, M.fx.lo) : t.src_r[comp * Ng + g],
                         0.0);
      else
        v = t.src_c[comp * Ng + g];
    }
    lds[(c * T + lt) * N + brev_n(k, logN)] = v;
  }
  __syncthreads();
  const int nbf = t.cpb * T * (N / 2);  // butterflies per stage
  // decimation in time: forward, or the inverse when the pass has no forward transform
  const bool conj1 = !t.fwd;
  for (int st = 1; st <= logN; ++st) {
    const int half = 1 << (st - 1);
    const int twstep = N >> st;
    for (int b = threadIdx.x; b < nbf; b += blockDim.x) {
      const int lt = b >> (logN - 1), j = b & (N / 2 - 1);
      const int grp = j >> (st - 1), pos = j & (half - 1);
      const int i1 = lt * N + grp * (2 * half) + pos, i2 = i1 + half;
      double2 w = tws[pos * twstep];
      if (conj1) w.y = -w.y;
      const double2 u = lds[i1];
      const double2 tt = cmul(lds[i2], w);
      lds[i1] = cadd(u, tt);
      lds[i2] = csub(u, tt);
    }
    __syncthreads();
  }
  const bool both = t.fwd && t.inv;
  if (both) {
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
      int c, lt, k;
      split(e, c, lt, k);
      const int64_t line = line0 + lt;
      if (line >= ax.nlines) continue;
      const int64_t g = node(line, k);
      const int li = (c * T + lt) * N + k;
      double2 v = lds[li];
      if (t.project) {
        int64_t idx[3];
        mode_index(M, g, idx);
        if (on_nyquist(M, idx)) {
          v = make_double2(0.0, 0.0);
          lds[li] = v;
        }
      }
      t.spec[(comp0 + c) * Ng + g] = v;
    }
    __syncthreads();
    // inverse by decimation in frequency
    for (int st = logN; st >= 1; --st) {
      const int half = 1 << (st - 1);
      const int twstep = N >> st;
      for (int b = threadIdx.x; b < nbf; b += blockDim.x) {
        const int lt = b >> (logN - 1), j = b & (N / 2 - 1);
        const int grp = j >> (st - 1), pos = j & (half - 1);
        const int i1 = lt * N + grp * (2 * half) + pos, i2 = i1 + half;
        double2 w = tws[pos * twstep];
        w.y = -w.y;
        const double2 u = lds[i1], v = lds[i2];
        lds[i1] = cadd(u, v);
        lds[i2] = cmul(csub(u, v), w);
      }
      __syncthreads();
    }
  }
  const double sc = t.inv ? 1.0 / (double)N : 1.0;
  for (int e = threadIdx.x; e < total; e += blockDim.x) {
    int c, lt, k;
    split(e, c, lt, k);
    const int64_t line = line0 + lt;
    if (line >= ax.nlines) continue;
    const int64_t g = node(line, k);
    const int64_t comp = comp0 + c;
    double2 v = cscale(lds[(c * T + lt) * N + (both ? brev_n(k, logN) : k)], sc);
    if (t.project && !both) {
      int64_t idx[3];
      mode_index(M, g, idx);
      if (on_nyquist(M, idx)) v = make_double2(0.0, 0.0);
    }
    if (OUT_REAL)
      t.dst_r[comp * Ng + g] = v.x;
    else
      t.dst_c[comp * Ng + g] = v;
    if (t.zero && comp < 3) {
      t.zero[2 * (comp * Ng + g)] = 0ull;
      t.zero[2 * (comp * Ng + g) + 1] = 0ull;
    }
  }
  if (t.res) {
    // the three components of H at each node of the workgroup's lines
    double part[kResParts];
#pragma unroll
    for (int v = 0; v < kResParts; ++v) part[v] = 0.0;
    for (int e = threadIdx.x; e < per; e += blockDim.x) {
      int c, lt, k;
      split(e, c, lt, k);
      const int64_t line = line0 + lt;
      if (line >= ax.nlines) continue;
      const int kk = both ? brev_n(k, logN) : k;
      const double H[3] = {lds[lt * N + kk].x * sc, lds[(T + lt) * N + kk].x * sc, lds[(2 * T + lt) * N + kk].x * sc};
      residual_node(t.ra, node(line, k), H, part);
    }
    // each wave through DPP, then the waves in order; the lines' LDS holds the wave sums
#pragma unroll
    for (int v = 0; v < kResParts; ++v)
      part[v] = (v == 3) ? wave_reduce_f64<true>(part[v]) : wave_reduce_f64<false>(part[v]);
    __syncthreads();
    double* shd = reinterpret_cast<double*>(lds);
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    if (lane == 0)
#pragma unroll
      for (int v = 0; v < kResParts; ++v) shd[wave * kResParts + v] = part[v];
    __syncthreads();
    if ((int)threadIdx.x < kResParts) {
      const int v = threadIdx.x;
      double acc = shd[v];
      for (int w = 1; w < (int)(blockDim.x / 64); ++w)
        acc = (v == 3) ? fmax(acc, shd[w * kResParts + v]) : acc + shd[w * kResParts + v];
      t.ra.partials[(int64_t)bx * kResParts + v] = acc;
    }
  }
}

template <int IN, bool OUT_REAL>
__global__ __launch_bounds__(kFftThreads) void k_fft_pass(FftTask t, CNArgs cn, Mesh M, const int32_t* stop) {
  if (stop && *stop) return;
  extern __shared__ double2 lds[];
  fft_body<IN, OUT_REAL>(t, cn, M, blockIdx.x, blockIdx.y, lds);
}

// Two independent passes in one launch: workgroup b < n1 is workgroup (b mod gx1,
// b div gx1) of pass 1, workgroup n1 + b' is (b' mod gx2, b' div gx2) of pass 2.
template <int IN1, bool OUT1, int IN2, bool OUT2>
__global__ __launch_bounds__(kFftThreads) void k_fft_pass2(FftTask t1, int gx1, int n1, FftTask t2, int gx2,
                                                           CNArgs cn, Mesh M, const int32_t* stop) {
  if (stop && *stop) return;
  extern __shared__ double2 lds[];
  const int b = blockIdx.x;
  if (b < n1)
    fft_body<IN1, OUT1>(t1, cn, M, b % gx1, b / gx1, lds);
  else
    fft_body<IN2, OUT2>(t2, cn, M, (b - n1) % gx2, (b - n1) / gx2, lds);
}

// Reduction of one value over nblocks partials p[b * bstride] (max or sum) by a
// workgroup of NT threads; the result is valid in thread 0.  Every maximum reduced here
// is of nonnegative values (iteration counts, residual ratios), so 0 is its identity and
// an empty set (no particles) reduces to 0.  Thread t folds blocks t,
// t + NT, ... into sixteen independent accumulators (so sixteen loads are in flight),
// combines them in a fixed order, then a fixed pairwise tree combines the threads: the
// result depends only on nblocks and NT.
template <int NT>
__device__ double reduce_value(const double* p, int nblocks, int64_t bstride, bool mx) {
  constexpr int NA = 16;
  const double id = 0.0;
  double acc16[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) acc16[k] = id;
  int b = threadIdx.x;
  for (; b + (NA - 1) * NT < nblocks; b += NA * NT) {
    double x[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) x[k] = p[(int64_t)(b + k * NT) * bstride];
#pragma unroll
    for (int k = 0; k < NA; ++k) acc16[k] = mx ? fmax(acc16[k], x[k]) : acc16[k] + x[k];
  }
#pragma unroll
  for (int k = 0; k < NA - 1; ++k) {
    const int bb = b + k * NT;
    if (bb < nblocks) {
      const double x = p[(int64_t)bb * bstride];
      acc16[k] = mx ? fmax(acc16[k], x) : acc16[k] + x;
    }
  }
  double acc = acc16[0];
#pragma unroll
  for (int k = 1; k < NA; ++k) acc = mx ? fmax(acc, acc16[k]) : acc + acc16[k];
  // each wave through DPP, then the wave sums in order
  acc = mx ? wave_reduce_f64<true>(acc) : wave_reduce_f64<false>(acc);
  __shared__ double sh[NT / 64];
  if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = acc;
  __syncthreads();
  double r = sh[0];
  for (int w = 1; w < NT / 64; ++w) r = mx ? fmax(r, sh[w]) : r + sh[w];
  return r;
}

__global__ __launch_bounds__(kBlock) void k_reduce(const double* partials, int nblocks, int64_t bstride,
                                                   int64_t vstride, int nvals, uint32_t max_mask, double* out,
                                                   const int32_t* stop) {
  if (stop && *stop) return;
  const int v = blockIdx.x;  // one workgroup per value
  if (v >= nvals) return;
  const double x = reduce_value<kBlock>(partials + (int64_t)v * vstride, nblocks, bstride, (max_mask >> v) & 1u);
  if (threadIdx.x == 0) out[v] = x;
}

// First level of a long reduction: workgroup (c, v) reduces blocks [c chunk, c chunk +
// chunk) of value v in a fixed order into out[v nchunks + c], so the second level reads
// nchunks values per value instead of nblocks.
__global__ __launch_bounds__(kBlock) void k_reduce_chunks(const double* p, int nblocks, int64_t vstride,
                                                          uint32_t max_mask, int chunk, double* out,
                                                          const int32_t* stop) {
  if (stop && *stop) return;
  const int c = blockIdx.x, v = blockIdx.y;
  const int b0 = c * chunk;
  const int nb = min(chunk, nblocks - b0);
  const double x = reduce_value<kBlock>(p + (int64_t)v * vstride + b0, nb, 1, (max_mask >> v) & 1u);
  if (threadIdx.x == 0) out[(int64_t)v * gridDim.x + c] = x;
}

__global__ __launch_bounds__(kBlock) void k_zero(double* y, int64_t n, const int32_t* stop) {
  if (stop && *stop) return;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = 0.0;
}

// Outer test of Picard iteration t.k (one thread; see launch_reduce_outer).
__device__ void outer_test(const OuterTest& t) {
  if (t.ctl[0]) return;
  const double* h = t.res;
  const double* r = t.res + t.koff;
  double* acc = t.acc;
  acc[0] += h[OP_ITERS];
  acc[1] += h[OP_SEGS];
  acc[2] = h[OP_ITMAX];
  acc[3] += 1.0;
  acc[10] = h[OP_ITERS];
  acc[12] = h[OP_REFINED];
  if (h[OP_FAIL] > 0.0) {
    acc[4] = h[OP_FAIL];
    acc[11] = h[OP_XLIM];
    t.ctl[1] = 1;
    t.ctl[2] = t.k;
    t.ctl[0] = 1;
    return;
  }
  const double rr = sqrt(r[0] / t.n3) / (t.tol_abs + 0.5 * t.tol_rel * (sqrt(r[1] / t.n3) + sqrt(r[2] / t.n3)));
  const double mr = r[3];
  acc[5] = rr;
  acc[6] = mr;
  if (rr <= 1.0 && mr <= 1.0) {
    acc[7] = h[OP_RA2];
    acc[8] = h[OP_WORK];
    acc[9] = r[4];
    t.ctl[2] = t.k;
    t.ctl[0] = 1;
  }
}

// Both partial sets in one launch, one workgroup per value; the last workgroup to finish
// (ticket ctl[3], left at zero) runs the outer test.
constexpr int kRedThreads = 1024;  // threads per workgroup of the merged reduction

// Workgroup bx of the nred = a.nvals + b.nvals reduction workgroups (kRedThreads each).
__device__ __forceinline__ void reduce_outer_body(const ReduceSet& a, const ReduceSet& b, const OuterTest& t,
                                                  int bx, int nred) {
  const bool inb = bx >= a.nvals;
  const ReduceSet& r = inb ? b : a;
  const int v = inb ? bx - a.nvals : bx;
  const double x = reduce_value<kRedThreads>(r.p + (int64_t)v * r.vstride, r.nblocks, r.bstride, (r.max_mask >> v) & 1u);
  __shared__ int s_last;
  if (threadIdx.x == 0) {
    r.out[v] = x;
    s_last = 0;
    if (t.ctl) {
      __threadfence();  // the value is visible before the ticket counts it
      s_last = atomicAdd(&t.ctl[3], 1) == nred - 1;
    }
  }
  __syncthreads();
  if (s_last && threadIdx.x == 0) {
    __threadfence();  // every other workgroup's value is visible
    t.ctl[3] = 0;
    outer_test(t);
  }
}

__global__ __launch_bounds__(kRedThreads) void k_reduce_outer(ReduceSet a, ReduceSet b, OuterTest t,
                                                              const int32_t* stop) {
  if (stop && *stop) return;
  reduce_outer_body(a, b, t, blockIdx.x, gridDim.x);
}

// The reduction with its outer test and an independent FFT pass in one launch: the first
// a.nvals + b.nvals workgroups reduce, workgroup nred + e is workgroup (e mod gx,
// e div gx) of the pass.
template <int IN, bool OUT_REAL>
__global__ __launch_bounds__(kRedThreads) void k_reduce_fft(ReduceSet a, ReduceSet b, OuterTest t, FftTask te,
                                                            int gx, CNArgs cn, Mesh M, const int32_t* stop) {
  if (stop && *stop) return;
  const int nred = a.nvals + b.nvals;
  if ((int)blockIdx.x < nred) {
    reduce_outer_body(a, b, t, blockIdx.x, nred);
    return;
  }
  extern __shared__ double2 lds[];
  const int e = (int)blockIdx.x - nred;
  fft_body<IN, OUT_REAL>(te, cn, M, e % gx, e / gx, lds);
}

// End of a Picard batch on the device (one workgroup): every value of the control block
// and the report accumulators is read, published to host memory and, once the outer
// test stopped the step (ctl[0] set, success or failure), cleared for the next step;
// the sequence number is stored last (the host spins on it).
__global__ __launch_bounds__(64) void k_ctl_publish(int32_t* ctl, double* acc, int nacc, CtlPublish pub,
                                                    uint32_t seq) {
  const int l = threadIdx.x;
  const bool stop = ctl[0] != 0;
  int32_t cv = 0;
  double av = 0.0;
  if (l < 4)
    cv = ctl[l];
  else if (l < 4 + nacc)
    av = acc[l - 4];
  __syncthreads();  // every value read before any is cleared
  if (l < 4) {
    pub.ctl[l] = cv;
    if (stop) ctl[l] = 0;
  } else if (l < 4 + nacc) {
    pub.acc[l - 4] = av;
    if (stop) acc[l - 4] = 0.0;
  }
  __syncthreads();
  if (l == 0) __hip_atomic_store(pub.seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
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

// Point weights of nodes j-1, j, j+1 (j the nearest node) under the quadratic S_2 or,
// for shape 1, the linear S_1.
__device__ __forceinline__ void pw(double xi, int n, int shape, int gi[3], double w[3]) {
  if (!(xi > -1.0e9 && xi < 1.0e9)) xi = 0.0;  // non-finite positions map to a valid node
  const int j = (int)floor(xi + 0.5);
  const double f = xi - (double)j;
  if (shape == 1) {
    w[0] = f < 0.0 ? -f : 0.0;
    w[1] = 1.0 - fabs(f);
    w[2] = f > 0.0 ? f : 0.0;
  } else {
    const double a = 0.5 - f, b = 0.5 + f;
    w[0] = 0.5 * a * a;
    w[1] = 0.75 - f * f;
    w[2] = 0.5 * b * b;
  }
  for (int c = 0; c < 3; ++c) gi[c] = wrapi(j + c - 1, n);
}

// Point-shape stencil of a particle: up to 27 (node, weight) pairs.
__device__ __forceinline__ int point_stencil(const Mesh& M, const double* const* x, int64_t i,
                                             int64_t* nodes, double* wts) {
  int gi[3][3];
  double w[3][3];
  for (int l = 0; l < 3; ++l) {
    if (l < M.d) {
      pw((x[l][i] - M.lo[l]) * M.inv_h[l], M.n[l], M.shape, gi[l], w[l]);
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
  const int64_t Ng = a.M.Ng;
  for (int k = 0; k < cnt; ++k) {
    fix_add(a.rho, nodes[k], qd * wts[k], a.M.fx.up);
    for (int c = 0; c < 3; ++c) fix_add(a.J, c * Ng + nodes[k], qd * v[c] * wts[k], a.M.fx.up);
  }
}

__global__ __launch_bounds__(kBlock) void k_fix_to_double(const unsigned long long* acc, double* out, int64_t n,
                                                          FixScale fx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = fix_value(acc, i, fx.hi, fx.lo);
}

// Sum of |q| (bound of the charge and current sums per node): one value per block in
// the first slot of its kDiagParts partials.
__global__ __launch_bounds__(kBlock) void k_abs_charge(const void* q, int prec, int64_t np, double* partials) {
  double part[kDiagParts];
  for (int v = 0; v < kDiagParts; ++v) part[v] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x)
    part[0] += fabs(ld_bulk(q, i, prec));
  block_store<kDiagParts>(part, 0u, partials);
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

// dst[id[i]] = src[i]: per-particle integers back to load order.
__global__ __launch_bounds__(kBlock) void k_unpermute_i32(const int32_t* src, int32_t* dst, const int32_t* id,
                                                          int64_t np) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < np) dst[id[i]] = src[i];
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

namespace {

constexpr int kFftLds = 4096;  // complex values of LDS per FFT workgroup (64 KiB)

// Whether cpb components of one line of this axis fit a workgroup's LDS.
bool fits(const FftPlanAxis& ax, int cpb) { return (int64_t)cpb * ax.N <= kFftLds; }

// Launch one pass over ncomp components (ncomp a multiple of t.cpb); in: 0 complex,
// 1 real, 2 CN solve.  The number of workgroups along x goes to *nblk when asked.
// Launch shape of one pass over ncomp components.
struct PassShape {
  FftTask t;      // with the lines per workgroup and the twiddle staging filled in
  unsigned gx;    // workgroups along the lines
  unsigned ny;    // workgroups along the components
  int threads;
  size_t lds;     // dynamic LDS bytes
};

// With want_threads, the lines per workgroup are instead as many as give that many
// butterflies per stage (for a launch whose workgroup size is fixed by another part).
hipError_t shape_pass(FftTask t, int ncomp, PassShape& p, int want_threads = 0) {
  FftPlanAxis& ax = t.ax;
  const int cpb = t.cpb;
  // lines per workgroup: enough workgroups to cover the chip (>= 512 when the mesh
  // allows), the lines and the staged twiddles within kFftLds complex values
  int64_t T = want_threads > 0 ? (2 * (int64_t)want_threads) / ((int64_t)cpb * ax.N)
                               : (ax.nlines * (ncomp / cpb)) / 512;
  T = std::max<int64_t>(1, std::min<int64_t>(T, std::max<int64_t>(1, kFftLds / ((int64_t)ax.N * cpb))));
  T = std::min<int64_t>(T, ax.nlines);
  while (T & (T - 1)) T &= T - 1;  // a power of two (nlines is one)
  while (T > 1 && T * ax.N * cpb + ax.N / 2 > kFftLds) T >>= 1;
  if (T * ax.N * cpb > kFftLds) return hipErrorInvalidValue;
  ax.lds_tw = (T * ax.N * cpb + ax.N / 2 <= kFftLds) ? 1 : 0;
  ax.T = (int)T;
  // one butterfly per thread and stage, up to kFftThreads
  const int threads = (int)std::min<int64_t>(kFftThreads, std::max<int64_t>(64, (cpb * T * ax.N / 2 + 63) / 64 * 64));
  const unsigned gx = (unsigned)((ax.nlines + ax.T - 1) / ax.T);
  // (at least the residual's wave sums: kFftThreads / 64 waves x kResParts doubles)
  const size_t lds = std::max<size_t>(sizeof(double) * (kFftThreads / 64) * kResParts,
                                      sizeof(double2) * ((size_t)cpb * ax.T * ax.N +
                                                         (ax.lds_tw ? (size_t)std::max(ax.N / 2, 1) : 0)));
  p = PassShape{t, gx, (unsigned)(ncomp / cpb), threads, lds};
  return hipSuccess;
}

hipError_t fft_pass(const Mesh& M, FftTask task, int ncomp, int in, bool out_real, const CNArgs* cn, hipStream_t s,
                    const int32_t* stop, int* nblk = nullptr) {
  PassShape p;
  hipError_t err = shape_pass(task, ncomp, p);
  if (err != hipSuccess) return err;
  const FftTask& t = p.t;
  const dim3 grid(p.gx, p.ny);
  const int threads = p.threads;
  const size_t lds = p.lds;
  const CNArgs c0 = cn ? *cn : CNArgs{};
  if (nblk) *nblk = (int)p.gx;
  if (in == 2) {
    if (out_real)
      hipLaunchKernelGGL((k_fft_pass<2, true>), grid, dim3(threads), lds, s, t, c0, M, stop);
    else
      hipLaunchKernelGGL((k_fft_pass<2, false>), grid, dim3(threads), lds, s, t, c0, M, stop);
  } else if (in == 1) {
    if (out_real)
      hipLaunchKernelGGL((k_fft_pass<1, true>), grid, dim3(threads), lds, s, t, c0, M, stop);
    else
      hipLaunchKernelGGL((k_fft_pass<1, false>), grid, dim3(threads), lds, s, t, c0, M, stop);
  } else {
    if (out_real)
      hipLaunchKernelGGL((k_fft_pass<0, true>), grid, dim3(threads), lds, s, t, c0, M, stop);
    else
      hipLaunchKernelGGL((k_fft_pass<0, false>), grid, dim3(threads), lds, s, t, c0, M, stop);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t fft_nd(const Mesh& M, const FftPlanAxis* axes, int ncomp, const double* src_r,
                  const double2* src_c, double2* dst_c, double* dst_r, double2* scratch_c,
                  bool inverse, bool project, hipStream_t s, const int32_t* stop) {
  // passes: axis 0 .. d-1 (forward) or the same order (inverse; axes commute)
  double2* work = dst_c ? dst_c : scratch_c;
  for (int l = 0; l < M.d; ++l) {
    const bool first = (l == 0), last = (l == M.d - 1);
    FftTask t{};
    t.ax = axes[l];
    t.cpb = 1;
    t.fwd = inverse ? 0 : 1;
    t.inv = inverse ? 1 : 0;
    t.project = (last && project && !inverse) ? 1 : 0;
    t.src_r = src_r;
    t.src_c = first ? src_c : work;
    t.dst_c = work;
    t.dst_r = dst_r;
    const bool in_real = first && src_r != nullptr;
    const bool out_real = last && dst_r != nullptr;
    hipError_t e = fft_pass(M, t, ncomp, in_real ? 1 : 0, out_real, nullptr, s, stop);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

namespace {

// field_trial's pass over axis l: the CN solve at load (l = 0), the inverse along l, and on
// the last axis the real trial fields with `zero` cleared.
FftTask trial_task(const Mesh& M, const FftPlanAxis* axes, int l, double* trial, double2* work,
                   unsigned long long* zero) {
  FftTask t{};
  t.ax = axes[l];
  t.cpb = 1;
  t.inv = 1;
  t.src_c = work;
  t.dst_c = work;
  t.dst_r = trial;
  t.zero = (l == M.d - 1) ? zero : nullptr;
  return t;
}

// field_h's forward pass over axis l < d - 1 (real J in on axis 0).
FftTask h_forward_task(const FftPlanAxis* axes, int l, const unsigned long long* J, double2* work) {
  FftTask t{};
  t.ax = axes[l];
  t.cpb = 1;
  t.fwd = 1;
  t.src_fx = J;
  t.src_c = work;
  t.dst_c = work;
  return t;
}

// field_h's pass over axis l of its inverse sweep: on axis d - 1 the forward transform
// first, the projected spectrum out, then the inverse; on axis 0 H out and, with
// fuse_res, the residual folded.
FftTask h_inverse_task(const Mesh& M, const FftPlanAxis* axes, int l, const unsigned long long* J, double2* spec,
                       double2* work, double* H, bool project, bool fuse_res, const ResidualArgs& ra) {
  const bool top = (l == M.d - 1), last = (l == 0);
  FftTask t{};
  t.ax = axes[l];
  t.fwd = top ? 1 : 0;
  t.inv = 1;
  t.project = (top && project) ? 1 : 0;
  t.cpb = (last && fuse_res) ? 3 : 1;
  t.res = (last && fuse_res) ? 1 : 0;
  t.src_fx = J;
  t.src_c = work;
  t.dst_c = work;
  t.dst_r = H;
  t.spec = spec;
  t.ra = ra;
  t.ra.H = H;
  return t;
}

}  // namespace

hipError_t field_trial(const Mesh& M, const FftPlanAxis* axes, const CNArgs& cn, double* trial, double2* work,
                       unsigned long long* zero, hipStream_t s) {
  const int d = M.d;
  for (int l = 0; l < d; ++l) {
    hipError_t e = fft_pass(M, trial_task(M, axes, l, trial, work, zero), d + 6, l == 0 ? 2 : 0, l == d - 1, &cn, s,
                            cn.stop);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t field_h(const Mesh& M, const FftPlanAxis* axes, const unsigned long long* J, double2* spec,
                   double2* work, double* H, bool project, const ResidualArgs& ra, int* res_blocks, hipStream_t s) {
  const int d = M.d;
  const int32_t* stop = ra.stop;
  const bool fuse_res = fits(axes[0], 3);
  // forward passes of axes 0 .. d-2
  for (int l = 0; l < d - 1; ++l) {
    hipError_t e = fft_pass(M, h_forward_task(axes, l, J, work), 3, l == 0 ? 1 : 0, false, nullptr, s, stop);
    if (e != hipSuccess) return e;
  }
  // axis d-1: forward, projected spectrum out, then its inverse; then the inverse passes
  // of axes d-2 .. 0.  The last pass (axis 0) writes H and folds the residual.
  for (int l = d - 1; l >= 0; --l) {
    const FftTask t = h_inverse_task(M, axes, l, J, spec, work, H, project, fuse_res, ra);
    int nb = 0;
    hipError_t e = fft_pass(M, t, 3, (l == d - 1 && d == 1) ? 1 : 0, l == 0, nullptr, s, stop, &nb);
    if (e != hipSuccess) return e;
    if (t.res) *res_blocks = nb;
  }
  if (!fuse_res) {
    ResidualArgs r = ra;
    r.H = H;
    const int rb = (int)std::min<int64_t>((M.Ng + kBlock - 1) / kBlock, 1024);
    hipLaunchKernelGGL(k_residual, dim3(rb), dim3(kBlock), 0, s, r);
    *res_blocks = rb;
    return hipGetLastError();
  }
  return hipSuccess;
}

bool field_h_next_fits(const Mesh& M, const FftPlanAxis* axes) { return fits(axes[0], 3); }

hipError_t field_h_next(const Mesh& M, const FftPlanAxis* axes, const unsigned long long* J, double2* spec,
                        double2* work, double* H, bool project, const ResidualArgs& ra, const ReduceSet& ro,
                        const ReduceSet& rr, const OuterTest& ot, const CNArgs& cn, double* trial, double2* twork,
                        unsigned long long* zero, hipStream_t s) {
  const int d = M.d;
  const int32_t* stop = ra.stop;
  if (!fits(axes[0], 3)) return hipErrorInvalidValue;
  // the passes of field_h down to axis 1, unchanged
  for (int l = 0; l < d - 1; ++l) {
    hipError_t e = fft_pass(M, h_forward_task(axes, l, J, work), 3, l == 0 ? 1 : 0, false, nullptr, s, stop);
    if (e != hipSuccess) return e;
  }
  for (int l = d - 1; l >= 1; --l) {
    hipError_t e = fft_pass(M, h_inverse_task(M, axes, l, J, spec, work, H, project, true, ra), 3, 0, false,
                            nullptr, s, stop);
    if (e != hipSuccess) return e;
  }
  const FftTask th = h_inverse_task(M, axes, 0, J, spec, work, H, project, true, ra);
  const FftTask tc = trial_task(M, axes, 0, trial, twork, zero);
  PassShape ph, pc;
  hipError_t e = shape_pass(th, 3, ph);
  if (e == hipSuccess) e = shape_pass(tc, d + 6, pc);
  // sharing one launch (d > 1), the narrower pass takes more lines per workgroup
  if (e == hipSuccess && d > 1 && ph.threads != pc.threads)
    e = ph.threads < pc.threads ? shape_pass(th, 3, ph, pc.threads) : shape_pass(tc, d + 6, pc, ph.threads);
  if (e != hipSuccess) return e;
  ReduceSet rrh = rr;
  rrh.nblocks = (int)ph.gx;  // residual partials: one set per workgroup of the H pass
  const int nred = ro.nvals + rrh.nvals;
  if (d == 1) {
    // the H pass stores the spectrum that the CN solve reads: it runs first, then the
    // reduction beside the CN pass (which is also the trial fields' last)
    hipLaunchKernelGGL((k_fft_pass<1, true>), dim3(ph.gx, ph.ny), dim3(ph.threads), ph.lds, s, ph.t, CNArgs{}, M,
                       stop);
    PassShape pd;
    e = shape_pass(trial_task(M, axes, 0, trial, twork, zero), d + 6, pd, kRedThreads);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_reduce_fft<2, true>), dim3((unsigned)nred + pd.gx * pd.ny), dim3(kRedThreads), pd.lds, s,
                       ro, rrh, ot, pd.t, (int)pd.gx, cn, M, stop);
    return hipGetLastError();
  }
  // axis 0: H with the residual fold beside the CN solve and axis-0 inverse of the next
  // trial fields (the spectrum it reads was stored by the axis d-1 pass)
  const unsigned n1 = ph.gx * ph.ny, n2 = pc.gx * pc.ny;
  hipLaunchKernelGGL((k_fft_pass2<0, true, 2, false>), dim3(n1 + n2), dim3(std::max(ph.threads, pc.threads)),
                     std::max(ph.lds, pc.lds), s, ph.t, (int)ph.gx, (int)n1, pc.t, (int)pc.gx, cn, M, stop);
  // the reduction and outer test beside the trial fields' axis-1 inverse
  PassShape pe;
  e = shape_pass(trial_task(M, axes, 1, trial, twork, zero), d + 6, pe, kRedThreads);
  if (e != hipSuccess) return e;
  const dim3 ge((unsigned)nred + pe.gx * pe.ny);
  if (d == 2)
    hipLaunchKernelGGL((k_reduce_fft<0, true>), ge, dim3(kRedThreads), pe.lds, s, ro, rrh, ot, pe.t, (int)pe.gx, cn,
                       M, stop);
  else
    hipLaunchKernelGGL((k_reduce_fft<0, false>), ge, dim3(kRedThreads), pe.lds, s, ro, rrh, ot, pe.t, (int)pe.gx,
                       cn, M, stop);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the trial fields' remaining axes
  for (int l = 2; l < d; ++l) {
    e = fft_pass(M, trial_task(M, axes, l, trial, twork, zero), d + 6, 0, l == d - 1, &cn, s, stop);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_reduce(const double* partials, int nblocks, int64_t bstride, int64_t vstride, int nvals,
                         uint32_t max_mask, double* out, hipStream_t s, const int32_t* stop) {
  hipLaunchKernelGGL(k_reduce, dim3((unsigned)nvals), dim3(kBlock), 0, s, partials, nblocks, bstride, vstride, nvals,
                     max_mask, out, stop);
  return hipGetLastError();
}

ReduceSet reduce_chunks(const ReduceSet& r, double* scratch, hipStream_t s, const int32_t* stop) {
  if (r.nblocks <= kReduceChunkMin || r.bstride != 1) return r;
  const int chunk = (r.nblocks + kReduceChunks - 1) / kReduceChunks;
  const int nch = (r.nblocks + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_reduce_chunks, dim3((unsigned)nch, (unsigned)r.nvals), dim3(kBlock), 0, s, r.p, r.nblocks,
                     r.vstride, r.max_mask, chunk, scratch, stop);
  ReduceSet o = r;
  o.p = scratch;
  o.nblocks = nch;
  o.bstride = 1;
  o.vstride = nch;
  return o;
}

hipError_t launch_zero(double* y, int64_t n, hipStream_t s, const int32_t* stop) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero, dim3(nblk(n)), dim3(kBlock), 0, s, y, n, stop);
  return hipGetLastError();
}

hipError_t launch_reduce_outer(const ReduceSet& a, const ReduceSet& b, const OuterTest& t, hipStream_t s,
                               const int32_t* stop) {
  hipLaunchKernelGGL(k_reduce_outer, dim3((unsigned)(a.nvals + b.nvals)), dim3(kRedThreads), 0, s, a, b, t, stop);
  return hipGetLastError();
}

hipError_t launch_ctl_publish(int32_t* ctl, double* acc, int nacc, const CtlPublish& pub, uint32_t seq,
                              hipStream_t s) {
  if (nacc < 0 || nacc > 16) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ctl_publish, dim3(1), dim3(64), 0, s, ctl, acc, nacc, pub, seq);
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

hipError_t launch_fix_to_double(const unsigned long long* acc, double* out, int64_t n, const FixScale& fx,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fix_to_double, dim3(nblk(n)), dim3(kBlock), 0, s, acc, out, n, fx);
  return hipGetLastError();
}

hipError_t launch_abs_charge(const void* q, int prec, int64_t np, double* partials, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(k_abs_charge, dim3((unsigned)blocks), dim3(kBlock), 0, s, q, prec, np, partials);
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

hipError_t launch_unpermute_i32(const int32_t* src, int32_t* dst, const int32_t* id, int64_t np, hipStream_t s) {
  if (np <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_unpermute_i32, dim3(nblk(np)), dim3(kBlock), 0, s, src, dst, id, np);
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
