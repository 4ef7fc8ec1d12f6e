// gmhc_internal.h -- device-side argument blocks and launch wrappers shared by the
// HIP translation units of libgmhc (orbit pass, spectral field step, sorting, C ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fixsum.h"

namespace gmhc {

constexpr int kBlock = 256;       // threads per workgroup (4 wave64)
constexpr int kOrbitBlock = 64;   // threads per orbit-pass workgroup (one wave64)
constexpr int kMaxGL = 8;         // Gauss-Legendre points per segment supported
constexpr int kMaxCross = 8;      // knot crossings per axis per step supported
constexpr int kOrbitParts = 9;    // per-block partial values written by the orbit pass
constexpr int kMaxRefine = 3;     // particle refinement: at most 2^3 sub-steps per step
constexpr int kResParts = 8;      // per-block partial values written by the residual pass
constexpr int kDiagParts = 8;

// Indices of the orbit pass partials.
enum OrbitPart {
  OP_FAIL = 0,    // failed inner solves (sum)
  OP_ITERS = 1,   // inner evaluations (sum)
  OP_ITMAX = 2,   // inner evaluations (max)
  OP_KIN = 3,     // kinetic energy of p^{n+1} (sum)
  OP_WORK = 4,    // sum q v_out . E-bar
  OP_RA2 = 5,     // sum |R_A|^2
  OP_SEGS = 6,    // knot-split segments over all evaluations (sum)
  OP_XLIM = 7,    // failed solves whose orbit reached the knot-crossing limit (sum)
  OP_REFINED = 8  // particles solved with sub-steps (sum)
};

// Particle momenta, charges and orbit velocities are stored in the bulk type: FP64
// (prec 0) or FP32 (prec 1, the FP32-bulk mode).  Off the orbit pass they are read and
// written through these helpers and computed with in FP64.
__device__ __forceinline__ double ld_bulk(const void* p, int64_t i, int prec) {
  return prec ? (double)static_cast<const float*>(p)[i] : static_cast<const double*>(p)[i];
}
__device__ __forceinline__ void st_bulk(void* p, int64_t i, double v, int prec) {
  if (prec)
    static_cast<float*>(p)[i] = (float)v;
  else
    static_cast<double*>(p)[i] = v;
}

// Mesh geometry in the form the kernels use.
struct Mesh {
  int d;
  int n[3];          // powers of two (1 on unused axes)
  int ln[3];         // log2 n
  int64_t Ng;
  double lo[3];
  double len[3];
  double h[3];
  double inv_h[3];
  double kf[3];      // 2 pi / len (wavenumber of mode 1; 0 on unused axes)
  double dV;
  int shape;         // B-spline degree of the particle shape (1 or 2)
  FixScale fx;       // fixed-point scale of the deposited current and charge (fixsum.h)
};

// Arguments of the orbit pass (one thread per particle).
struct OrbitArgs {
  Mesh M;
  int64_t np;
  double dt, kappa;
  double tol_abs, tol_rel;
  int max_inner;
  int iterate;           // 0: single evaluation, 1: inner Picard loop
  int deposit;           // 1: deposit the orbit current
  int ngl;
  double glx[kMaxGL], glw[kMaxGL];
  // particle SoA blocks, component c of particle i at [c * ps + i].  Positions are
  // FP64; P, q and v are FP64, or FP32 in the FP32-bulk precision mode.
  int64_t ps;
  int precision;         // GMHC_FP64 (0) or GMHC_FP32_BULK (1)
  const double* x;       // [d]
  const void* P;         // [3]
  const void* q;         // [1]
  const void* vin;       // [3] v_in warm start (may be v itself)
  void* v;               // [3] out: v_out of the final evaluation
  double* xn;            // [d] out: wrapped x^n + dt v_in
  void* Pn;              // [3] out: P^{n+1}
  int32_t* iters;        // out: inner evaluations (may be null)
  // mesh arrays, component stride Ng
  const double* gphi;    // [d] grad_h phi^{n+1/2}
  const double* An;      // [3] A^n
  const double* Anp1;    // [3] A^{n+1}
  const double* Uh;      // [3] U^{n+1/2}
  unsigned long long* J;  // [3] orbit current accumulator, one fixed-point pair per value
  double* partials;      // [kOrbitParts][pstride]: value v of block b at v * pstride + b
  int64_t pstride;       // >= gridDim.x
  const int32_t* stop;   // optional device flag: nonzero = skip the pass
  // Convergence-triggered particle refinement (refine_levels > 0 and iterate = 1; else
  // rstate is null).  rstate[i]: bits 0-7 the particle's level within the step (K = 2^level
  // sub-steps; 0 the full step), bits 8-31 the evaluations of a full-step attempt of this
  // pass that failed.  rblock[b]: workgroup b of the pass holds a particle to refine.  Ab:
  // the vector potential A(j / 2^refine_levels) = (1 - s) A^n + s A^{n+1} at the interior
  // fractions, [j - 1][3][Ng].
  int refine_levels;
  int32_t* rstate;
  int32_t* rblock;
  double* Ab;
};

// With events e0 and e1, the launch itself records its start and stop in them (no
// separate marker packets on the stream); with no particles both are recorded at once.
// With refinement (a.rstate set) the refinement pass follows the main pass in the same
// call, and the events span both.
hipError_t launch_orbit(const OrbitArgs& a, int ngl, hipStream_t s, hipEvent_t e0 = nullptr,
                        hipEvent_t e1 = nullptr);
// Every particle back to the full step (refinement level 0), at the start of a step.
hipError_t launch_refine_reset(int32_t* rstate, int64_t np, hipStream_t s);

// ---- spectral field step ---------------------------------------------------------

struct FftPlanAxis {
  int N;
  int logN;
  int64_t stride;   // element stride of the axis (a power of two)
  int lstride;      // log2 stride
  int64_t nlines;   // Ng / N
  int T;            // lines per workgroup (a power of two)
  int lds_tw;       // 1: twiddles staged in LDS after the lines, 0: read from tw
  const double2* tw;  // exp(-2 pi i m / N), m < N/2
};

// Batched multi-dimensional FFT of `ncomp` components (component stride Ng).
// src may be real (src_r) or complex (src_c); dst may be real (dst_r, real part of
// the result) or complex (dst_c).  Forward is unnormalized, inverse carries 1/Ng.
// project = 1 zeroes the even-grid Nyquist planes of a forward result.
hipError_t fft_nd(const Mesh& M, const FftPlanAxis* axes, int ncomp, const double* src_r,
                  const double2* src_c, double2* dst_c, double* dst_r, double2* scratch_c,
                  bool inverse, bool project, hipStream_t s, const int32_t* stop = nullptr);

struct CNArgs {
  Mesh M;
  double dt, kappa2, sigma1, sigma2;
  const double2* jh;     // [3][Ng] projected trial current
  const double2* phi; const double2* psi; const double2* rho;
  const double2* A;      // [3][Ng]
  const double2* U;      // [3][Ng]
  double2* phi1; double2* psi1; double2* rho1;
  double2* A1; double2* U1;
  const int32_t* stop;   // optional device flag: nonzero = skip (outer iteration done)
};

struct ResidualArgs {
  Mesh M;
  double tol_abs, tol_rel;
  const double* H;       // [3][Ng]
  const double* j;       // [3][Ng]
  const double* gphi;    // [d][Ng]
  const double* Uh;      // [3][Ng]
  double* partials;      // [blocks][kResParts]
  const int32_t* stop;   // optional device flag: nonzero = skip
};

// out[v] = reduce over blocks b of partials[b * bstride + v * vstride]; max_mask bit v
// set = max, else sum.
hipError_t launch_reduce(const double* partials, int nblocks, int64_t bstride, int64_t vstride, int nvals,
                         uint32_t max_mask, double* out, hipStream_t s, const int32_t* stop = nullptr);

// Trial fields of the outer iteration: the Crank-Nicolson solve at the trial current
// (cn.jh) computed while loading the first inverse-FFT pass, the new
// state stored to cn.rho1 .. cn.U1, and the real trial fields [d+6][Ng] written to trial
// (i k phi^{n+1/2} (d), A^{n+1} (3), U^{n+1/2} (3)) through the complex scratch work;
// the fixed-point accumulator zero (3 Ng pairs) is cleared on the way (may be null).  Skipped when *cn.stop is set.
hipError_t field_trial(const Mesh& M, const FftPlanAxis* axes, const CNArgs& cn, double* trial, double2* work,
                       unsigned long long* zero, hipStream_t s);

// H = P J of the deposited current J (3 Ng fixed-point pairs, fixsum.h): the (Nyquist-projected when project)
// spectrum to spec [3][Ng] and the real field to H [3][Ng] through the complex scratch
// work, with the residual partials of ra (ra.H is H) written to ra.partials; their
// block count goes to *res_blocks.  The residual is folded into the last FFT pass when
// three components of an axis-0 line fit a workgroup.  Skipped when *ra.stop is set.
hipError_t field_h(const Mesh& M, const FftPlanAxis* axes, const unsigned long long* J, double2* spec,
                   double2* work, double* H, bool project, const ResidualArgs& ra, int* res_blocks, hipStream_t s);

// Partials of one reduction: out[v] = reduce over blocks b of p[b * bstride + v * vstride]
// for v < nvals; max_mask bit v set = max, else sum.
struct ReduceSet {
  const double* p;
  int nblocks;
  int64_t bstride, vstride;
  int nvals;
  uint32_t max_mask;
  double* out;
};

// Long reductions (more than kReduceChunkMin blocks of unit stride, such as the orbit
// pass's per-workgroup partials at 67M particles) first reduce up to kReduceChunks
// chunks of consecutive blocks in a fixed order into scratch [nvals][kReduceChunks];
// returns the set that reads those.  Shorter sets are returned unchanged.
constexpr int kReduceChunkMin = 16384;
constexpr int kReduceChunks = 1024;
ReduceSet reduce_chunks(const ReduceSet& r, double* scratch, hipStream_t s, const int32_t* stop = nullptr);

// Device-side outer test of Picard iteration k (ctl == nullptr: none): reads the pass
// results res[0..7] and residual sums res[koff..], accumulates the step report in acc and,
// when the mixed tests pass or an inner solve failed, sets ctl[0] (stop) and records the
// iteration k.  ctl: [0] stop, [1] failed, [2] iteration that stopped, [3] ticket
// counter (zero between launches).  acc: [0] evaluations, [1] segments, [2] inner max,
// [3] iterations, [4] failed count, [5] rms ratio, [6] max ratio, [7] sum |R_A|^2,
// [8] particle work, [9] mesh work, [10] evaluations of the last iteration.
struct OuterTest {
  const double* res;
  int koff;
  int32_t* ctl;
  double* acc;
  int k;
  double n3, tol_abs, tol_rel;
};

// Reductions a and b in one launch; with t.ctl, the last workgroup then runs the outer
// test on their results.  Skipped when *stop is set.
hipError_t launch_reduce_outer(const ReduceSet& a, const ReduceSet& b, const OuterTest& t, hipStream_t s,
                               const int32_t* stop);

// field_h, launch_reduce_outer (with rr.nblocks set to the residual's block count) and
// field_trial of the next iteration in fewer launches, for a next current equal to H
// (undamped Picard): the next trial fields are solved from the projected spectrum of H
// and transformed beside H's last pass and beside the reduction, into trial and the new
// state of cn, through the complex scratch twork (not work).  cn.jh must be spec.
// Requires field_h_next_fits (the residual folded into the last pass).
bool field_h_next_fits(const Mesh& M, const FftPlanAxis* axes);
hipError_t field_h_next(const Mesh& M, const FftPlanAxis* axes, const unsigned long long* J, double2* spec,
                        double2* work, double* H, bool project, const ResidualArgs& ra, const ReduceSet& ro,
                        const ReduceSet& rr, const OuterTest& ot, const CNArgs& cn, double* trial, double2* twork,
                        unsigned long long* zero, hipStream_t s);

// Host-visible (coherent pinned) copy of the Picard control block: ctl[0..3] and
// acc[0..nacc), then seq, written last with a system-scope release.
struct CtlPublish {
  int32_t* ctl;
  double* acc;
  uint32_t* seq;
};

// Device-side end of a Picard batch (one workgroup, nacc <= 16): ctl[0..3] and
// acc[0..nacc) are published to pub, then, when ctl[0] is set (the step stopped),
// cleared for the next step; the sequence number seq is stored last.
hipError_t launch_ctl_publish(int32_t* ctl, double* acc, int nacc, const CtlPublish& pub, uint32_t seq,
                              hipStream_t s);

// y = a x + b z over n values (z may be null).
hipError_t launch_axpbz(double* y, double a, const double* x, double b, const double* z, int64_t n,
                        hipStream_t s);

// Pairwise dot products of up to kMaxDotVecs vectors: per-block partials of the upper
// triangle (pairs (k1, k2), k1 <= k2, in row order), kMaxDots values per block.
constexpr int kMaxDotVecs = 9;
constexpr int kMaxDots = kMaxDotVecs * (kMaxDotVecs + 1) / 2;
struct DotArgs {
  int K;
  int64_t n;
  const double* v[kMaxDotVecs];
  double* partials;  // [blocks][kMaxDots]
};
hipError_t launch_dots(const DotArgs& a, int blocks, hipStream_t s);

// y[0..n) = 0 with a kernel (safe inside captured graphs, unlike a memset node).
hipError_t launch_zero(double* y, int64_t n, hipStream_t s, const int32_t* stop = nullptr);
hipError_t launch_axpy2(double* y, const double* x, double2* yc, const double2* xc, double beta,
                        int64_t nreal, int64_t ncplx, hipStream_t s, const int32_t* stop = nullptr);

// ---- initialization and diagnostics ----------------------------------------------

struct InitArgs {
  Mesh M;
  int64_t np;
  double kappa;
  int prec;              // bulk type of P, q, v
  const double* x[3];
  void* P[3];            // in: mechanical p; out: unchanged (canonical pass adds q A)
  const void* q;
  void* v[3];            // out: V(p)
  unsigned long long* rho;  // [Ng] fixed-point accumulator pairs
  unsigned long long* J;    // [3][Ng] fixed-point accumulator pairs
};
hipError_t launch_init_deposit(const InitArgs& a, hipStream_t s);

// out[i] = the FP64 value of fixed-point pair i of acc, i < n.
hipError_t launch_fix_to_double(const unsigned long long* acc, double* out, int64_t n, const FixScale& fx,
                                hipStream_t s);

// Per-block sums of |q_i| (bulk type prec) into partials[b * kDiagParts] (the other
// values of the block are zero), for the fixed-point scale.
hipError_t launch_abs_charge(const void* q, int prec, int64_t np, double* partials, int blocks, hipStream_t s);

struct InitSpecArgs {
  Mesh M;
  double kappa2, sigma1;
  int project;
  double2* rho; double2* phi; double2* psi; double2* A; double2* U; double2* J;
};
hipError_t launch_init_spectral(const InitSpecArgs& a, hipStream_t s);

struct CanonArgs {
  Mesh M;
  int64_t np;
  int prec;              // bulk type of P, q
  const double* x[3];
  void* P[3];
  const void* q;
  const double* A[3];    // real A^0
  double sign;           // +1: P = p + q A ; -1: p = P - q A
};
hipError_t launch_canonical(const CanonArgs& a, hipStream_t s);

struct KinArgs {
  Mesh M;
  int64_t np;
  double kappa;
  int prec;              // bulk type of P, q
  const double* x[3];
  const void* P[3];
  const void* q;
  const double* A[3];
  double* partials;      // [blocks][kDiagParts]: K, sum|q|(vy^2+vz^2), sum|q|
};
hipError_t launch_kinetic(const KinArgs& a, int blocks, hipStream_t s);

struct SpecDiagArgs {
  Mesh M;
  double kappa2, sigma1, sigma2;
  const double2* phi; const double2* psi; const double2* rho;
  const double2* A; const double2* U;
  double* partials;      // [blocks][kDiagParts]: sum|E|^2, sum|B|^2, sum|RG|^2, sum|RL|^2
};
hipError_t launch_spec_diag(const SpecDiagArgs& a, int blocks, hipStream_t s);

// Spectral E (= -i k phi - U) and B (= i k x A) into out [3][Ng].
hipError_t launch_spec_field(const Mesh& M, int which_e, const double2* phi, const double2* A,
                             const double2* U, double2* out, hipStream_t s);

// Loaded particle state into the bulk type: q_i from qd, P[c][i] = |q_i| kappa u[c][i]
// (mechanical momentum from u = p/(m kappa), with m = |q| as stored).
hipError_t launch_load_state(double* const u[3], const double* qd, void* const P[3], void* q, int prec,
                             double kappa, int64_t np, hipStream_t s);
hipError_t launch_iota(int32_t* id, int64_t np, hipStream_t s);

// ---- particle permutation -------------------------------------------------------
// dst[c][id[i]] = src[c][i] for c < ncomp (un-permute to load order); src in the
// given type (prec 0 FP64, 1 FP32), dst FP64.
hipError_t launch_unpermute(const void* const* src, int src_prec, double* const* dst, int ncomp,
                            const int32_t* id, int64_t np, hipStream_t s);
// dst[id[i]] = src[i] for per-particle int32 values.
hipError_t launch_unpermute_i32(const int32_t* src, int32_t* dst, const int32_t* id, int64_t np, hipStream_t s);
// dst[c][i] = src[c][id[i]]: gather load-order FP64 data into sorted order, stored in
// the given type.
hipError_t launch_permute_in(const double* const* src, void* const* dst, int dst_prec, int ncomp,
                             const int32_t* id, int64_t np, hipStream_t s);


// ---- host-side configuration helpers (api.hip) ---------------------------------

}  // namespace gmhc
struct gmhc_config;
namespace gmhc {
// The validation rules gmhc_create documents.
bool config_ok(const gmhc_config& c);
// Mesh geometry and the Gauss-Legendre rule (nodes and weights on [0, 1], kMaxGL slots)
// of a valid configuration.
void set_geometry(const gmhc_config& c, Mesh& M, int& ngl, double* glx, double* glw);
// The calling thread's last gmhc_orbit_pass_static error (static_pass.hip).
const char* static_last_error();

// Sort of particles by nearest-node cell: the stable radix sort (stable = 1) or the
// counting sort with atomic cursors (stable = 0); see sort.hip.
struct SortArgs {
  Mesh M;
  int64_t np;
  int ncomp;              // number of arrays to move
  const void* src[12];
  void* dst[12];
  int32_t esz[12];        // element size of each array, 4 or 8 bytes
  const int32_t* id_src;
  int32_t* id_dst;
  const double* x[3];     // positions (also among src)
  int32_t* key;           // [np]
  int32_t* count;         // [Ng + 1] (counting sort)
  int32_t* cursor;        // [Ng] (counting sort)
  int stable;             // 1: the stable radix sort
  int32_t* key2;          // [np] (radix sort: keys and indices ping-pong)
  int32_t* idx;           // [np]
  int32_t* idx2;          // [np]
  int32_t* rcount;        // [radix_count_ints(np)] digit counts and scan block sums
  // radix sort: the particles whose orbit under the accepted velocity v (bulk type, prec)
  // crosses a knot follow the others, within each cell or (where they are dense) after all
  // of them, so most waves walk one orbit segment and the rest two; xcount [1]: their count
  const void* v[3];
  int prec;
  double dt;
  int32_t* xcount;         // [cross_count_ints()]
};
hipError_t sort_by_cell(const SortArgs& a, void* scan_tmp, size_t scan_tmp_bytes, hipStream_t s);
size_t sort_scan_tmp_bytes(int64_t Ng);
int64_t radix_count_ints(int64_t np);
int cross_count_ints();

}  // namespace gmhc
