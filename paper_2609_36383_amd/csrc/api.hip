// api.hip -- the C ABI of libgmhc (include/gmhc.h): context, workspace carving, the
// outer current iteration of the implicit step (Algorithm 1 with damped Picard on
// the mesh current), initialization, diagnostics and read-outs.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "gmhc.h"
#include "adjoint.h"
#include "gmhc_internal.h"

using namespace gmhc;

static_assert(GMHC_MAX_ORBIT_CELLS == kMaxCross - 1, "the orbit pass supports |dt v / h| < kMaxCross - 1");
static_assert(kMaxRefine == 3, "gmhc_config.refine_levels is documented as 0..3");

struct gmhc_ctx {
  gmhc_config cfg;
  Mesh M;
  int ngl = 0;
  double glx[kMaxGL], glw[kMaxGL];
  int64_t np = 0;
  hipStream_t stream = nullptr;
  int device = 0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool bound = false, loaded = false, initialized = false, have_pot = false, frozen = false,
       pass_done = false;
  // particles (sorted order), SoA.  Positions are FP64 in both modes; momenta, charges
  // and orbit velocities are stored in the bulk type (double, or float in FP32-bulk).
  int prec = GMHC_FP64;
  size_t es = sizeof(double);  // bytes per bulk element
  double* x[3] = {};
  double* x2[3] = {};
  void* P[3] = {};
  void* P2[3] = {};
  void* q = nullptr;
  void* q2 = nullptr;
  void* vb[3] = {};     // accepted orbit-velocity iterate (warm start)
  void* vw[3] = {};     // working iterate of the current step / last frozen pass
  bool vin_first = false;  // the next orbit pass starts from vb (first pass of a step)
  bool timed_now = false;  // orbit launches of the current call are timed
  bool ctl_clean = false;  // the device control block and accumulators are zero
  bool ahead = false;      // the next step's first outer iteration is already enqueued
  double* pscr[3] = {}; // FP64 staging for loads and read-outs
  int32_t* id = nullptr;
  int32_t* id2 = nullptr;
  int32_t* iters = nullptr;
  int32_t* key = nullptr;
  int32_t* key2 = nullptr;  // radix sort buffers
  int32_t* ridx = nullptr;
  int32_t* ridx2 = nullptr;
  int32_t* rcount = nullptr;
  int32_t* xcount = nullptr;  // knot-crossing particles counted by the sort
  // refinement (refine_levels > 0): per-particle level within the step, per-workgroup
  // flags of the orbit pass, and the interpolated vector potentials of the sub-steps
  int32_t* rstate = nullptr;
  int32_t* rblock = nullptr;
  double* Ab = nullptr;
  bool pass_levels = false;  // the last frozen pass ran with refinement (rstate holds its levels)
  // mesh
  double* tacc = nullptr;   // [d+6][Ng] block in the trial layout whose A part is A^n; at
                            // commit it trades places with the converged trial block
  double* An = nullptr;     // [3][Ng] real A^n (= tacc + d Ng)
  double* trial[2] = {};    // [d+6][Ng] real: grad phi^{n+1/2}, A^{n+1}, U^{n+1/2}, by parity
  unsigned long long* Jdep = nullptr;  // [3][Ng] deposited current, fixed-point pairs (fixsum.h)
  double* pot0 = nullptr;   // [6][Ng] loaded initial potentials A0, U0 (real space)
  double* jr[3] = {};       // real current slots [3][Ng]; slot 0 = accepted J^{n-1/2}
  double2* jh[3] = {};      // spectral current slots
  double2* S0 = nullptr;    // accepted spectral state [9][Ng]: phi psi rho A(3) U(3)
  double2* S1[2] = {};      // trial spectral state, by outer-iteration parity
  double2* cout = nullptr;  // [9][Ng] complex scratch (CN outputs, FFT work)
  double2* cscr = nullptr;  // [9][Ng] complex scratch
  double* rscr = nullptr;   // [9][Ng] real scratch
  int32_t* count = nullptr;
  int32_t* cursor = nullptr;
  void* scan_tmp = nullptr;
  size_t scan_tmp_bytes = 0;
  double* partials = nullptr;
  double* pchunk = nullptr;  // first-level sums of long reductions [kOrbitParts][kReduceChunks]
  int64_t max_blocks = 0;
  // outer Anderson solver (outer_scheme 1): iterate, residual, direction [3 Ng] and
  // the history columns (differences of iterates and of residuals)
  double* jA = nullptr;
  double* rA = nullptr;
  double* dA = nullptr;
  double* hJ[8] = {};
  double* hR[8] = {};
  // device-side Picard control (see run_picard): stop flags, report accumulators,
  // pinned host copies, per-iteration timing events, predicted iteration count
  int32_t* dctl = nullptr;
  double* dacc = nullptr;
  int32_t* hctl = nullptr;       // coherent pinned block: control, accumulators, sequence
  double* hacc = nullptr;
  uint32_t* hseq = nullptr;
  CtlPublish dpub{};              // the same block as the device addresses it
  uint32_t pub_seq = 0;           // sequence number of the last batch published
  std::vector<hipEvent_t> evs;
  int last_outer = 0;
  double* ddot = nullptr;   // device dot products [kMaxDots]
  double* hdot = nullptr;   // pinned host copy
  double* dres = nullptr;   // device results [32]
  double* hres = nullptr;   // pinned host results [32]
  double2* tw[3] = {};
  FftPlanAxis axes[3];
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // HIP graphs of the outer iteration, keyed by the buffers and slots they use
  struct GraphEntry {
    std::vector<uintptr_t> key;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;
  bool graphs_off = false;  // capture failed once: run eagerly
  // bookkeeping
  double t = 0.0;
  int64_t step = 0;
  double E0 = 0.0;
  double last_chain = 0.0, last_work = 0.0, last_rr = 0.0, last_mr = 0.0;
  gmhc_pass_report last_pass{};
  std::string err;
};

namespace {

const int kResOff = 16;  // offset of residual results in dres
const size_t kCtlBytes = sizeof(int32_t) * 4 + sizeof(double) * 16;  // control block + accumulators

int32_t fail(gmhc_ctx* c, int32_t st, const std::string& msg) {
  if (c) c->err = msg;
  return st;
}

// Discard an enqueued first outer iteration: the next step starts afresh, with the
// control block cleared again.
void drop_ahead(gmhc_ctx* ctx) {
  if (!ctx->ahead) return;
  ctx->ahead = false;
  ctx->ctl_clean = false;
}

#define HIPCK(expr)                                                                  \
  do {                                                                               \
    hipError_t e_ = (expr);                                                          \
    if (e_ != hipSuccess)                                                            \
      return fail(ctx, GMHC_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Gauss-Legendre nodes and weights on [0,1]: Newton on P_n in long double.
void gl01(int n, double* x, double* w) {
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 0; i < n; ++i) {
    long double z = cosl(pi * (n - i - 0.25L) / (n + 0.5L));  // ascending order
    long double dp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      long double p1 = 1.0L, p2 = 0.0L;
      for (int k = 1; k <= n; ++k) {
        long double p3 = p2;
        p2 = p1;
        p1 = ((2.0L * k - 1.0L) * z * p2 - (k - 1.0L) * p3) / k;
      }
      dp = n * (z * p1 - p2) / (z * z - 1.0L);
      long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) break;
    }
    long double p1 = 1.0L, p2 = 0.0L;
    for (int k = 1; k <= n; ++k) {
      long double p3 = p2;
      p2 = p1;
      p1 = ((2.0L * k - 1.0L) * z * p2 - (k - 1.0L) * p3) / k;
    }
    dp = n * (z * p1 - p2) / (z * z - 1.0L);
    x[i] = (double)(0.5L * (1.0L + z));
    w[i] = (double)(1.0L / ((1.0L - z * z) * dp * dp));
  }
}

int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * count;
    return p;
  }
};

// Lay out every device buffer; with base == nullptr only the size is computed.
size_t carve(gmhc_ctx* c, char* base, int64_t np) {
  Carver cv{base};
  const int d = c->M.d;
  const int64_t Ng = c->M.Ng;
  const size_t N = (size_t)std::max<int64_t>(np, 1);
  // each SoA group is one contiguous block with component stride N
  const size_t es = c->es;
  double* xb = cv.take<double>(d * N);
  double* x2b = cv.take<double>(d * N);
  char* Pb = cv.take<char>(3 * N * es);
  char* P2b = cv.take<char>(3 * N * es);
  char* vbb = cv.take<char>(3 * N * es);
  char* vwb = cv.take<char>(3 * N * es);
  double* psb = cv.take<double>(3 * N);
  for (int l = 0; l < 3; ++l) {
    c->x[l] = (l < d && xb) ? xb + l * N : nullptr;
    c->x2[l] = (l < d && x2b) ? x2b + l * N : nullptr;
    c->P[l] = Pb ? Pb + l * N * es : nullptr;
    c->P2[l] = P2b ? P2b + l * N * es : nullptr;
    c->vb[l] = vbb ? vbb + l * N * es : nullptr;
    c->vw[l] = vwb ? vwb + l * N * es : nullptr;
    c->pscr[l] = psb ? psb + l * N : nullptr;
  }
  c->q = cv.take<char>(N * es);
  c->q2 = cv.take<char>(N * es);
  c->id = cv.take<int32_t>(N);
  c->id2 = cv.take<int32_t>(N);
  c->iters = cv.take<int32_t>(N);
  c->key = cv.take<int32_t>(N);
  c->key2 = cv.take<int32_t>(N);
  c->ridx = cv.take<int32_t>(N);
  c->ridx2 = cv.take<int32_t>(N);
  c->rcount = cv.take<int32_t>((size_t)radix_count_ints(np));
  c->xcount = cv.take<int32_t>((size_t)cross_count_ints());
  const int rl = c->cfg.refine_levels;
  if (rl > 0) c->rstate = cv.take<int32_t>(N);
  c->tacc = cv.take<double>((size_t)(d + 6) * Ng);
  c->An = c->tacc + (size_t)d * Ng;
  for (int p = 0; p < 2; ++p) c->trial[p] = cv.take<double>((size_t)(d + 6) * Ng);
  c->Jdep = cv.take<unsigned long long>(6 * Ng);
  c->pot0 = cv.take<double>(6 * Ng);
  for (int s = 0; s < 3; ++s) {
    c->jr[s] = cv.take<double>(3 * Ng);
    c->jh[s] = cv.take<double2>(3 * Ng);
  }
  c->S0 = cv.take<double2>(9 * Ng);
  for (int p = 0; p < 2; ++p) c->S1[p] = cv.take<double2>(9 * Ng);
  c->cout = cv.take<double2>(9 * Ng);
  c->cscr = cv.take<double2>(9 * Ng);
  c->rscr = cv.take<double>(9 * Ng);
  c->count = cv.take<int32_t>(Ng + 1);
  c->cursor = cv.take<int32_t>(Ng + 1);
  c->scan_tmp_bytes = sort_scan_tmp_bytes(Ng);
  c->scan_tmp = cv.take<char>(c->scan_tmp_bytes);
  c->max_blocks = std::max<int64_t>((np + kOrbitBlock - 1) / kOrbitBlock, 1024);
  // orbit partials, then residual / diagnostic partials: at most one block per axis-0
  // line (the residual folded into the last FFT pass) or 1024
  const int64_t res_cap = std::max<int64_t>(1024, c->M.Ng / c->M.n[0]);
  c->partials = cv.take<double>((size_t)c->max_blocks * kOrbitParts + (size_t)res_cap * 8);
  if (rl > 0) {
    c->rblock = cv.take<int32_t>((size_t)c->max_blocks);
    c->Ab = cv.take<double>((size_t)((1 << rl) - 1) * 3 * Ng);
  }
  c->pchunk = cv.take<double>((size_t)kOrbitParts * kReduceChunks);
  c->dres = cv.take<double>(64);
  c->ddot = cv.take<double>(kMaxDots);
  // control block [4] int32 then the report accumulators [16] double, contiguous
  c->dctl = cv.take<int32_t>(kCtlBytes / sizeof(int32_t));
  c->dacc = c->dctl ? reinterpret_cast<double*>(c->dctl + 4) : nullptr;
  if (c->cfg.outer_scheme == 1) {
    c->jA = cv.take<double>(3 * Ng);
    c->rA = cv.take<double>(3 * Ng);
    c->dA = cv.take<double>(3 * Ng);
    for (int m = 0; m < c->cfg.anderson_m; ++m) {
      c->hJ[m] = cv.take<double>(3 * Ng);
      c->hR[m] = cv.take<double>(3 * Ng);
    }
  }
  for (int l = 0; l < d; ++l) c->tw[l] = cv.take<double2>(std::max(c->M.n[l] / 2, 1));
  return (cv.off + 255) & ~(size_t)255;
}

struct DevGuard {
  int old = -1;
  explicit DevGuard(int dev) {
    if (hipGetDevice(&old) != hipSuccess) old = -1;
    if (old != dev) (void)hipSetDevice(dev);
  }
  ~DevGuard() {
    if (old >= 0) (void)hipSetDevice(old);
  }
};

hipMemcpyKind kind_of(int32_t ptr_kind, bool to_device) {
  if (ptr_kind == GMHC_DEVICE) return hipMemcpyDeviceToDevice;
  return to_device ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost;
}

OrbitArgs orbit_args(gmhc_ctx* c, int iterate, int par = 0) {
  OrbitArgs a{};
  a.M = c->M;
  a.np = c->np;
  a.dt = c->cfg.dt;
  a.kappa = c->cfg.kappa;
  a.tol_abs = c->cfg.tol_inner_abs;
  a.tol_rel = c->cfg.tol_inner_rel;
  a.max_inner = c->cfg.max_inner;
  a.iterate = iterate;
  a.deposit = 1;
  a.ngl = c->ngl;
  for (int k = 0; k < kMaxGL; ++k) {
    a.glx[k] = c->glx[k];
    a.glw[k] = c->glw[k];
  }
  a.ps = std::max<int64_t>(c->np, 1);
  a.precision = c->cfg.precision;
  a.x = c->x[0];
  a.xn = c->x2[0];
  a.P = c->P[0];
  a.Pn = c->P2[0];
  a.vin = c->vin_first ? c->vb[0] : c->vw[0];
  a.v = c->vw[0];
  a.gphi = c->trial[par];
  a.Anp1 = c->trial[par] + (int64_t)c->M.d * c->M.Ng;
  a.Uh = c->trial[par] + (int64_t)(c->M.d + 3) * c->M.Ng;
  a.An = c->An;
  a.J = c->Jdep;
  a.q = c->q;
  a.iters = c->iters;
  a.partials = c->partials;
  a.pstride = c->max_blocks;
  if (c->cfg.refine_levels > 0 && iterate) {
    a.refine_levels = c->cfg.refine_levels;
    a.rstate = c->rstate;
    a.rblock = c->rblock;
    a.Ab = c->Ab;
  }
  return a;
}

// Residual and diagnostic partials, after the orbit pass's.
double* res_partials(const gmhc_ctx* c) { return c->partials + (size_t)c->max_blocks * kOrbitParts; }

int orbit_blocks(const gmhc_ctx* c) { return (int)((c->np + kOrbitBlock - 1) / kOrbitBlock); }

// Orbit pass + first-level reduction to dres[0..7]; optional HIP-event timing.
int32_t run_orbit(gmhc_ctx* ctx, int iterate, double* ms) {
  OrbitArgs a = orbit_args(ctx, iterate);
  HIPCK(launch_zero(reinterpret_cast<double*>(ctx->Jdep), 6 * ctx->M.Ng, ctx->stream));
  if (a.rstate) HIPCK(launch_refine_reset(ctx->rstate, ctx->np, ctx->stream));
  ctx->pass_levels = a.rstate != nullptr;
  const bool timed = ctx->timed_now;
  HIPCK(launch_orbit(a, ctx->ngl, ctx->stream, timed ? ctx->ev0 : nullptr, timed ? ctx->ev1 : nullptr));
  const int nb = (int)((ctx->np + kOrbitBlock - 1) / kOrbitBlock);
  if (nb > 0) {
    const ReduceSet r = reduce_chunks(
        ReduceSet{ctx->partials, nb, 1, ctx->max_blocks, kOrbitParts, 1u << OP_ITMAX, ctx->dres}, ctx->pchunk,
        ctx->stream);
    HIPCK(launch_reduce(r.p, r.nblocks, r.bstride, r.vstride, r.nvals, r.max_mask, r.out, ctx->stream));
  } else {
    HIPCK(hipMemsetAsync(ctx->dres, 0, sizeof(double) * kOrbitParts, ctx->stream));
  }
  (void)ms;
  return GMHC_OK;
}

int res_blocks(const gmhc_ctx* c) {
  return (int)std::min<int64_t>((c->M.Ng + kBlock - 1) / kBlock, 1024);
}

int32_t wait_results(gmhc_ctx* ctx, double* orbit_ms);

int32_t fetch_results(gmhc_ctx* ctx, double* orbit_ms) {
  HIPCK(hipMemcpyAsync(ctx->hres, ctx->dres, sizeof(double) * 32, hipMemcpyDeviceToHost, ctx->stream));
  return wait_results(ctx, orbit_ms);
}

int32_t wait_results(gmhc_ctx* ctx, double* orbit_ms) {
  HIPCK(hipStreamSynchronize(ctx->stream));
  if (ctx->timed_now && orbit_ms) {
    float f = 0.0f;
    HIPCK(hipEventElapsedTime(&f, ctx->ev0, ctx->ev1));
    *orbit_ms += (double)f;
  }
  return GMHC_OK;
}

int32_t sort_particles(gmhc_ctx* ctx) {
  SortArgs a{};
  a.M = ctx->M;
  a.np = ctx->np;
  int k = 0;
  const int d = ctx->M.d;
  for (int l = 0; l < d; ++l) {
    a.esz[k] = sizeof(double);
    a.src[k] = ctx->x[l];
    a.dst[k++] = ctx->x2[l];
  }
  for (int l = 0; l < 3; ++l) {
    a.esz[k] = (int32_t)ctx->es;
    a.src[k] = ctx->P[l];
    a.dst[k++] = ctx->P2[l];
  }
  for (int l = 0; l < 3; ++l) {
    a.esz[k] = (int32_t)ctx->es;
    a.src[k] = ctx->vb[l];
    a.dst[k++] = ctx->vw[l];
  }
  a.esz[k] = (int32_t)ctx->es;
  a.src[k] = ctx->q;
  a.dst[k++] = ctx->q2;
  a.ncomp = k;
  a.id_src = ctx->id;
  a.id_dst = ctx->id2;
  for (int l = 0; l < d; ++l) a.x[l] = ctx->x[l];
  a.key = ctx->key;
  a.count = ctx->count;
  a.cursor = ctx->cursor;
  a.stable = ctx->cfg.deterministic != 0;
  a.key2 = ctx->key2;
  a.idx = ctx->ridx;
  a.idx2 = ctx->ridx2;
  a.rcount = ctx->rcount;
  for (int l = 0; l < 3; ++l) a.v[l] = ctx->vb[l];
  a.prec = ctx->prec;
  a.dt = ctx->cfg.dt;
  a.xcount = ctx->xcount;
  HIPCK(sort_by_cell(a, ctx->scan_tmp, ctx->scan_tmp_bytes, ctx->stream));
  for (int l = 0; l < d; ++l) std::swap(ctx->x[l], ctx->x2[l]);
  for (int l = 0; l < 3; ++l) {
    std::swap(ctx->P[l], ctx->P2[l]);
    std::swap(ctx->vb[l], ctx->vw[l]);
  }
  std::swap(ctx->q, ctx->q2);
  std::swap(ctx->id, ctx->id2);
  return GMHC_OK;
}

// Real-space read-out of accepted field `which` into rscr; returns ncomp.
int32_t field_to_rscr(gmhc_ctx* ctx, int32_t which, int* ncomp) {
  const int64_t Ng = ctx->M.Ng;
  double2* S = ctx->S0;
  const double2* src = nullptr;
  int nc = 1;
  switch (which) {
    case GMHC_PHI: src = S; break;
    case GMHC_PSI: src = S + Ng; break;
    case GMHC_RHO: src = S + 2 * Ng; break;
    case GMHC_A:
      HIPCK(hipMemcpyAsync(ctx->rscr, ctx->An, sizeof(double) * 3 * Ng, hipMemcpyDeviceToDevice, ctx->stream));
      *ncomp = 3;
      return GMHC_OK;
    case GMHC_U: src = S + 6 * Ng; nc = 3; break;
    case GMHC_J:
      HIPCK(hipMemcpyAsync(ctx->rscr, ctx->jr[0], sizeof(double) * 3 * Ng, hipMemcpyDeviceToDevice, ctx->stream));
      *ncomp = 3;
      return GMHC_OK;
    case GMHC_E:
    case GMHC_B:
      HIPCK(launch_spec_field(ctx->M, which == GMHC_E, S, S + 3 * Ng, S + 6 * Ng, ctx->cscr, ctx->stream));
      src = ctx->cscr;
      nc = 3;
      break;
    default: return fail(ctx, GMHC_EINVAL, "unknown field selector");
  }
  HIPCK(fft_nd(ctx->M, ctx->axes, nc, nullptr, src, nullptr, ctx->rscr, ctx->cout, true, false, ctx->stream));
  *ncomp = nc;
  return GMHC_OK;
}

// Fixed-point scale of the deposited charge and current (fixsum.h): every sum of
// contributions to one node is bounded by max(kappa, 1) sum_i |q_i| / dV (|v| < kappa,
// and the shape weights of a particle sum to one).  Synchronizes the stream.
int32_t set_fix_scale(gmhc_ctx* ctx) {
  double qsum = 0.0;
  if (ctx->np > 0) {
    const int kb = (int)std::min<int64_t>((ctx->np + kBlock - 1) / kBlock, 1024);
    HIPCK(launch_abs_charge(ctx->q, ctx->prec, ctx->np, ctx->partials, kb, ctx->stream));
    HIPCK(launch_reduce(ctx->partials, kb, kDiagParts, 1, 1, 0u, ctx->dres, ctx->stream));
    HIPCK(hipMemcpyAsync(ctx->hres, ctx->dres, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  }
  HIPCK(hipStreamSynchronize(ctx->stream));
  if (ctx->np > 0) qsum = ctx->hres[0];
  if (!isfinite(qsum)) return fail(ctx, GMHC_EINVAL, "non-finite particle charges");
  ctx->M.fx = fix_scale(std::max(ctx->cfg.kappa, 1.0) * qsum / ctx->M.dV);
  return GMHC_OK;
}

// Text of an inner-solve failure: failed particles, and those whose orbit reached the
// supported knot-crossing range.
std::string inner_fail_msg(double failed, double xlim) {
  std::string m = "particle inner solve failed (" + std::to_string((long long)failed) + " particles)";
  if (xlim > 0.0)
    m += "; " + std::to_string((long long)xlim) + " of them with an orbit of " +
         std::to_string(GMHC_MAX_ORBIT_CELLS) +
         " or more cells on some axis (|dt v / h| >= GMHC_MAX_ORBIT_CELLS, the supported knot-crossing range)";
  return m;
}

// Image of the accepted state (gmhc_save / gmhc_load): this header, then the sections
// listed by state_sections, each at an 8-byte boundary.
struct StateHeader {
  char magic[8];
  int32_t abi, dim, n[3], precision, shape, have_pot, last_outer, pad;
  int64_t np, ng, step, bytes;
  double t, E0, last_chain, last_work, last_rr, last_mr;
  double fx[3];
};
constexpr char kStateMagic[8] = {'G', 'M', 'H', 'C', 'S', 'T', 'A', 'T'};

struct StateSection {
  void* dev;
  size_t bytes;
};

// Device buffers of the accepted state, in image order: particles in the internal
// (sorted) order with their load-order ids, positions, canonical momenta, accepted orbit
// velocities, charges; the spectral state, real A^n, the accepted current (real and
// spectral) and the loaded initial potentials.
std::vector<StateSection> state_sections(gmhc_ctx* c) {
  const size_t np = (size_t)c->np, Ng = (size_t)c->M.Ng, es = c->es;
  std::vector<StateSection> v;
  for (int l = 0; l < c->M.d; ++l) v.push_back({c->x[l], sizeof(double) * np});
  for (int l = 0; l < 3; ++l) v.push_back({c->P[l], es * np});
  for (int l = 0; l < 3; ++l) v.push_back({c->vb[l], es * np});
  v.push_back({c->q, es * np});
  v.push_back({c->id, sizeof(int32_t) * np});
  v.push_back({c->S0, sizeof(double2) * 9 * Ng});
  v.push_back({c->An, sizeof(double) * 3 * Ng});
  v.push_back({c->jr[0], sizeof(double) * 3 * Ng});
  v.push_back({c->jh[0], sizeof(double2) * 3 * Ng});
  v.push_back({c->pot0, sizeof(double) * 6 * Ng});
  return v;
}

size_t state_bytes(gmhc_ctx* c) {
  size_t off = (sizeof(StateHeader) + 7) & ~(size_t)7;
  for (const auto& sc : state_sections(c)) off += (sc.bytes + 7) & ~(size_t)7;
  return off;
}

int ncomp_of(int32_t which) {
  return (which == GMHC_PHI || which == GMHC_PSI || which == GMHC_RHO) ? 1 : 3;
}

}  // namespace

namespace gmhc {

// Host-side validation of a configuration (the rules gmhc_create documents).
bool config_ok(const gmhc_config& c) {
  if (c.dim < 1 || c.dim > 3) return false;
  int64_t ng = 1;
  for (int l = 0; l < c.dim; ++l) {
    const int n = c.n[l];
    if (n < 4 || n > 4096 || (n & (n - 1)) != 0) return false;
    ng *= n;
    if (ng > (int64_t)1 << 30) return false;  // node indices stay within int32
    if (!(c.len[l] > 0.0) || !isfinite(c.lo[l])) return false;
  }
  if (!(c.dt > 0.0) || !(c.kappa > 0.0) || !(c.sigma1 > 0.0) || !(c.sigma2 > 0.0)) return false;
  if (fabs(c.sigma1 - c.kappa * c.kappa * c.sigma2) > 1e-14 * fabs(c.sigma1)) return false;
  if (c.gl_order < 0 || c.gl_order > kMaxGL) return false;
  if (c.shape_order < 0 || c.shape_order > 2) return false;
  if (c.precision != GMHC_FP64 && c.precision != GMHC_FP32_BULK) return false;
  if (c.max_outer < 1 || c.max_inner < 1 || !(c.beta > 0.0 && c.beta <= 1.0)) return false;
  if (c.timing < 0) return false;
  if (c.deterministic != 0 && c.deterministic != 1) return false;
  if (c.refine_levels < 0 || c.refine_levels > kMaxRefine) return false;
  if (c.outer_scheme != 0 && c.outer_scheme != 1) return false;
  if (c.outer_scheme == 1 &&
      (c.anderson_m < 1 || c.anderson_m > 8 || c.anderson_start < 1 || c.ls_halvings < 0 || c.ls_halvings > 30 ||
       !(c.anderson_lambda >= 0.0) || !(c.ls_decrease >= 0.0 && c.ls_decrease < 1.0) || !(c.ls_growth >= 1.0)))
    return false;
  if (c.tol_outer_abs < 0 || c.tol_outer_rel < 0 || c.tol_inner_abs < 0 || c.tol_inner_rel < 0) return false;
  return true;
}

// Mesh geometry and the Gauss-Legendre rule of a valid configuration.
void set_geometry(const gmhc_config& c, Mesh& M, int& ngl, double* glx, double* glw) {
  M = Mesh{};
  M.d = c.dim;
  M.shape = c.shape_order == 1 ? 1 : 2;
  M.Ng = 1;
  M.dV = 1.0;
  for (int l = 0; l < 3; ++l) {
    const bool r = l < c.dim;
    M.n[l] = r ? c.n[l] : 1;
    M.lo[l] = r ? c.lo[l] : 0.0;
    M.len[l] = r ? c.len[l] : 1.0;
    M.ln[l] = ilog2(M.n[l]);
    M.h[l] = M.len[l] / M.n[l];
    M.inv_h[l] = 1.0 / M.h[l];
    M.kf[l] = r ? 2.0 * M_PI / M.len[l] : 0.0;
    M.Ng *= M.n[l];
    if (r) M.dV *= M.h[l];
  }
  ngl = c.gl_order ? c.gl_order : (M.shape == 1 ? (c.dim + 2) / 2 : c.dim + 1);
  for (int k = 0; k < kMaxGL; ++k) glx[k] = glw[k] = 0.0;
  gl01(ngl, glx, glw);
}

}  // namespace gmhc

extern "C" {

int32_t gmhc_abi_version(void) { return GMHC_ABI_VERSION; }

const char* gmhc_status_str(int32_t s) {
  switch (s) {
    case GMHC_OK: return "ok";
    case GMHC_EINVAL: return "invalid argument";
    case GMHC_ESTATE: return "call out of order";
    case GMHC_ENOMEM: return "workspace too small";
    case GMHC_EDEVICE: return "HIP runtime error";
    case GMHC_EINNER: return "particle inner solve failed";
    case GMHC_ENOCONV: return "outer iteration did not converge";
    default: return "unknown status";
  }
}

const char* gmhc_last_error(const gmhc_ctx* ctx) { return ctx ? ctx->err.c_str() : static_last_error(); }

int32_t gmhc_create(const gmhc_config* cfg, gmhc_ctx** out) {
  if (!cfg || !out) return GMHC_EINVAL;
  *out = nullptr;
  if (!config_ok(*cfg)) return GMHC_EINVAL;
  gmhc_ctx* ctx = new gmhc_ctx();
  ctx->cfg = *cfg;
  ctx->prec = cfg->precision;
  ctx->es = cfg->precision == GMHC_FP32_BULK ? sizeof(float) : sizeof(double);
  set_geometry(*cfg, ctx->M, ctx->ngl, ctx->glx, ctx->glw);
  *out = ctx;
  return GMHC_OK;
}

void gmhc_destroy(gmhc_ctx* ctx) {
  if (!ctx) return;
  if (ctx->bound) {
    DevGuard g(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->hres) (void)hipHostFree(ctx->hres);
    if (ctx->hdot) (void)hipHostFree(ctx->hdot);
    if (ctx->hctl) (void)hipHostFree(ctx->hctl);
    for (hipEvent_t e : ctx->evs) (void)hipEventDestroy(e);
    for (auto& e : ctx->graphs) (void)hipGraphExecDestroy(e.exec);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
  }
  delete ctx;
}

int32_t gmhc_workspace_bytes(const gmhc_ctx* ctx, int64_t n_particles, size_t* bytes) {
  if (!ctx || !bytes || n_particles < 0 || n_particles > INT32_MAX) return GMHC_EINVAL;
  gmhc_ctx tmp;
  tmp.cfg = ctx->cfg;
  tmp.M = ctx->M;
  tmp.prec = ctx->prec;
  tmp.es = ctx->es;
  *bytes = carve(&tmp, nullptr, n_particles);
  return GMHC_OK;
}

int32_t gmhc_bind(gmhc_ctx* ctx, int64_t n_particles, void* dev_workspace, size_t bytes,
                  void* hip_stream) {
  if (!ctx) return GMHC_EINVAL;
  if (ctx->bound) return fail(ctx, GMHC_ESTATE, "context already bound");
  if (n_particles < 0 || n_particles > INT32_MAX || !dev_workspace)
    return fail(ctx, GMHC_EINVAL, "bad particle count or workspace");
  size_t need = carve(ctx, nullptr, n_particles);
  if (bytes < need) return fail(ctx, GMHC_ENOMEM, "workspace smaller than gmhc_workspace_bytes");
  if ((reinterpret_cast<uintptr_t>(dev_workspace) & 255) != 0)
    return fail(ctx, GMHC_EINVAL, "workspace must be 256-byte aligned");
  HIPCK(hipGetDevice(&ctx->device));
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  ctx->ws = static_cast<char*>(dev_workspace);
  ctx->ws_bytes = bytes;
  ctx->np = n_particles;
  carve(ctx, ctx->ws, n_particles);
  HIPCK(hipHostMalloc(reinterpret_cast<void**>(&ctx->hres), sizeof(double) * 64, hipHostMallocDefault));
  HIPCK(hipHostMalloc(reinterpret_cast<void**>(&ctx->hdot), sizeof(double) * kMaxDots, hipHostMallocDefault));
  // the control block is published by a kernel straight into coherent host memory
  HIPCK(hipHostMalloc(reinterpret_cast<void**>(&ctx->hctl), kCtlBytes + 64, hipHostMallocMapped | hipHostMallocCoherent));
  ctx->hacc = reinterpret_cast<double*>(ctx->hctl + 4);
  ctx->hseq = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(ctx->hctl) + kCtlBytes);
  *ctx->hseq = 0;
  {
    void* dp = nullptr;
    HIPCK(hipHostGetDevicePointer(&dp, ctx->hctl, 0));
    char* db = static_cast<char*>(dp);
    ctx->dpub = CtlPublish{reinterpret_cast<int32_t*>(db), reinterpret_cast<double*>(db + 4 * sizeof(int32_t)),
                           reinterpret_cast<uint32_t*>(db + kCtlBytes)};
  }
  HIPCK(hipEventCreate(&ctx->ev0));
  HIPCK(hipEventCreate(&ctx->ev1));
  // FFT plans and twiddles exp(-2 pi i m / N)
  const long double pi = 3.141592653589793238462643383279502884L;
  int64_t stride = 1;
  for (int l = 0; l < ctx->M.d; ++l) {
    const int N = ctx->M.n[l];
    std::vector<double2> tw(std::max(N / 2, 1));
    for (int m = 0; m < N / 2; ++m) {
      long double ang = -2.0L * pi * m / N;
      tw[m] = make_double2((double)cosl(ang), (double)sinl(ang));
    }
    HIPCK(hipMemcpy(ctx->tw[l], tw.data(), sizeof(double2) * tw.size(), hipMemcpyHostToDevice));
    FftPlanAxis& ax = ctx->axes[l];
    ax.N = N;
    ax.logN = ilog2(N);
    ax.stride = stride;
    ax.lstride = ilog2((int)stride);
    ax.nlines = ctx->M.Ng / N;
    ax.T = std::max(1, 4096 / N);
    if (ax.T > ax.nlines) ax.T = (int)ax.nlines;
    ax.tw = ctx->tw[l];
    stride *= N;
  }
  HIPCK(hipMemsetAsync(ctx->S0, 0, sizeof(double2) * 9 * ctx->M.Ng, ctx->stream));
  HIPCK(hipMemsetAsync(ctx->jr[0], 0, sizeof(double) * 3 * ctx->M.Ng, ctx->stream));
  HIPCK(hipMemsetAsync(ctx->jh[0], 0, sizeof(double2) * 3 * ctx->M.Ng, ctx->stream));
  HIPCK(hipMemsetAsync(ctx->An, 0, sizeof(double) * 3 * ctx->M.Ng, ctx->stream));
  for (int p = 0; p < 2; ++p)
    HIPCK(hipMemsetAsync(ctx->trial[p], 0, sizeof(double) * (ctx->M.d + 6) * ctx->M.Ng, ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));
  ctx->bound = true;
  return GMHC_OK;
}

int32_t gmhc_load_particles(gmhc_ctx* ctx, const double* x, const double* u, const double* q,
                            int32_t ptr_kind) {
  if (!ctx) return GMHC_EINVAL;
  drop_ahead(ctx);
  if (!ctx->bound) return fail(ctx, GMHC_ESTATE, "bind before loading particles");
  const int64_t np = ctx->np;
  if (np > 0 && (!x || !u || !q)) return fail(ctx, GMHC_EINVAL, "null particle array");
  DevGuard g(ctx->device);
  const size_t b = sizeof(double) * (size_t)np;
  for (int l = 0; l < ctx->M.d; ++l)
    if (np) HIPCK(hipMemcpyAsync(ctx->x[l], x + l * np, b, kind_of(ptr_kind, true), ctx->stream));
  // u and q are staged in FP64 (pscr, and x2 which is free until the first sort),
  // then stored in the bulk type with p = |q| kappa u
  for (int l = 0; l < 3; ++l)
    if (np) HIPCK(hipMemcpyAsync(ctx->pscr[l], u + l * np, b, kind_of(ptr_kind, true), ctx->stream));
  if (np) HIPCK(hipMemcpyAsync(ctx->x2[0], q, b, kind_of(ptr_kind, true), ctx->stream));
  HIPCK(launch_load_state(ctx->pscr, ctx->x2[0], ctx->P, ctx->q, ctx->prec, ctx->cfg.kappa, np, ctx->stream));
  HIPCK(launch_iota(ctx->id, np, ctx->stream));
  for (int l = 0; l < 3; ++l)
    if (np) HIPCK(hipMemsetAsync(ctx->vb[l], 0, ctx->es * (size_t)np, ctx->stream));
  int32_t st = set_fix_scale(ctx);
  if (st) return st;
  ctx->loaded = true;
  ctx->initialized = false;
  return GMHC_OK;
}

int32_t gmhc_load_potentials(gmhc_ctx* ctx, const double* A0, const double* U0, int32_t ptr_kind) {
  if (!ctx || !A0 || !U0) return GMHC_EINVAL;
  drop_ahead(ctx);
  if (!ctx->bound) return fail(ctx, GMHC_ESTATE, "bind before loading potentials");
  DevGuard g(ctx->device);
  const int64_t Ng = ctx->M.Ng;
  // kept in real space: every later gmhc_initialize starts from them
  HIPCK(hipMemcpyAsync(ctx->pot0, A0, sizeof(double) * 3 * Ng, kind_of(ptr_kind, true), ctx->stream));
  HIPCK(hipMemcpyAsync(ctx->pot0 + 3 * Ng, U0, sizeof(double) * 3 * Ng, kind_of(ptr_kind, true), ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));
  ctx->have_pot = true;
  ctx->initialized = false;
  return GMHC_OK;
}

int32_t gmhc_initialize(gmhc_ctx* ctx) {
  if (!ctx) return GMHC_EINVAL;
  drop_ahead(ctx);
  if (!ctx->loaded) return fail(ctx, GMHC_ESTATE, "load particles before initialize");
  DevGuard g(ctx->device);
  const Mesh& M = ctx->M;
  const int64_t Ng = M.Ng;
  hipStream_t s = ctx->stream;
  if (ctx->have_pot)
    HIPCK(fft_nd(M, ctx->axes, 6, ctx->pot0, nullptr, ctx->S0 + 3 * Ng, nullptr, nullptr, false, false, s));
  else
    HIPCK(hipMemsetAsync(ctx->S0 + 3 * Ng, 0, sizeof(double2) * 6 * Ng, s));
  // point-shape deposit of rho and J as fixed-point sums (rho in cscr, J in Jdep), then
  // to FP64 in rscr (rho) and rscr + Ng (J); v = V(p)
  unsigned long long* rho_fx = reinterpret_cast<unsigned long long*>(ctx->cscr);
  HIPCK(hipMemsetAsync(rho_fx, 0, sizeof(unsigned long long) * 2 * Ng, s));
  HIPCK(hipMemsetAsync(ctx->Jdep, 0, sizeof(unsigned long long) * 6 * Ng, s));
  InitArgs ia{};
  ia.M = M;
  ia.np = ctx->np;
  ia.kappa = ctx->cfg.kappa;
  for (int l = 0; l < 3; ++l) {
    ia.x[l] = ctx->x[l];
    ia.P[l] = ctx->P[l];
    ia.v[l] = ctx->vb[l];
  }
  ia.J = ctx->Jdep;
  ia.q = ctx->q;
  ia.prec = ctx->prec;
  ia.rho = rho_fx;
  HIPCK(launch_init_deposit(ia, s));
  HIPCK(launch_fix_to_double(rho_fx, ctx->rscr, Ng, M.fx, s));
  HIPCK(launch_fix_to_double(ctx->Jdep, ctx->rscr + Ng, 3 * Ng, M.fx, s));
  HIPCK(fft_nd(M, ctx->axes, 1, ctx->rscr, nullptr, ctx->S0 + 2 * Ng, nullptr, nullptr, false, false, s));
  HIPCK(fft_nd(M, ctx->axes, 3, ctx->rscr + Ng, nullptr, ctx->jh[0], nullptr, nullptr, false, false, s));
  InitSpecArgs sa{};
  sa.M = M;
  sa.kappa2 = ctx->cfg.kappa * ctx->cfg.kappa;
  sa.sigma1 = ctx->cfg.sigma1;
  sa.project = ctx->cfg.project_nyquist;
  sa.phi = ctx->S0;
  sa.psi = ctx->S0 + Ng;
  sa.rho = ctx->S0 + 2 * Ng;
  sa.A = ctx->S0 + 3 * Ng;
  sa.U = ctx->S0 + 6 * Ng;
  sa.J = ctx->jh[0];
  HIPCK(launch_init_spectral(sa, s));
  HIPCK(fft_nd(M, ctx->axes, 3, nullptr, ctx->jh[0], nullptr, ctx->jr[0], ctx->cscr, true, false, s));
  HIPCK(fft_nd(M, ctx->axes, 3, nullptr, ctx->S0 + 3 * Ng, nullptr, ctx->An, ctx->cscr, true, false, s));
  CanonArgs ca{};
  ca.M = M;
  ca.np = ctx->np;
  for (int l = 0; l < 3; ++l) {
    ca.x[l] = ctx->x[l];
    ca.P[l] = ctx->P[l];
    ca.A[l] = ctx->An + l * Ng;
  }
  ca.q = ctx->q;
  ca.prec = ctx->prec;
  ca.sign = 1.0;
  HIPCK(launch_canonical(ca, s));
  HIPCK(hipStreamSynchronize(s));
  ctx->t = 0.0;
  ctx->step = 0;
  ctx->last_chain = ctx->last_work = ctx->last_rr = ctx->last_mr = 0.0;
  ctx->initialized = true;
  gmhc_diag d;
  int32_t st = gmhc_diagnostics(ctx, &d);
  if (st) return st;
  ctx->E0 = d.total;
  return GMHC_OK;
}

// Parts of one outer iteration's device work (see enqueue_outer).
// Parts of an outer iteration: all, the field solve before the orbit pass, the orbit
// pass, the field step after it, and the last two together.
enum OuterPart { OUTER_ALL = 0, OUTER_PRE = 1, OUTER_ORBIT = 2, OUTER_POST = 3, OUTER_TAIL = 4 };

// CN solve arguments: the trial current spectrum jh against the accepted state S0, new
// state into S1.
CNArgs cn_args(const gmhc_ctx* ctx, const double2* jh, double2* S1, const int32_t* stop) {
  const int64_t Ng = ctx->M.Ng;
  CNArgs ca{};
  ca.M = ctx->M;
  ca.dt = ctx->cfg.dt;
  ca.kappa2 = ctx->cfg.kappa * ctx->cfg.kappa;
  ca.sigma1 = ctx->cfg.sigma1;
  ca.sigma2 = ctx->cfg.sigma2;
  ca.jh = jh;
  ca.phi = ctx->S0;
  ca.psi = ctx->S0 + Ng;
  ca.rho = ctx->S0 + 2 * Ng;
  ca.A = ctx->S0 + 3 * Ng;
  ca.U = ctx->S0 + 6 * Ng;
  ca.phi1 = S1;
  ca.psi1 = S1 + Ng;
  ca.rho1 = S1 + 2 * Ng;
  ca.A1 = S1 + 3 * Ng;
  ca.U1 = S1 + 6 * Ng;
  ca.stop = stop;
  return ca;
}

// Device work of one outer iteration for the trial current in slot cur, with H(j)
// written to slot hs: CN field step and trial fields (PRE), the orbit pass with its
// inner Picard loop (ORBIT, bracketed by the timing events when timing is on), then
// the pass reduction, projected orbit current, outer residual and the copy of the
// results to pinned host memory (POST).  Enqueued without host synchronization, so
// the parts can be captured as HIP graphs.
//
// With a device control block (stop != nullptr) every kernel first checks the stop flag
// and returns when an earlier iteration already converged or failed; the iteration ends
// with the device-side outer test of iteration k and, for beta < 1, the damped update of
// the next trial current in slot hs, instead of copying the results to the host.
//
// The trial fields and new-time spectra of iteration k live in the buffers of parity
// k & 1 (host-controlled iterations pass k = 0).  With next (undamped Picard under device
// control) POST also solves and transforms those of iteration k + 1 into the other
// parity, from the projected spectrum of H, which is that iteration's current; the next
// iteration then runs as OUTER_TAIL, without PRE.  The iteration that converges keeps its
// own buffers.
int32_t enqueue_outer(gmhc_ctx* ctx, int cur, int hs, int part, const int32_t* stop = nullptr, int k = 0,
                      hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr, bool next = false) {
  const Mesh& M = ctx->M;
  const int64_t Ng = M.Ng;
  const int d = M.d;
  const int par = k & 1;
  hipStream_t s = ctx->stream;
  if (!e0) {
    e0 = ctx->ev0;
    e1 = ctx->ev1;
  }
  if (part == OUTER_ALL || part == OUTER_PRE) {
    // CN solve, trial fields in real space, deposit buffer cleared
    HIPCK(field_trial(M, ctx->axes, cn_args(ctx, ctx->jh[cur], ctx->S1[par], stop), ctx->trial[par], ctx->cout,
                      ctx->Jdep, s));
  }
  if (part == OUTER_ALL || part == OUTER_ORBIT || part == OUTER_TAIL) {
    // timed launches record their own start and stop (never inside a captured graph:
    // timed graph runs launch the orbit pass eagerly)
    const bool timed = ctx->timed_now && (part == OUTER_ORBIT || stop != nullptr);
    OrbitArgs oa = orbit_args(ctx, 1, par);
    oa.stop = stop;
    HIPCK(launch_orbit(oa, ctx->ngl, s, timed ? e0 : nullptr, timed ? e1 : nullptr));
    ctx->vin_first = false;  // later passes of the step start from their predecessor's v_out
  }
  if (part == OUTER_ALL || part == OUTER_POST || part == OUTER_TAIL) {
    // H(j) = P J_orb in spectral and real space, with the residual partials
    ResidualArgs ra{};
    ra.M = M;
    ra.tol_abs = ctx->cfg.tol_outer_abs;
    ra.tol_rel = ctx->cfg.tol_outer_rel;
    ra.j = ctx->jr[cur];
    ra.gphi = ctx->trial[par];
    ra.Uh = ctx->trial[par] + (int64_t)(d + 3) * Ng;
    ra.partials = res_partials(ctx);  // disjoint from orbit partials
    ra.stop = stop;
    const bool proj = ctx->cfg.project_nyquist != 0;
    // pass and residual sums, then (device control) the outer test
    const ReduceSet ro = reduce_chunks(
        ReduceSet{ctx->partials, orbit_blocks(ctx), 1, ctx->max_blocks, kOrbitParts, 1u << OP_ITMAX, ctx->dres},
        ctx->pchunk, s, stop);
    ReduceSet rr{ra.partials, 0, kResParts, 1, kResParts, 1u << 3, ctx->dres + kResOff};
    OuterTest ot{};
    if (stop)
      ot = OuterTest{ctx->dres, kResOff, ctx->dctl, ctx->dacc, k, 3.0 * (double)Ng, ctx->cfg.tol_outer_abs,
                     ctx->cfg.tol_outer_rel};
    if (next) {
      // the next iteration's trial fields are solved and transformed beside these passes
      const int np1 = par ^ 1;
      HIPCK(field_h_next(M, ctx->axes, ctx->Jdep, ctx->jh[hs], ctx->cscr, ctx->jr[hs], proj, ra, ro, rr, ot,
                         cn_args(ctx, ctx->jh[hs], ctx->S1[np1], stop), ctx->trial[np1], ctx->cout, ctx->Jdep, s));
      return GMHC_OK;
    }
    int rb = 0;
    HIPCK(field_h(M, ctx->axes, ctx->Jdep, ctx->jh[hs], ctx->cscr, ctx->jr[hs], proj, ra, &rb, s));
    rr.nblocks = rb;
    HIPCK(launch_reduce_outer(ro, rr, ot, s, stop));
    if (stop) {
      if (ctx->cfg.beta != 1.0)
        HIPCK(launch_axpy2(ctx->jr[hs], ctx->jr[cur], ctx->jh[hs], ctx->jh[cur], 1.0 - ctx->cfg.beta, 3 * Ng,
                           3 * Ng, s, stop));
    } else {
      HIPCK(hipMemcpyAsync(ctx->hres, ctx->dres, sizeof(double) * 32, hipMemcpyDeviceToHost, s));
    }
  }
  return GMHC_OK;
}

// The graph of enqueue_outer(cur, hs, part) for the current buffer layout: reused
// while the buffers and slots it touches are the same (they alternate with commits and
// sorts), captured on first use.  *ex = nullptr when capture is not possible; the
// caller then runs the same work eagerly.
int32_t outer_graph(gmhc_ctx* ctx, int cur, int hs, int part, hipGraphExec_t* ex) {
  *ex = nullptr;
  std::vector<uintptr_t> key = {(uintptr_t)cur, (uintptr_t)hs, (uintptr_t)part,
                                (uintptr_t)ctx->S0, (uintptr_t)ctx->S1[0], (uintptr_t)ctx->q,
                                (uintptr_t)(ctx->vin_first ? ctx->vb[0] : ctx->vw[0])};
  for (int l = 0; l < 3; ++l) {
    key.push_back((uintptr_t)ctx->x[l]);
    key.push_back((uintptr_t)ctx->x2[l]);
    key.push_back((uintptr_t)ctx->P[l]);
    key.push_back((uintptr_t)ctx->P2[l]);
    key.push_back((uintptr_t)ctx->vw[l]);
    key.push_back((uintptr_t)ctx->jr[l]);
    key.push_back((uintptr_t)ctx->jh[l]);
  }
  for (auto& e : ctx->graphs)
    if (e.key == key) {
      *ex = e.exec;
      return GMHC_OK;
    }
  hipStream_t s = ctx->stream;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    ctx->graphs_off = true;
    return GMHC_OK;
  }
  const int32_t st = enqueue_outer(ctx, cur, hs, part);
  hipGraph_t g = nullptr;
  const hipError_t ee = hipStreamEndCapture(s, &g);
  hipGraphExec_t exec = nullptr;
  const bool ok = st == GMHC_OK && ee == hipSuccess && g &&
                  hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (!ok) {
    (void)hipGetLastError();
    ctx->err.clear();
    ctx->graphs_off = true;
    return GMHC_OK;
  }
  if (ctx->graphs.size() >= 24) {
    (void)hipGraphExecDestroy(ctx->graphs.front().exec);
    ctx->graphs.erase(ctx->graphs.begin());
  }
  ctx->graphs.push_back({key, exec});
  *ex = exec;
  return GMHC_OK;
}

// One outer iteration's device work: replayed graphs (with the orbit launch eager
// between two graphs when its launches are timed), or eager launches.
int32_t run_outer(gmhc_ctx* ctx, int cur, int hs, bool& use_graph, int32_t& replays) {
  hipStream_t s = ctx->stream;
  if (use_graph) {
    const int parts[3] = {OUTER_PRE, OUTER_ORBIT, OUTER_POST};
    const int np = ctx->timed_now ? 3 : 1;
    hipGraphExec_t ex[3] = {nullptr, nullptr, nullptr};
    bool ok = true;
    for (int k = 0; k < np && ok; ++k) {
      if (np == 3 && parts[k] == OUTER_ORBIT) continue;  // launched eagerly
      int32_t st = outer_graph(ctx, cur, hs, np == 3 ? parts[k] : OUTER_ALL, &ex[k]);
      if (st) return st;
      ok = ex[k] != nullptr;
    }
    if (ok) {
      for (int k = 0; k < np; ++k) {
        if (np == 3 && parts[k] == OUTER_ORBIT) {
          int32_t st = enqueue_outer(ctx, cur, hs, OUTER_ORBIT);
          if (st) return st;
        } else {
          HIPCK(hipGraphLaunch(ex[k], s));
        }
      }
      ctx->vin_first = false;  // the iteration's orbit pass has run
      replays += 1;
      return GMHC_OK;
    }
    use_graph = false;
  }
  if (ctx->timed_now) {
    for (int part : {OUTER_PRE, OUTER_ORBIT, OUTER_POST}) {
      int32_t st = enqueue_outer(ctx, cur, hs, part);
      if (st) return st;
    }
    return GMHC_OK;
  }
  return enqueue_outer(ctx, cur, hs, OUTER_ALL);
}

// Evaluate the outer map at the trial current in slot cur (H(j) written to slot hs)
// and read back the pass and residual results: rr and mr are the mixed RMS and
// max-node test ratios.  GMHC_EINNER if an inner particle solve failed.
int32_t eval_outer(gmhc_ctx* ctx, int cur, int hs, gmhc_step_report& R, bool& use_graph, double& rr, double& mr) {
  const int64_t Ng = ctx->M.Ng, np = ctx->np;
  int32_t st = run_outer(ctx, cur, hs, use_graph, R.graph_replays);
  if (st) return st;
  double oms = 0.0;
  st = wait_results(ctx, &oms);
  if (st) return st;
  R.orbit_ms += oms;
  R.orbit_launches += 1;
  const double* h = ctx->hres;
  R.outer_iters += 1;
  R.evaluations += (int64_t)llround(h[OP_ITERS]);
  R.segments += (int64_t)llround(h[OP_SEGS]);
  R.inner_max = (int32_t)llround(h[OP_ITMAX]);
  R.inner_mean = np ? h[OP_ITERS] / (double)np : 0.0;
  R.refined = (int32_t)llround(h[OP_REFINED]);
  if (h[OP_FAIL] > 0.0) return fail(ctx, GMHC_EINNER, inner_fail_msg(h[OP_FAIL], h[OP_XLIM]));
  const double* r = ctx->hres + kResOff;
  const double n3 = 3.0 * (double)Ng;
  rr = sqrt(r[0] / n3) /
       (ctx->cfg.tol_outer_abs + 0.5 * ctx->cfg.tol_outer_rel * (sqrt(r[1] / n3) + sqrt(r[2] / n3)));
  mr = r[3];
  R.res_rms_ratio = rr;
  R.res_max_ratio = mr;
  return GMHC_OK;
}

// Commit the state of the converged evaluation at the trial current in slot cur, whose
// trial fields and new-time spectra sit in the buffers of parity par; ra2, pwork and
// mwork are its sum |R_A|^2, particle work and mesh work.
int32_t commit_outer(gmhc_ctx* ctx, int cur, double rr, double mr, double ra2, double pwork, double mwork,
                     int par = 0) {
  const Mesh& M = ctx->M;
  const int64_t Ng = M.Ng, np = ctx->np;
  const int d = M.d;
  std::swap(ctx->S0, ctx->S1[par]);
  // A^{n+1} of the converged trial fields becomes A^n: their block takes the place of
  // the accepted one, whose storage the next trial fields of this parity reuse (the
  // device work of the step has finished or is ordered before any later use)
  std::swap(ctx->tacc, ctx->trial[par]);
  ctx->An = ctx->tacc + (int64_t)d * Ng;
  if (cur != 0) {  // the accepted current becomes slot 0
    std::swap(ctx->jr[0], ctx->jr[cur]);
    std::swap(ctx->jh[0], ctx->jh[cur]);
  }
  for (int l = 0; l < d; ++l) std::swap(ctx->x[l], ctx->x2[l]);
  for (int l = 0; l < 3; ++l) {
    std::swap(ctx->P[l], ctx->P2[l]);
    std::swap(ctx->vb[l], ctx->vw[l]);
  }
  // no wait: the next step's work is ordered behind the copy on the same stream, and
  // every read-out synchronizes the stream itself
  ctx->last_chain = np ? sqrt(ra2 / (3.0 * (double)np)) : 0.0;
  ctx->last_work = ctx->cfg.dt * (pwork - mwork * M.dV);
  ctx->last_rr = rr;
  ctx->last_mr = mr;
  ctx->t += ctx->cfg.dt;
  ctx->step += 1;
  return GMHC_OK;
}

// Commit after a host-driven evaluation (its results are in hres).
int32_t commit_host(gmhc_ctx* ctx, int cur, double rr, double mr) {
  return commit_outer(ctx, cur, rr, mr, ctx->hres[OP_RA2], ctx->hres[OP_WORK], ctx->hres[kResOff + 4]);
}

// Damped Picard with the outer test on the device: iterations are enqueued in batches
// (the size of the last step's count) without waiting; each ends with the device-side
// test, and once it passes (or an inner solve fails) the kernels of the iterations
// already queued return at once.  The host synchronizes once per batch, so the GPU does
// not idle between outer iterations.
// Per-step flags: the first orbit pass reads the accepted v from vb, and the orbit
// launches of every timing-th step are timed.  With refinement every particle starts
// the step at the full step again.
int32_t begin_step(gmhc_ctx* ctx) {
  ctx->vin_first = true;
  const int tk = ctx->cfg.timing;
  ctx->timed_now = tk == 1 || (tk > 1 && ctx->step % tk == 0);
  if (ctx->rstate) HIPCK(launch_refine_reset(ctx->rstate, ctx->np, ctx->stream));
  return GMHC_OK;
}

// Enqueue outer iteration k (1-based) of a device-controlled Picard step from current
// slot cur into slot 1 or 2 (whichever cur is not); timed steps record events 2(k-1)
// and 2(k-1)+1 around the orbit launch.
int32_t enqueue_picard_iter(gmhc_ctx* ctx, int k, int cur) {
  const int hs = (cur == 1) ? 2 : 1;
  // undamped: each iteration also prepares the next one's trial fields
  const bool next = ctx->cfg.beta == 1.0 && field_h_next_fits(ctx->M, ctx->axes);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (ctx->timed_now) {
    while ((int)ctx->evs.size() < 2 * k) {
      hipEvent_t e;
      HIPCK(hipEventCreate(&e));
      ctx->evs.push_back(e);
    }
    e0 = ctx->evs[2 * (k - 1)];
    e1 = ctx->evs[2 * (k - 1) + 1];
  }
  return enqueue_outer(ctx, cur, hs, (next && k > 1) ? OUTER_TAIL : OUTER_ALL, ctx->dctl, k, e0, e1, next);
}

// Steps that can start before the caller asks for them: device-controlled Picard
// without graphs, and no particle sort due at the step's start.
bool can_run_ahead(const gmhc_ctx* ctx) {
  const gmhc_config& c = ctx->cfg;
  const bool graph = c.graphs != 0 && ctx->stream != nullptr && !ctx->graphs_off;
  const bool sort = c.sort_every > 0 && ctx->step % c.sort_every == 0;
  return c.outer_scheme != 1 && !graph && !sort && c.max_outer >= 1;
}

// After a commit, enqueue the next step's first outer iteration at once: it reads only
// the accepted state and writes only scratch (trial fields, the new-time spectra, the
// deposit, the slot 1 current, the new particle slots and the control block), so the
// GPU need not wait for the caller's next gmhc_step.  The read-outs of the accepted
// state (diagnostics, particles, fields, mode amplitudes) leave it in place: they use
// only reduction and transform scratch that the iteration has consumed by the time they
// run and that the next iteration rewrites before reading.  Every other call discards
// it (drop_ahead), and the next step then starts afresh.
int32_t run_ahead(gmhc_ctx* ctx) {
  if (!can_run_ahead(ctx)) return GMHC_OK;
  int32_t st = begin_step(ctx);
  if (st) return st;
  ctx->ctl_clean = false;
  st = enqueue_picard_iter(ctx, 1, 0);
  if (st) return st;
  ctx->ahead = true;
  return GMHC_OK;
}

int32_t run_picard(gmhc_ctx* ctx, gmhc_step_report& R) {
  hipStream_t s = ctx->stream;
  const int64_t np = ctx->np;
  const int maxo = ctx->cfg.max_outer;
  std::vector<int> slot(maxo + 1, 0);
  int k = 0, cur = 0;
  if (ctx->ahead) {  // iteration 1 was enqueued when the previous step committed
    ctx->ahead = false;
    k = 1;
    cur = 1;
  } else {
    if (!ctx->ctl_clean) HIPCK(hipMemsetAsync(ctx->dctl, 0, kCtlBytes, s));
    ctx->ctl_clean = false;
  }
  const bool timed = ctx->timed_now;
  int batch = std::max(1, std::min(ctx->last_outer, maxo));
  int k0 = 0;
  while (true) {
    while (k < k0 + batch && k < maxo) {
      ++k;
      slot[k] = cur;
      int32_t st = enqueue_picard_iter(ctx, k, cur);
      if (st) return st;
      cur = (cur == 1) ? 2 : 1;
    }
    // the batch-end kernel publishes the control block to host memory and, once the step
    // stopped, clears it for the next step on the device, so nothing waits for the host
    // between steps
    if (++ctx->pub_seq == 0) ++ctx->pub_seq;
    const uint32_t want = ctx->pub_seq;
    HIPCK(launch_ctl_publish(ctx->dctl, ctx->dacc, 16, ctx->dpub, want, s));
    // spin on the sequence number (a blocking wait or an event query adds tens of
    // microseconds of wake-up); the stream is queried now and then so that the wait
    // ends even if the word never arrives
    for (uint32_t spin = 1; __atomic_load_n(ctx->hseq, __ATOMIC_ACQUIRE) != want; ++spin) {
      if (spin % 4096 != 0) continue;
      const hipError_t q = hipStreamQuery(s);
      if (q == hipErrorNotReady) continue;
      if (q != hipSuccess) HIPCK(q);
      if (__atomic_load_n(ctx->hseq, __ATOMIC_ACQUIRE) != want)
        return fail(ctx, GMHC_EDEVICE, "the batch control block was not published");
    }
    const int32_t* c = ctx->hctl;
    const double* acc = ctx->hacc;
    const int ran = (int)llround(acc[3]);  // iterations that ran (the rest returned at once)
    if (timed && std::min(k, ran) > k0)
      HIPCK(hipEventSynchronize(ctx->evs[2 * (std::min(k, ran) - 1) + 1]));
    if (timed)
      for (int kk = k0 + 1; kk <= std::min(k, ran); ++kk) {
        float f = 0.0f;
        HIPCK(hipEventElapsedTime(&f, ctx->evs[2 * (kk - 1)], ctx->evs[2 * (kk - 1) + 1]));
        R.orbit_ms += (double)f;
      }
    R.outer_iters = ran;
    R.outer_updates = ran - 1;  // every evaluation after the first follows one Picard update
    R.orbit_launches = ran;
    R.evaluations = (int64_t)llround(acc[0]);
    R.segments = (int64_t)llround(acc[1]);
    R.inner_max = (int32_t)llround(acc[2]);
    R.inner_mean = np ? acc[10] / (double)np : 0.0;
    R.refined = (int32_t)llround(acc[12]);
    R.res_rms_ratio = acc[5];
    R.res_max_ratio = acc[6];
    if (c[0]) {
      ctx->ctl_clean = true;  // cleared by launch_ctl_publish
      if (c[1]) return fail(ctx, GMHC_EINNER, inner_fail_msg(acc[4], acc[11]));
      ctx->last_outer = c[2];
      int32_t st = commit_outer(ctx, slot[c[2]], acc[5], acc[6], acc[7], acc[8], acc[9], c[2] & 1);
      if (st) return st;
      return run_ahead(ctx);
    }
    if (k >= maxo) return fail(ctx, GMHC_ENOCONV, "outer iteration limit reached");
    k0 = k;
    batch = 1;
  }
}

// Solve A x = b (n <= 8, row-major A) by Gaussian elimination with partial pivoting;
// false when a pivot vanishes or the result is not finite.
bool solve_small(double* A, double* b, int n, double* x) {
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (fabs(A[r * n + c]) > fabs(A[p * n + c])) p = r;
    const double piv = A[p * n + c];
    if (!(fabs(piv) > 0.0) || !isfinite(piv)) return false;
    if (p != c) {
      for (int k = 0; k < n; ++k) std::swap(A[c * n + k], A[p * n + k]);
      std::swap(b[c], b[p]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      b[r] -= f * b[c];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    double v = b[c];
    for (int k = c + 1; k < n; ++k) v -= A[c * n + k] * x[k];
    x[c] = v / A[c * n + c];
    if (!isfinite(x[c])) return false;
  }
  return true;
}

// The paper's outer solver: limited-memory type-II Anderson acceleration of the current
// iteration (section on the implicit solver).  With residual differences dR and
// iterate differences dJ as history columns,
//   [dR^T dR + lambda tr(dR^T dR)/m_h I] gamma = dR^T r,  j_A = j + beta r - (dJ + beta dR) gamma,
// backtracking alpha = 1, 1/2, ... along the direction, accepting a trial whose scaled
// RMS residual drops by at least a factor 1 - c alpha and whose scaled max-node
// residual grows by at most the growth limit.  The history is cleared when unusable,
// when a trial's RMS residual grows past the growth limit, or when the Anderson
// direction is rejected, which is then retried as damped Picard (j + beta r).
int32_t step_anderson(gmhc_ctx* ctx, gmhc_step_report& R, bool& use_graph) {
  const Mesh& M = ctx->M;
  const int64_t n = 3 * M.Ng;
  hipStream_t s = ctx->stream;
  const gmhc_config& c = ctx->cfg;
  double rr = 0.0, mr = 0.0;
  int32_t st = eval_outer(ctx, 0, 2, R, use_graph, rr, mr);
  if (st) return st;
  if (rr <= 1.0 && mr <= 1.0) return commit_host(ctx, 0, rr, mr);
  HIPCK(launch_axpbz(ctx->jA, 1.0, ctx->jr[0], 0.0, nullptr, n, s));
  HIPCK(launch_axpbz(ctx->rA, 1.0, ctx->jr[2], -1.0, ctx->jr[0], n, s));
  double err = rr, emr = mr;
  const int mem = c.anderson_m;
  int mh = 0, head = 0;  // history column k (oldest first) lives at index (head + k) % mem
  while (R.outer_iters < c.max_outer) {
    const int k = R.outer_iters;
    bool accepted = false;
    for (int pass = 0; pass < 2 && !accepted; ++pass) {
      const bool use_a = pass == 0 && k >= c.anderson_start && mh > 0;
      if (pass == 0 && !use_a) continue;
      HIPCK(launch_axpbz(ctx->dA, c.beta, ctx->rA, 0.0, nullptr, n, s));
      if (use_a) {
        DotArgs da{};
        da.K = mh + 1;
        da.n = n;
        for (int m = 0; m < mh; ++m) da.v[m] = ctx->hR[(head + m) % mem];
        da.v[mh] = ctx->rA;
        da.partials = ctx->partials;
        const int nb = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 128);
        HIPCK(launch_dots(da, nb, s));
        HIPCK(launch_reduce(ctx->partials, nb, kMaxDots, 1, kMaxDots, 0u, ctx->ddot, s));
        HIPCK(hipMemcpyAsync(ctx->hdot, ctx->ddot, sizeof(double) * kMaxDots, hipMemcpyDeviceToHost, s));
        HIPCK(hipStreamSynchronize(s));
        // unpack the upper triangle (k1 <= k2, row order over kMaxDotVecs vectors)
        auto dot = [&](int k1, int k2) {
          if (k1 > k2) std::swap(k1, k2);
          return ctx->hdot[k1 * kMaxDotVecs - k1 * (k1 - 1) / 2 + (k2 - k1)];
        };
        double G[64], b[8], gam[8];
        double tr = 0.0;
        for (int a1 = 0; a1 < mh; ++a1) {
          b[a1] = dot(a1, mh);
          for (int a2 = 0; a2 < mh; ++a2) G[a1 * mh + a2] = dot(a1, a2);
          tr += G[a1 * mh + a1];
        }
        for (int a1 = 0; a1 < mh; ++a1) G[a1 * mh + a1] += c.anderson_lambda * tr / mh;
        if (!solve_small(G, b, mh, gam)) {
          mh = 0;  // unusable history: damped Picard
          continue;
        }
        for (int m = 0; m < mh; ++m) {
          const int col = (head + m) % mem;
          HIPCK(launch_axpbz(ctx->dA, 1.0, ctx->dA, -gam[m], ctx->hJ[col], n, s));
          HIPCK(launch_axpbz(ctx->dA, 1.0, ctx->dA, -gam[m] * c.beta, ctx->hR[col], n, s));
        }
      }
      double alpha = 1.0;
      for (int hh = 0; hh <= c.ls_halvings && R.outer_iters < c.max_outer; ++hh, alpha *= 0.5) {
        // trial j_t = j + alpha d in slot 1, with its projected spectrum for the field step
        HIPCK(launch_axpbz(ctx->jr[1], 1.0, ctx->jA, alpha, ctx->dA, n, s));
        HIPCK(fft_nd(M, ctx->axes, 3, ctx->jr[1], nullptr, ctx->jh[1], nullptr, nullptr, false,
                     c.project_nyquist != 0, s));
        st = eval_outer(ctx, 1, 2, R, use_graph, rr, mr);
        if (st) return st;
        if (rr <= 1.0 && mr <= 1.0) return commit_host(ctx, 1, rr, mr);
        if (use_a && rr > c.ls_growth * err) mh = 0;
        if (rr <= (1.0 - c.ls_decrease * alpha) * err && mr <= c.ls_growth * emr) {
          int col;
          if (mh < mem) {
            col = (head + mh) % mem;
            ++mh;
          } else {
            col = head;
            head = (head + 1) % mem;
          }
          // history column: dJ = j_t - j, dR = (H_t - j_t) - r; then j = j_t, r = H_t - j_t
          HIPCK(launch_axpbz(ctx->hJ[col], 1.0, ctx->jr[1], -1.0, ctx->jA, n, s));
          HIPCK(launch_axpbz(ctx->hR[col], 1.0, ctx->jr[2], -1.0, ctx->jr[1], n, s));
          HIPCK(launch_axpbz(ctx->hR[col], 1.0, ctx->hR[col], -1.0, ctx->rA, n, s));
          HIPCK(launch_axpbz(ctx->jA, 1.0, ctx->jr[1], 0.0, nullptr, n, s));
          HIPCK(launch_axpbz(ctx->rA, 1.0, ctx->jr[2], -1.0, ctx->jr[1], n, s));
          err = rr;
          emr = mr;
          accepted = true;
          ++R.outer_updates;
          break;
        }
      }
      if (!accepted && use_a) mh = 0;  // rejected Anderson direction: retry as damped Picard
    }
    if (!accepted) return fail(ctx, GMHC_ENOCONV, "no outer direction accepted by the backtracking safeguards");
  }
  return fail(ctx, GMHC_ENOCONV, "outer iteration limit reached");
}

int32_t gmhc_step(gmhc_ctx* ctx, gmhc_step_report* rep) {
  if (!ctx) return GMHC_EINVAL;
  if (!ctx->initialized) return fail(ctx, GMHC_ESTATE, "initialize before step");
  DevGuard gd(ctx->device);
  const Mesh& M = ctx->M;
  const int64_t Ng = M.Ng;
  hipStream_t s = ctx->stream;
  gmhc_step_report R{};
  auto done = [&](int32_t st) {
    if (rep) *rep = R;
    return st;
  };
  ctx->pass_done = false;  // the step reuses the frozen pass's buffers
  if (!ctx->ahead) {  // else the previous step began this one (no sort was due)
    if (ctx->cfg.sort_every > 0 && ctx->step % ctx->cfg.sort_every == 0) {
      int32_t st = sort_particles(ctx);
      if (st) return done(st);
    }
    int32_t st = begin_step(ctx);
    if (st) return done(st);
  }
  bool use_graph = ctx->cfg.graphs != 0 && ctx->stream != nullptr && !ctx->graphs_off;
  if (ctx->cfg.outer_scheme == 1) return done(step_anderson(ctx, R, use_graph));
  // damped Picard: j <- j + beta (H(j) - j); the outer test runs on the device unless
  // the outer iterations are replayed as graphs
  if (!use_graph) return done(run_picard(ctx, R));
  int cur = 0;
  while (R.outer_iters < ctx->cfg.max_outer) {
    const int hs = (cur == 1) ? 2 : 1;
    double rr = 0.0, mr = 0.0;
    int32_t st = eval_outer(ctx, cur, hs, R, use_graph, rr, mr);
    if (st) return done(st);
    if (rr <= 1.0 && mr <= 1.0) return done(commit_host(ctx, cur, rr, mr));
    if (ctx->cfg.beta != 1.0)
      HIPCK(launch_axpy2(ctx->jr[hs], ctx->jr[cur], ctx->jh[hs], ctx->jh[cur], 1.0 - ctx->cfg.beta, 3 * Ng,
                         3 * Ng, s));
    ++R.outer_updates;
    cur = hs;
  }
  return done(fail(ctx, GMHC_ENOCONV, "outer iteration limit reached"));
}

int32_t gmhc_diagnostics(gmhc_ctx* ctx, gmhc_diag* out) {
  if (!ctx || !out) return GMHC_EINVAL;
  if (!ctx->initialized) return fail(ctx, GMHC_ESTATE, "initialize before diagnostics");
  DevGuard gd(ctx->device);
  const Mesh& M = ctx->M;
  const int64_t Ng = M.Ng;
  hipStream_t s = ctx->stream;
  KinArgs ka{};
  ka.M = M;
  ka.np = ctx->np;
  ka.kappa = ctx->cfg.kappa;
  for (int l = 0; l < 3; ++l) {
    ka.x[l] = ctx->x[l];
    ka.P[l] = ctx->P[l];
    ka.A[l] = ctx->An + l * Ng;
  }
  ka.q = ctx->q;
  ka.prec = ctx->prec;
  ka.partials = ctx->partials;
  const int kb = (int)std::min<int64_t>(std::max<int64_t>((ctx->np + kBlock - 1) / kBlock, 1), 1024);
  HIPCK(launch_kinetic(ka, kb, s));
  HIPCK(launch_reduce(ctx->partials, kb, kDiagParts, 1, kDiagParts, 0u, ctx->dres, s));
  SpecDiagArgs sa{};
  sa.M = M;
  sa.kappa2 = ctx->cfg.kappa * ctx->cfg.kappa;
  sa.sigma1 = ctx->cfg.sigma1;
  sa.sigma2 = ctx->cfg.sigma2;
  sa.phi = ctx->S0;
  sa.psi = ctx->S0 + Ng;
  sa.rho = ctx->S0 + 2 * Ng;
  sa.A = ctx->S0 + 3 * Ng;
  sa.U = ctx->S0 + 6 * Ng;
  sa.partials = res_partials(ctx);
  const int sb = res_blocks(ctx);
  HIPCK(launch_spec_diag(sa, sb, s));
  HIPCK(launch_reduce(sa.partials, sb, kDiagParts, 1, kDiagParts, 0u, ctx->dres + kResOff, s));
  HIPCK(hipMemcpyAsync(ctx->hres, ctx->dres, sizeof(double) * 32, hipMemcpyDeviceToHost, s));
  HIPCK(hipStreamSynchronize(s));
  const double* h = ctx->hres;
  const double* sp = ctx->hres + kResOff;
  memset(out, 0, sizeof(*out));
  out->t = ctx->t;
  out->step = ctx->step;
  out->kinetic = h[0];
  out->vperp_rms = h[2] > 0.0 ? sqrt(h[1] / h[2]) : 0.0;
  // Parseval: sum_g |f_g|^2 = (1/Ng) sum_k |f_hat_k|^2
  const double ng = (double)Ng;
  out->field = M.dV / ng * (sp[0] / (2.0 * ctx->cfg.sigma1) + sp[1] / (2.0 * ctx->cfg.sigma2));
  out->total = out->kinetic + out->field;
  out->energy_rel = ctx->E0 != 0.0 ? fabs(out->total - ctx->E0) / fabs(ctx->E0) : 0.0;
  out->gauss_rms = sqrt(sp[2]) / ng;
  out->lorenz_rms = sqrt(sp[3]) / ng;
  out->chain_rms = ctx->last_chain;
  out->work_residual = ctx->last_work;
  out->res_rms_ratio = ctx->last_rr;
  out->res_max_ratio = ctx->last_mr;
  return GMHC_OK;
}

int32_t gmhc_read_particles(gmhc_ctx* ctx, double* x, double* P, double* vbar, int32_t ptr_kind) {
  if (!ctx) return GMHC_EINVAL;
  if (!ctx->loaded) return fail(ctx, GMHC_ESTATE, "no particles loaded");
  DevGuard gd(ctx->device);
  const int64_t np = ctx->np;
  if (!np) return GMHC_OK;
  hipStream_t s = ctx->stream;
  const size_t b = sizeof(double) * (size_t)np;
  auto emit = [&](void* const* src, int prec, int nc, double* dst) -> int32_t {
    HIPCK(launch_unpermute(src, prec, ctx->pscr, nc, ctx->id, np, s));
    for (int c = 0; c < nc; ++c)
      HIPCK(hipMemcpyAsync(dst + c * np, ctx->pscr[c], b, kind_of(ptr_kind, false), s));
    HIPCK(hipStreamSynchronize(s));
    return GMHC_OK;
  };
  int32_t st = GMHC_OK;
  void* const xs[3] = {ctx->x[0], ctx->x[1], ctx->x[2]};
  if (x && (st = emit(xs, GMHC_FP64, ctx->M.d, x))) return st;
  if (P && (st = emit(ctx->P, ctx->prec, 3, P))) return st;
  if (vbar && (st = emit(ctx->vb, ctx->prec, 3, vbar))) return st;
  return GMHC_OK;
}

int32_t gmhc_set_particle_state(gmhc_ctx* ctx, const double* x, const double* P, const double* vbar,
                                int32_t ptr_kind) {
  if (!ctx) return GMHC_EINVAL;
  drop_ahead(ctx);
  if (!ctx->loaded) return fail(ctx, GMHC_ESTATE, "no particles loaded");
  DevGuard gd(ctx->device);
  const int64_t np = ctx->np;
  if (!np) return GMHC_OK;
  hipStream_t s = ctx->stream;
  const size_t b = sizeof(double) * (size_t)np;
  auto take = [&](const double* src, int nc, void* const* dst, int prec) -> int32_t {
    for (int c = 0; c < nc; ++c)
      HIPCK(hipMemcpyAsync(ctx->pscr[c], src + c * np, b, kind_of(ptr_kind, true), s));
    HIPCK(launch_permute_in(ctx->pscr, dst, prec, nc, ctx->id, np, s));
    HIPCK(hipStreamSynchronize(s));
    return GMHC_OK;
  };
  int32_t st = GMHC_OK;
  void* const xs[3] = {ctx->x[0], ctx->x[1], ctx->x[2]};
  if (x && (st = take(x, ctx->M.d, xs, GMHC_FP64))) return st;
  if (P && (st = take(P, 3, ctx->P, ctx->prec))) return st;
  if (vbar && (st = take(vbar, 3, ctx->vb, ctx->prec))) return st;
  return GMHC_OK;
}

int32_t gmhc_read_field(gmhc_ctx* ctx, int32_t which, double* dst, int32_t ptr_kind) {
  if (!ctx || !dst) return GMHC_EINVAL;
  if (!ctx->bound) return fail(ctx, GMHC_ESTATE, "bind before reading fields");
  DevGuard gd(ctx->device);
  int nc = 0;
  int32_t st = field_to_rscr(ctx, which, &nc);
  if (st) return st;
  HIPCK(hipMemcpyAsync(dst, ctx->rscr, sizeof(double) * nc * ctx->M.Ng, kind_of(ptr_kind, false), ctx->stream));
  HIPCK(hipStreamSynchronize(ctx->stream));
  return GMHC_OK;
}

int32_t gmhc_mode_amplitude(gmhc_ctx* ctx, int32_t which, int32_t comp, const int32_t mode[3], double* amp) {
  if (!ctx || !mode || !amp) return GMHC_EINVAL;
  if (!ctx->bound) return fail(ctx, GMHC_ESTATE, "bind before reading modes");
  if (comp < 0 || comp >= ncomp_of(which)) return fail(ctx, GMHC_EINVAL, "bad component");
  DevGuard gd(ctx->device);
  const Mesh& M = ctx->M;
  const int64_t Ng = M.Ng;
  int64_t idx[3];
  for (int l = 0; l < 3; ++l) idx[l] = ((mode[l] % M.n[l]) + M.n[l]) % M.n[l];
  const int64_t g = idx[0] + (int64_t)M.n[0] * (idx[1] + (int64_t)M.n[1] * idx[2]);
  auto fetch = [&](const double2* base, double2* v) -> int32_t {
    HIPCK(hipMemcpy(v, base + g, sizeof(double2), hipMemcpyDeviceToHost));
    return GMHC_OK;
  };
  HIPCK(hipStreamSynchronize(ctx->stream));
  const long double pi = 3.141592653589793238462643383279502884L;
  double k[3];
  for (int l = 0; l < 3; ++l) {
    const int n = M.n[l];
    if (l >= M.d || (n % 2 == 0 && idx[l] == n / 2)) {
      k[l] = 0.0;
    } else {
      const int64_t ms = (idx[l] <= n / 2) ? idx[l] : idx[l] - n;
      k[l] = (double)(2.0L * pi * ms / M.len[l]);
    }
  }
  double2 v{0.0, 0.0};
  int32_t st = GMHC_OK;
  const double2* S = ctx->S0;
  switch (which) {
    case GMHC_PHI: st = fetch(S, &v); break;
    case GMHC_PSI: st = fetch(S + Ng, &v); break;
    case GMHC_RHO: st = fetch(S + 2 * Ng, &v); break;
    case GMHC_A: st = fetch(S + (3 + comp) * Ng, &v); break;
    case GMHC_U: st = fetch(S + (6 + comp) * Ng, &v); break;
    case GMHC_J: st = fetch(ctx->jh[0] + comp * Ng, &v); break;
    case GMHC_E: {
      double2 ph, u;
      if ((st = fetch(S, &ph)) || (st = fetch(S + (6 + comp) * Ng, &u))) break;
      // E = -i k phi - U
      v = make_double2(k[comp] * ph.y - u.x, -k[comp] * ph.x - u.y);
      break;
    }
    case GMHC_B: {
      double2 A[3];
      for (int c = 0; c < 3 && !st; ++c) st = fetch(S + (3 + c) * Ng, &A[c]);
      if (st) break;
      const int a = (comp + 1) % 3, b = (comp + 2) % 3;
      // (i k x A)_comp = i (k_a A_b - k_b A_a)
      const double2 w = make_double2(k[a] * A[b].x - k[b] * A[a].x, k[a] * A[b].y - k[b] * A[a].y);
      v = make_double2(-w.y, w.x);
      break;
    }
    default: return fail(ctx, GMHC_EINVAL, "unknown field selector");
  }
  if (st) return st;
  *amp = hypot(v.x, v.y) / (double)Ng;
  return GMHC_OK;
}

int32_t gmhc_set_frozen_fields(gmhc_ctx* ctx, const double* gradphi, const double* An, const double* Anp1,
                               const double* Uh, int32_t ptr_kind) {
  if (!ctx || !gradphi || !An || !Anp1 || !Uh) return GMHC_EINVAL;
  drop_ahead(ctx);
  if (!ctx->bound) return fail(ctx, GMHC_ESTATE, "bind before setting fields");
  DevGuard gd(ctx->device);
  const int64_t Ng = ctx->M.Ng;
  const int d = ctx->M.d;
  hipStream_t s = ctx->stream;
  HIPCK(hipMemcpyAsync(ctx->trial[0], gradphi, sizeof(double) * d * Ng, kind_of(ptr_kind, true), s));
  HIPCK(hipMemcpyAsync(ctx->An, An, sizeof(double) * 3 * Ng, kind_of(ptr_kind, true), s));
  HIPCK(hipMemcpyAsync(ctx->trial[0] + d * Ng, Anp1, sizeof(double) * 3 * Ng, kind_of(ptr_kind, true), s));
  HIPCK(hipMemcpyAsync(ctx->trial[0] + (d + 3) * Ng, Uh, sizeof(double) * 3 * Ng, kind_of(ptr_kind, true), s));
  HIPCK(hipStreamSynchronize(s));
  ctx->frozen = true;
  ctx->initialized = false;  // A^n of the stepping state was replaced
  return GMHC_OK;
}

int32_t gmhc_orbit_pass_frozen(gmhc_ctx* ctx, int32_t iterate, gmhc_pass_report* rep) {
  if (!ctx) return GMHC_EINVAL;
  drop_ahead(ctx);
  if (!ctx->loaded || !ctx->frozen) return fail(ctx, GMHC_ESTATE, "load particles and set frozen fields first");
  DevGuard gd(ctx->device);
  const int64_t np = ctx->np;
  hipStream_t s = ctx->stream;
  for (int l = 0; l < 3; ++l)
    if (np) HIPCK(hipMemcpyAsync(ctx->vw[l], ctx->vb[l], ctx->es * np, hipMemcpyDeviceToDevice, s));
  ctx->vin_first = false;
  ctx->timed_now = ctx->cfg.timing != 0;
  int32_t st = run_orbit(ctx, iterate ? 1 : 0, nullptr);
  if (st) return st;
  double oms = 0.0;
  st = fetch_results(ctx, &oms);
  if (st) return st;
  gmhc_pass_report R{};
  const double* h = ctx->hres;
  R.failed = (int64_t)llround(h[OP_FAIL]);
  R.over_limit = (int32_t)llround(h[OP_XLIM]);
  R.inner_max = (int32_t)llround(h[OP_ITMAX]);
  R.evaluations = (int64_t)llround(h[OP_ITERS]);
  R.segments = (int64_t)llround(h[OP_SEGS]);
  R.inner_mean = np ? h[OP_ITERS] / (double)np : 0.0;
  R.refined = (int64_t)llround(h[OP_REFINED]);
  R.orbit_ms = oms;
  ctx->last_pass = R;
  ctx->pass_done = true;
  if (rep) *rep = R;
  return GMHC_OK;
}

int32_t gmhc_read_pass(gmhc_ctx* ctx, double* vout, double* Pnp1, double* J, int32_t* iters, int32_t* levels,
                       int32_t ptr_kind) {
  if (!ctx) return GMHC_EINVAL;
  drop_ahead(ctx);
  if (!ctx->pass_done) return fail(ctx, GMHC_ESTATE, "no frozen pass has run");
  DevGuard gd(ctx->device);
  const int64_t np = ctx->np, Ng = ctx->M.Ng;
  hipStream_t s = ctx->stream;
  const size_t b = sizeof(double) * (size_t)np;
  if (vout && np) {
    HIPCK(launch_unpermute(ctx->vw, ctx->prec, ctx->pscr, 3, ctx->id, np, s));
    for (int c = 0; c < 3; ++c) HIPCK(hipMemcpyAsync(vout + c * np, ctx->pscr[c], b, kind_of(ptr_kind, false), s));
    HIPCK(hipStreamSynchronize(s));
  }
  if (Pnp1 && np) {
    HIPCK(launch_unpermute(ctx->P2, ctx->prec, ctx->pscr, 3, ctx->id, np, s));
    for (int c = 0; c < 3; ++c) HIPCK(hipMemcpyAsync(Pnp1 + c * np, ctx->pscr[c], b, kind_of(ptr_kind, false), s));
    HIPCK(hipStreamSynchronize(s));
  }
  if (iters && np) {
    int32_t* tmp = reinterpret_cast<int32_t*>(ctx->pscr[0]);
    HIPCK(launch_unpermute_i32(ctx->iters, tmp, ctx->id, np, s));
    HIPCK(hipMemcpyAsync(iters, tmp, sizeof(int32_t) * np, kind_of(ptr_kind, false), s));
    HIPCK(hipStreamSynchronize(s));
  }
  if (levels && np) {
    int32_t* tmp = reinterpret_cast<int32_t*>(ctx->pscr[0]);
    if (ctx->pass_levels)
      HIPCK(launch_unpermute_i32(ctx->rstate, tmp, ctx->id, np, s));
    else
      HIPCK(hipMemsetAsync(tmp, 0, sizeof(int32_t) * np, s));
    HIPCK(hipMemcpyAsync(levels, tmp, sizeof(int32_t) * np, kind_of(ptr_kind, false), s));
    HIPCK(hipStreamSynchronize(s));
  }
  if (J) {
    HIPCK(launch_fix_to_double(ctx->Jdep, ctx->rscr, 3 * Ng, ctx->M.fx, s));
    HIPCK(hipMemcpyAsync(J, ctx->rscr, sizeof(double) * 3 * Ng, kind_of(ptr_kind, false), s));
  }
  HIPCK(hipStreamSynchronize(s));
  return GMHC_OK;
}

}  // extern "C"

// ---- adjoint of the step and of initialization (adjoint.hip) ----------------------

namespace {

// Device scratch of the adjoint calls, carved from the caller's buffer.
struct AdjScratch {
  double2* jh;
  double2* S1;
  double* trial;
  double2* work;
  double2* Lf;
  unsigned long long* acc;
  double* Pr;
  double2* Pb;
  double2* Lout;
  double* Lreal;
  double* mu;
  double* partials;
  double* red;
  double* cache;
};

size_t adj_carve(const gmhc_ctx* c, char* base, AdjScratch& a) {
  Carver cv{base};
  const int64_t Ng = c->M.Ng;
  const int d = c->M.d;
  a.jh = cv.take<double2>(3 * Ng);
  a.S1 = cv.take<double2>(9 * Ng);
  a.trial = cv.take<double>((size_t)(d + 6) * Ng);
  a.work = cv.take<double2>(12 * Ng);
  a.Lf = cv.take<double2>(9 * Ng);
  const int nv = adj_nvals(d);
  a.acc = cv.take<unsigned long long>((size_t)2 * nv * Ng);
  a.Pr = cv.take<double>((size_t)nv * Ng);
  a.Pb = cv.take<double2>((size_t)nv * Ng);
  a.Lout = cv.take<double2>(12 * Ng);
  a.Lreal = cv.take<double>(12 * Ng);
  a.mu = cv.take<double>(3 * Ng);
  a.partials = cv.take<double>((size_t)adj_particle_blocks(std::max<int64_t>(c->np, 1)));
  a.red = cv.take<double>(8);
  a.cache = cv.take<double>((size_t)adj_ncache(d) * std::max<int64_t>(c->np, 1));
  return (cv.off + 255) & ~(size_t)255;
}

// The configurations the adjoint covers: quadratic shape, FP64, no refinement, a
// Gauss-Legendre order that integrates the derivative integrands exactly (>= dim + 1).
int32_t adj_supported(gmhc_ctx* ctx) {
  if (ctx->M.shape != 2 || ctx->prec != GMHC_FP64 || ctx->cfg.refine_levels != 0 ||
      ctx->ngl < ctx->M.d + 1)
    return fail(ctx, GMHC_EINVAL,
                "the adjoint covers shape_order 2, precision FP64, refine_levels 0 and gl_order 0 or >= dim + 1");
  return GMHC_OK;
}

int32_t adj_prepare(gmhc_ctx* ctx, void* scratch, size_t bytes, AdjScratch& a) {
  if (!ctx->initialized) return fail(ctx, GMHC_ESTATE, "initialize (or load a state) before the adjoint");
  int32_t st = adj_supported(ctx);
  if (st) return st;
  if (!scratch) return fail(ctx, GMHC_EINVAL, "null adjoint scratch");
  if (reinterpret_cast<uintptr_t>(scratch) & 255) return fail(ctx, GMHC_EINVAL, "adjoint scratch not 256-byte aligned");
  if (bytes < adj_carve(ctx, nullptr, a)) return fail(ctx, GMHC_ENOMEM, "adjoint scratch smaller than gmhc_adjoint_bytes");
  adj_carve(ctx, static_cast<char*>(scratch), a);
  drop_ahead(ctx);
  return GMHC_OK;
}

AdjArgs adj_args(const gmhc_ctx* c, const AdjScratch& a, const double* vbar, const double* lx, const double* lP) {
  AdjArgs r{};
  r.M = c->M;
  r.np = c->np;
  r.dt = c->cfg.dt;
  r.kappa = c->cfg.kappa;
  r.ngl = c->ngl;
  for (int k = 0; k < kMaxGL; ++k) {
    r.glx[k] = c->glx[k];
    r.glw[k] = c->glw[k];
  }
  r.ps = std::max<int64_t>(c->np, 1);
  r.x = c->x[0];
  r.P = static_cast<const double*>(c->P[0]);
  r.q = static_cast<const double*>(c->q);
  r.id = c->id;
  r.vbar = vbar;
  r.lx = lx;
  r.lP = lP;
  r.gphi = a.trial;
  r.An = c->An;
  r.Anp1 = a.trial + (int64_t)c->M.d * c->M.Ng;
  r.partials = a.partials;
  r.acc = a.acc;
  r.cache = a.cache;
  return r;
}

}  // namespace

extern "C" {

int32_t gmhc_adjoint_bytes(const gmhc_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return GMHC_EINVAL;
  AdjScratch a{};
  *bytes = adj_carve(ctx, nullptr, a);
  return GMHC_OK;
}

int32_t gmhc_energy_grad(gmhc_ctx* ctx, double* gf, int32_t ptr_kind) {
  if (!ctx || !gf) return GMHC_EINVAL;
  if (!ctx->initialized) return fail(ctx, GMHC_ESTATE, "initialize (or load a state) before gmhc_energy_grad");
  drop_ahead(ctx);
  DevGuard gd(ctx->device);
  const Mesh& M = ctx->M;
  hipStream_t s = ctx->stream;
  HIPCK(launch_energy_grad(M, ctx->cfg.sigma1, ctx->cfg.sigma2, ctx->S0, ctx->cscr, s));
  HIPCK(fft_nd(M, ctx->axes, 9, nullptr, ctx->cscr, nullptr, ctx->rscr, ctx->cout, true, false, s));
  HIPCK(hipMemcpyAsync(gf, ctx->rscr, sizeof(double) * 9 * M.Ng, kind_of(ptr_kind, false), s));
  HIPCK(hipStreamSynchronize(s));
  return GMHC_OK;
}

int32_t gmhc_adjoint_step(gmhc_ctx* ctx, void* scratch, size_t scratch_bytes, const double* j, const double* vbar,
                          const double* lx, const double* lP, const double* lf, double* gx, double* gP, double* gq,
                          double* gf, gmhc_adjoint_report* rep) {
  if (!ctx || !j || !vbar || !lx || !lP || !lf || !gx || !gP || !gq || !gf) return GMHC_EINVAL;
  AdjScratch a{};
  int32_t st = adj_prepare(ctx, scratch, scratch_bytes, a);
  if (st) return st;
  DevGuard gd(ctx->device);
  const Mesh& M = ctx->M;
  const int64_t Ng = M.Ng;
  hipStream_t s = ctx->stream;
  const bool proj = ctx->cfg.project_nyquist != 0;
  // trial fields of the converged current: projected spectrum, CN solve, real fields
  HIPCK(fft_nd(M, ctx->axes, 3, j, nullptr, a.jh, nullptr, nullptr, false, proj, s));
  HIPCK(field_trial(M, ctx->axes, cn_args(ctx, a.jh, a.S1, nullptr), a.trial, a.work, nullptr, s));
  HIPCK(fft_nd(M, ctx->axes, 9, lf, nullptr, a.Lf, nullptr, nullptr, false, false, s));
  HIPCK(launch_zero(a.mu, 3 * Ng, s));
  AdjFieldArgs fa{};
  fa.M = M;
  fa.dt = ctx->cfg.dt;
  fa.kappa2 = ctx->cfg.kappa * ctx->cfg.kappa;
  fa.sigma1 = ctx->cfg.sigma1;
  fa.sigma2 = ctx->cfg.sigma2;
  fa.project = proj ? 1 : 0;
  fa.Lf = a.Lf;
  fa.Pb = a.Pb;
  fa.Ls = a.Lout;
  fa.Lj = a.Lout + 9 * Ng;
  const double tol = std::max(ctx->cfg.tol_outer_rel, 1e-15);
  const int64_t nb = adj_particle_blocks(ctx->np);
  gmhc_adjoint_report R{};
  double hr[2] = {0.0, 0.0};
  bool done = false;
  {  // the values of the step that do not depend on the adjoint current
    AdjArgs pa = adj_args(ctx, a, vbar, lx, lP);
    pa.mode = ADJ_PREP;
    HIPCK(launch_adj_particle(pa, s));
  }
  for (int it = 0; it < ctx->cfg.max_outer && !done; ++it) {
    AdjArgs pa = adj_args(ctx, a, vbar, lx, lP);
    pa.mu = it ? a.mu : nullptr;
    // scale of the exact fixed-point sums from a bound on every scattered value, computed
    // on the device (red[4..6]), so no host round trip sits between the two passes
    pa.mode = ADJ_BOUND;
    HIPCK(launch_adj_iter(pa, s));
    HIPCK(launch_adj_sum(a.partials, ctx->np ? nb : 0, a.red, s));
    HIPCK(launch_adj_scale(a.red, a.red + 4, s));
    HIPCK(launch_zero(reinterpret_cast<double*>(a.acc), 2 * adj_nvals(M.d) * Ng, s));
    pa.mode = ADJ_SCATTER;
    pa.fx = a.red + 4;
    HIPCK(launch_adj_iter(pa, s));
    HIPCK(launch_adj_fix_to_double(a.acc, a.Pr, adj_nvals(M.d) * Ng, a.red + 4, s));
    HIPCK(fft_nd(M, ctx->axes, adj_nvals(M.d), a.Pr, nullptr, a.Pb, nullptr, nullptr, false, false, s));
    HIPCK(launch_adj_field(fa, s));
    HIPCK(fft_nd(M, ctx->axes, 12, nullptr, a.Lout, nullptr, a.Lreal, a.work, true, false, s));
    HIPCK(launch_adj_update(a.mu, a.Lreal + 9 * Ng, 3 * Ng, it ? ctx->cfg.beta : 1.0, a.red, s));
    HIPCK(hipMemcpyAsync(hr, a.red, sizeof(hr), hipMemcpyDeviceToHost, s));
    HIPCK(hipStreamSynchronize(s));
    R.iterations = it + 1;
    R.change_ratio = hr[1] > 0.0 ? hr[0] / hr[1] : 0.0;
    done = hr[0] <= tol * hr[1];
  }
  if (rep) *rep = R;
  if (!done) return fail(ctx, GMHC_ENOCONV, "adjoint current did not settle within max_outer iterations");
  AdjArgs pa = adj_args(ctx, a, vbar, lx, lP);
  pa.mu = a.mu;
  pa.mode = ADJ_FINAL;
  pa.gx = gx;
  pa.gP = gP;
  pa.gq = gq;
  HIPCK(launch_adj_particle(pa, s));
  HIPCK(hipMemcpyAsync(gf, a.Lreal, sizeof(double) * 9 * Ng, hipMemcpyDeviceToDevice, s));
  HIPCK(hipStreamSynchronize(s));
  return GMHC_OK;
}

int32_t gmhc_adjoint_initialize(gmhc_ctx* ctx, void* scratch, size_t scratch_bytes, const double* lx,
                                const double* lP, const double* lf, double* gx, double* gu, double* gq) {
  if (!ctx || !lx || !lP || !lf || !gx || !gu || !gq) return GMHC_EINVAL;
  AdjScratch a{};
  int32_t st = adj_prepare(ctx, scratch, scratch_bytes, a);
  if (st) return st;
  if (ctx->step != 0) return fail(ctx, GMHC_ESTATE, "gmhc_adjoint_initialize needs the initial state (step 0)");
  DevGuard gd(ctx->device);
  const Mesh& M = ctx->M;
  hipStream_t s = ctx->stream;
  HIPCK(fft_nd(M, ctx->axes, 9, lf, nullptr, a.Lf, nullptr, nullptr, false, false, s));
  HIPCK(launch_adj_init_field(M, ctx->cfg.sigma1, ctx->cfg.project_nyquist, a.Lf, a.Lout, s));
  HIPCK(fft_nd(M, ctx->axes, 1, nullptr, a.Lout, nullptr, a.Lreal, a.work, true, false, s));
  AdjInitArgs ia{};
  ia.M = M;
  ia.np = ctx->np;
  ia.ps = std::max<int64_t>(ctx->np, 1);
  ia.kappa = ctx->cfg.kappa;
  ia.x = ctx->x[0];
  ia.P = static_cast<const double*>(ctx->P[0]);
  ia.q = static_cast<const double*>(ctx->q);
  ia.id = ctx->id;
  ia.A0 = ctx->An;
  ia.rb = a.Lreal;
  ia.lx = lx;
  ia.lP = lP;
  ia.gx = gx;
  ia.gu = gu;
  ia.gq = gq;
  HIPCK(launch_adj_init_particle(ia, s));
  HIPCK(hipStreamSynchronize(s));
  return GMHC_OK;
}

int32_t gmhc_state_bytes(const gmhc_ctx* cctx, size_t* bytes) {
  gmhc_ctx* ctx = const_cast<gmhc_ctx*>(cctx);
  if (!ctx || !bytes) return GMHC_EINVAL;
  if (!ctx->bound) return fail(ctx, GMHC_ESTATE, "bind before asking for the state size");
  *bytes = state_bytes(ctx);
  return GMHC_OK;
}

int32_t gmhc_save(gmhc_ctx* ctx, void* dst, size_t bytes, int32_t ptr_kind) {
  if (!ctx || !dst) return GMHC_EINVAL;
  if (!ctx->initialized) return fail(ctx, GMHC_ESTATE, "initialize (or load a state) before saving");
  if (bytes < state_bytes(ctx)) return fail(ctx, GMHC_EINVAL, "destination smaller than gmhc_state_bytes");
  DevGuard gd(ctx->device);
  hipStream_t s = ctx->stream;
  StateHeader h{};
  memcpy(h.magic, kStateMagic, sizeof(h.magic));
  h.abi = GMHC_ABI_VERSION;
  h.dim = ctx->M.d;
  for (int l = 0; l < 3; ++l) h.n[l] = ctx->M.n[l];
  h.precision = ctx->prec;
  h.shape = ctx->M.shape;
  h.have_pot = ctx->have_pot ? 1 : 0;
  h.last_outer = ctx->last_outer;
  h.np = ctx->np;
  h.ng = ctx->M.Ng;
  h.step = ctx->step;
  h.bytes = (int64_t)state_bytes(ctx);
  h.t = ctx->t;
  h.E0 = ctx->E0;
  h.last_chain = ctx->last_chain;
  h.last_work = ctx->last_work;
  h.last_rr = ctx->last_rr;
  h.last_mr = ctx->last_mr;
  h.fx[0] = ctx->M.fx.up;
  h.fx[1] = ctx->M.fx.hi;
  h.fx[2] = ctx->M.fx.lo;
  char* out = static_cast<char*>(dst);
  const hipMemcpyKind to = kind_of(ptr_kind, false);
  HIPCK(hipMemcpyAsync(out, &h, sizeof(h), ptr_kind == GMHC_DEVICE ? hipMemcpyHostToDevice : hipMemcpyHostToHost, s));
  size_t off = (sizeof(StateHeader) + 7) & ~(size_t)7;
  for (const auto& sc : state_sections(ctx)) {
    if (sc.bytes) HIPCK(hipMemcpyAsync(out + off, sc.dev, sc.bytes, to, s));
    off += (sc.bytes + 7) & ~(size_t)7;
  }
  HIPCK(hipStreamSynchronize(s));  // also keeps h alive until its copy is done
  return GMHC_OK;
}

int32_t gmhc_load(gmhc_ctx* ctx, const void* src, size_t bytes, int32_t ptr_kind) {
  if (!ctx || !src) return GMHC_EINVAL;
  drop_ahead(ctx);
  if (!ctx->bound) return fail(ctx, GMHC_ESTATE, "bind before loading a state");
  DevGuard gd(ctx->device);
  hipStream_t s = ctx->stream;
  const char* in = static_cast<const char*>(src);
  StateHeader h{};
  if (bytes < sizeof(h)) return fail(ctx, GMHC_EINVAL, "state image too small");
  HIPCK(hipMemcpy(&h, in, sizeof(h), ptr_kind == GMHC_DEVICE ? hipMemcpyDeviceToHost : hipMemcpyHostToHost));
  bool same = memcmp(h.magic, kStateMagic, sizeof(h.magic)) == 0 && h.abi == GMHC_ABI_VERSION &&
              h.dim == ctx->M.d && h.precision == ctx->prec && h.shape == ctx->M.shape && h.np == ctx->np &&
              h.ng == ctx->M.Ng && h.bytes == (int64_t)state_bytes(ctx) && bytes >= (size_t)h.bytes;
  for (int l = 0; l < 3; ++l) same = same && h.n[l] == ctx->M.n[l];
  if (!same)
    return fail(ctx, GMHC_EINVAL,
                "state image does not match this context (mesh, particle count, precision, shape or ABI)");
  const hipMemcpyKind from = kind_of(ptr_kind, true);
  size_t off = (sizeof(StateHeader) + 7) & ~(size_t)7;
  for (const auto& sc : state_sections(ctx)) {
    if (sc.bytes) HIPCK(hipMemcpyAsync(sc.dev, in + off, sc.bytes, from, s));
    off += (sc.bytes + 7) & ~(size_t)7;
  }
  HIPCK(hipStreamSynchronize(s));
  ctx->M.fx = FixScale{h.fx[0], h.fx[1], h.fx[2]};
  ctx->have_pot = h.have_pot != 0;
  ctx->last_outer = h.last_outer;
  ctx->t = h.t;
  ctx->step = h.step;
  ctx->E0 = h.E0;
  ctx->last_chain = h.last_chain;
  ctx->last_work = h.last_work;
  ctx->last_rr = h.last_rr;
  ctx->last_mr = h.last_mr;
  ctx->loaded = true;
  ctx->initialized = true;
  ctx->frozen = false;
  ctx->pass_done = false;
  ctx->ctl_clean = false;
  return GMHC_OK;
}

}  // extern "C"
