// static_pass.hip -- gmhc_orbit_pass_static: the orbit pass of gmhc_orbit_pass_frozen on
// caller-owned device arrays, for callers that cannot allocate device memory.  Its scratch
// (per-workgroup partial sums, their chunk sums, the reduced pass results and the
// fixed-point current accumulator) is a file-scope device array of fixed size, one copy
// per GPU; the kernels are those of the stepping path.
#include <math.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "gmhc.h"
#include "gmhc_internal.h"

using namespace gmhc;

namespace {

// Its scratch lives in the file-scope device array `scratch`: the per-workgroup partial
// sums of the pass, their first-level chunk sums, the reduced pass results and the
// fixed-point current accumulator, at these byte offsets.
constexpr int64_t kStaticBlocks = GMHC_STATIC_MAX_PARTICLES / kOrbitBlock;
constexpr size_t kStPartials = 0;  // [kOrbitParts][kStaticBlocks] double
constexpr size_t kStChunks = kStPartials + sizeof(double) * kOrbitParts * kStaticBlocks;  // [kOrbitParts][1024]
constexpr size_t kStRes = kStChunks + sizeof(double) * kOrbitParts * kReduceChunks;       // [64] double
constexpr size_t kStJ = kStRes + sizeof(double) * 64;  // [3][Ng] fixed-point pairs
constexpr size_t kStEnd = kStJ + sizeof(unsigned long long) * 6 * (size_t)GMHC_STATIC_MAX_NODES;
static_assert(kStEnd == GMHC_STATIC_SCRATCH_BYTES, "static scratch layout");
static_assert(kStChunks % 256 == 0 && kStRes % 256 == 0 && kStJ % 256 == 0, "256-byte aligned parts");

std::mutex g_static_mu;
void* g_static_ptr[64] = {};       // device address of `scratch`, per device
thread_local std::string g_static_err;  // gmhc_last_error(NULL)

int32_t static_fail(int32_t st, const std::string& msg) {
  g_static_err = msg;
  return st;
}

}  // namespace

// One copy per GPU, held until the process ends.  Host code never uses this name as an
// address: it takes the device address from hipGetSymbolAddress (static_scratch).
static __device__ __align__(256) char scratch[GMHC_STATIC_SCRATCH_BYTES];

namespace {

// Device address of this device's `scratch`, looked up once per device with the device
// current.
int32_t static_scratch(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return static_fail(GMHC_EDEVICE, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= 64) return static_fail(GMHC_EDEVICE, "device index beyond 63");
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return static_fail(GMHC_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_static_ptr[dev] = p;
  }
  *out = static_cast<char*>(g_static_ptr[dev]);
  return GMHC_OK;
}

}  // namespace

namespace gmhc {
const char* static_last_error() { return g_static_err.c_str(); }
}  // namespace gmhc

extern "C" {

int32_t gmhc_orbit_pass_static(const gmhc_config* cfg, int64_t n, const double* x, const double* P,
                               const double* q, const double* vin, const double* gradphi, const double* An,
                               const double* Anp1, const double* Uh, int32_t iterate, double* vout, double* Pnp1,
                               double* xnp1, double* J, void* hip_stream, gmhc_pass_report* rep) {
  g_static_err.clear();
  if (!cfg || !config_ok(*cfg)) return static_fail(GMHC_EINVAL, "invalid configuration (see gmhc_create)");
  if (cfg->precision != GMHC_FP64) return static_fail(GMHC_EINVAL, "the static orbit pass runs in FP64 only");
  if (cfg->refine_levels != 0)
    return static_fail(GMHC_EINVAL, "the static orbit pass has no particle refinement (refine_levels must be 0)");
  if (n < 0 || n > GMHC_STATIC_MAX_PARTICLES)
    return static_fail(GMHC_EINVAL, "particle count " + std::to_string((long long)n) +
                                        " outside 0..GMHC_STATIC_MAX_PARTICLES (" +
                                        std::to_string((long long)GMHC_STATIC_MAX_PARTICLES) + ")");
  Mesh M;
  int ngl = 0;
  double glx[kMaxGL], glw[kMaxGL];
  set_geometry(*cfg, M, ngl, glx, glw);
  if (M.Ng > GMHC_STATIC_MAX_NODES)
    return static_fail(GMHC_EINVAL, "mesh of " + std::to_string((long long)M.Ng) +
                                        " nodes exceeds GMHC_STATIC_MAX_NODES (" +
                                        std::to_string((long long)GMHC_STATIC_MAX_NODES) + ")");
  if (!gradphi || !An || !Anp1 || !Uh || !J) return static_fail(GMHC_EINVAL, "null field or current array");
  if (n > 0 && (!x || !P || !q || !vin || !vout || !Pnp1 || !xnp1))
    return static_fail(GMHC_EINVAL, "null particle array");
  char* sp = nullptr;
  int32_t st = static_scratch(&sp);
  if (st) return st;
  double* partials = reinterpret_cast<double*>(sp + kStPartials);
  double* pchunk = reinterpret_cast<double*>(sp + kStChunks);
  double* dres = reinterpret_cast<double*>(sp + kStRes);
  unsigned long long* Jfx = reinterpret_cast<unsigned long long*>(sp + kStJ);
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  auto ck = [](hipError_t e, const char* what) -> int32_t {
    if (e == hipSuccess) return GMHC_OK;
    return static_fail(GMHC_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  };
  // fixed-point scale of the current from sum |q| (as gmhc_load_particles sets it)
  double qsum = 0.0;
  if (n > 0) {
    const int kb = (int)std::min<int64_t>((n + kBlock - 1) / kBlock, 1024);
    if ((st = ck(launch_abs_charge(q, GMHC_FP64, n, partials, kb, s), "abs charge"))) return st;
    if ((st = ck(launch_reduce(partials, kb, kDiagParts, 1, 1, 0u, dres, s), "reduce"))) return st;
    if ((st = ck(hipMemcpyAsync(&qsum, dres, sizeof(double), hipMemcpyDeviceToHost, s), "copy"))) return st;
    if ((st = ck(hipStreamSynchronize(s), "synchronize"))) return st;
    if (!isfinite(qsum)) return static_fail(GMHC_EINVAL, "non-finite particle charges");
  }
  M.fx = fix_scale(std::max(cfg->kappa, 1.0) * qsum / M.dV);
  if ((st = ck(launch_zero(reinterpret_cast<double*>(Jfx), 6 * M.Ng, s), "zero"))) return st;
  OrbitArgs a{};
  a.M = M;
  a.np = n;
  a.dt = cfg->dt;
  a.kappa = cfg->kappa;
  a.tol_abs = cfg->tol_inner_abs;
  a.tol_rel = cfg->tol_inner_rel;
  a.max_inner = cfg->max_inner;
  a.iterate = iterate ? 1 : 0;
  a.deposit = 1;
  a.ngl = ngl;
  for (int k = 0; k < kMaxGL; ++k) {
    a.glx[k] = glx[k];
    a.glw[k] = glw[k];
  }
  a.ps = std::max<int64_t>(n, 1);
  a.precision = GMHC_FP64;
  a.x = x;
  a.xn = xnp1;
  a.P = P;
  a.Pn = Pnp1;
  a.q = q;
  a.vin = vin;
  a.v = vout;
  a.iters = nullptr;
  a.gphi = gradphi;
  a.An = An;
  a.Anp1 = Anp1;
  a.Uh = Uh;
  a.J = Jfx;
  a.partials = partials;
  a.pstride = kStaticBlocks;
  if ((st = ck(launch_orbit(a, ngl, s), "orbit pass"))) return st;
  const int nb = (int)((n + kOrbitBlock - 1) / kOrbitBlock);
  if (nb > 0) {
    const ReduceSet r =
        reduce_chunks(ReduceSet{partials, nb, 1, kStaticBlocks, kOrbitParts, 1u << OP_ITMAX, dres}, pchunk, s);
    if ((st = ck(launch_reduce(r.p, r.nblocks, r.bstride, r.vstride, r.nvals, r.max_mask, r.out, s), "reduce")))
      return st;
  } else if ((st = ck(launch_zero(dres, kOrbitParts, s), "zero"))) {
    return st;
  }
  if ((st = ck(launch_fix_to_double(Jfx, J, 3 * M.Ng, M.fx, s), "current"))) return st;
  if (rep) {
    double h[kOrbitParts];
    if ((st = ck(hipMemcpyAsync(h, dres, sizeof(h), hipMemcpyDeviceToHost, s), "copy"))) return st;
    if ((st = ck(hipStreamSynchronize(s), "synchronize"))) return st;
    gmhc_pass_report R{};
    R.failed = (int64_t)llround(h[OP_FAIL]);
    R.over_limit = (int32_t)llround(h[OP_XLIM]);
    R.inner_max = (int32_t)llround(h[OP_ITMAX]);
    R.evaluations = (int64_t)llround(h[OP_ITERS]);
    R.segments = (int64_t)llround(h[OP_SEGS]);
    R.inner_mean = n ? h[OP_ITERS] / (double)n : 0.0;
    *rep = R;
  }
  return GMHC_OK;
}

}  // extern "C"
