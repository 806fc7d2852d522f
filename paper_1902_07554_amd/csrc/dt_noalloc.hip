// dt_triangulate_noalloc (include/dt.h): the direct triangulation of
// dt_triangulate (k = 1) for callers that cannot allocate device memory.
// Every scratch buffer of the call is carved from one static device array
// per GPU; inputs and outputs are the caller's.
#include <string.h>

#include <mutex>

#include "dt_common.hpp"
#include "dt_internal.hpp"
#include "dt_pipeline.hpp"
#include "dt_prep.hpp"
#include "dt_prims.hpp"
#include "dt_stages.hpp"

// The scratch array.  In host code its name is only a stand-in for the
// device symbol: its device address comes from hipGetSymbolAddress, once
// per device, and only that address is ever passed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[DT_NOALLOC_SCRATCH_BYTES];

namespace dtk {
namespace {

constexpr int MAX_DEV = 64;
std::mutex g_dev_mu[MAX_DEV];       // one call at a time per device
std::mutex g_addr_mu;
void* g_addr[MAX_DEV] = {};

// Device address of the scratch array on the current device `dev`.
int scratch_address(int dev, void** out) {
  std::lock_guard<std::mutex> g(g_addr_mu);
  if (!g_addr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return DT_E_DEVICE;
    g_addr[dev] = p;
  }
  *out = g_addr[dev];
  return DT_OK;
}

int run_direct(const double* points, uint32_t n, int D, const dt_options& o, int32_t* rows,
               int64_t cap_rows, int64_t* count, hipStream_t st) {
  Ctx cx;
  DT_TRY(cx.init());
  DevBuf setoff, pset, pts, scratch_prep;
  DT_TRY(setoff.alloc(8));
  const uint32_t off[2] = {0, n};
  DT_HIP(hipMemcpyAsync(setoff.p, off, 8, hipMemcpyHostToDevice, st));
  DT_TRY(pset.alloc((size_t)n * 4));
  DT_HIP(hipMemsetAsync(pset.p, 0, (size_t)n * 4, st));
  DT_TRY(pts.alloc((size_t)n * sizeof(double4)));
  DT_TRY(prep_points(points, nullptr, nullptr, n, D, pts.as<double4>(), scratch_prep,
                     cx.dflag.as<uint32_t>(), cx.hflag, st));
  scratch_prep.release();
  double lo[3], hi[3];
  DT_TRY(bbox(pts.as<double4>(), n, lo, hi, st));
  DT_TRY(spatial_sort(pts, n, D, lo, hi, nullptr, 0, st));
  LocalJob job;
  job.D = D;
  job.npts = n;
  job.nsets = 1;
  job.pts = pts.as<double4>();
  job.pset = pset.as<uint32_t>();
  job.set_off = setoff.as<uint32_t>();
  job.fp32 = o.precision == DT_PREC_FP32;
  job.tune(o);
  CellPool pool;
  K4Stats ks;
  DT_TRY(k4_run(job, pool, cx.dc(), cx.hctr, st, ks));
  DT_TRY(k4_extract(job, pool, nullptr, cx.dflag.as<uint32_t>(), nullptr, st));
  DT_HIP(hipMemcpyAsync(cx.hflag, cx.dflag.p, 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  const int64_t m = *cx.hflag;
  *count = m;
  if (m == 0) return DT_E_DEGENERATE;
  if (m > cap_rows) return DT_E_INVALID_ARG;
  DT_TRY(k4_extract(job, pool, rows, cx.dflag.as<uint32_t>(), nullptr, st));
  return DT_OK;
}

}  // namespace
}  // namespace dtk

using namespace dtk;

extern "C" int dt_triangulate_noalloc(const double* points, int64_t n, int D,
                                      const dt_options* opt, int32_t* rows, int64_t cap_rows,
                                      int64_t* count, void* stream) {
  if (!count) return DT_E_INVALID_ARG;
  *count = 0;
  if ((D != 2 && D != 3) || n < 0 || !points || cap_rows < 0 || (cap_rows > 0 && !rows))
    return DT_E_INVALID_ARG;
  dt_options o;
  DT_TRY(check_options(opt, o));
  if (o.sort_output) return DT_E_INVALID_ARG;
  if (n > (D == 2 ? DT_NOALLOC_MAX_POINTS_2D : DT_NOALLOC_MAX_POINTS_3D)) return DT_E_NOMEM;
  if (n < D + 1) return DT_E_DEGENERATE;
  int dev = 0;
  DT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEV) return DT_E_DEVICE;
  std::lock_guard<std::mutex> g(g_dev_mu[dev]);
  void* base = nullptr;
  DT_TRY(scratch_address(dev, &base));
  hipStream_t st = (hipStream_t)stream;
  Workspace ws;
  ws.base = static_cast<char*>(base);
  ws.cap = DT_NOALLOC_SCRATCH_BYTES;
  int s;
  {
    WorkspaceScope scope(&ws);
    s = run_direct(points, (uint32_t)n, D, o, rows, cap_rows, count, st);
  }
  // the scratch is reused by the next call: leave no work in flight on it
  if (hipStreamSynchronize(st) != hipSuccess && s == DT_OK) s = DT_E_DEVICE;
  return s;
}
