// Batch evaluation of the library's geometric predicates (dt_predicates in
// include/dt.h): the same filter chain (FP32 -> FP64 -> exact, or FP64 ->
// exact) that decides every orientation and in-sphere test of the
// triangulation, applied to caller-given point tuples.
#include "dt_common.hpp"
#include "dt_internal.hpp"
#include "dt_pred.hpp"

namespace dtk {

// One thread per tuple.  stage: 0 decided by the FP32 filter, 1 by the
// FP64 filter, 2 by the exact stage.
template <int D, bool F32, bool INS>
__global__ void k_predicates(const double* pts, const long long* keys, uint32_t nq, int8_t* sign,
                             int8_t* stage, uint32_t* flags) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nq) return;
  constexpr int NP = INS ? D + 2 : D + 1;
  PtsX X;
  const double* q = pts + (size_t)t * NP * D;
#pragma unroll
  for (int i = 0; i < NP; i++) {
#pragma unroll
    for (int a = 0; a < 3; a++) X.p[i][a] = (a < D) ? q[i * D + a] : 0.0;
    X.key[i] = keys ? (unsigned long long)keys[(size_t)t * NP + i] : (unsigned long long)i;
  }
  PredT<F32> pr;
  pr.init(flags);
  int s;
  if (INS) s = pr.template insphere<D>(X);
  else s = pr.template orient<D>(X);
  const int w = INS ? 1 : 0;
  sign[t] = (int8_t)s;
  if (stage) {
    int8_t g;
    if (F32) g = pr.st.f32ok[w] ? 0 : (pr.st.exact[w] ? 2 : 1);
    else g = pr.st.exact[w] ? 2 : 1;
    stage[t] = g;
  }
}

template <int D, bool F32>
static void launch(int kind, dim3 g, hipStream_t st, const double* pts, const long long* keys,
                   uint32_t nq, int8_t* sign, int8_t* stage, uint32_t* flags) {
  if (kind == DT_PRED_INSPHERE)
    hipLaunchKernelGGL((k_predicates<D, F32, true>), g, dim3(256), 0, st, pts, keys, nq, sign,
                       stage, flags);
  else
    hipLaunchKernelGGL((k_predicates<D, F32, false>), g, dim3(256), 0, st, pts, keys, nq, sign,
                       stage, flags);
}

}  // namespace dtk

using namespace dtk;

extern "C" int dt_predicates(int kind, int D, int precision, const double* pts,
                             const int64_t* keys, int64_t nq, int8_t* sign, int8_t* stage,
                             void* stream) {
  if (kind != DT_PRED_ORIENT && kind != DT_PRED_INSPHERE) return DT_E_INVALID_ARG;
  if ((D != 2 && D != 3) || nq < 0 || nq > 0x7FFFFFF0ll) return DT_E_INVALID_ARG;
  if (precision != DT_PREC_FP64 && precision != DT_PREC_FP32) return DT_E_INVALID_ARG;
  if (nq == 0) return DT_OK;
  if (!pts || !sign) return DT_E_INVALID_ARG;
  hipStream_t st = (hipStream_t)stream;
  UseStreamScope use(st);
  DevBuf flag;
  DT_TRY(flag.alloc(4));
  DT_HIP(hipMemsetAsync(flag.p, 0, 4, st));
  const dim3 g((uint32_t)((nq + 255) / 256));
  const long long* k = (const long long*)keys;
  uint32_t* f = flag.as<uint32_t>();
  const uint32_t n = (uint32_t)nq;
  if (D == 2 && precision == DT_PREC_FP32) launch<2, true>(kind, g, st, pts, k, n, sign, stage, f);
  else if (D == 2) launch<2, false>(kind, g, st, pts, k, n, sign, stage, f);
  else if (precision == DT_PREC_FP32) launch<3, true>(kind, g, st, pts, k, n, sign, stage, f);
  else launch<3, false>(kind, g, st, pts, k, n, sign, stage, f);
  DT_HIP(hipGetLastError());
  uint32_t hf = 0;
  DT_HIP(hipMemcpyAsync(&hf, flag.p, 4, hipMemcpyDeviceToHost, st));
  DT_HIP(hipStreamSynchronize(st));
  return hf ? DT_E_INTERNAL : DT_OK;
}
