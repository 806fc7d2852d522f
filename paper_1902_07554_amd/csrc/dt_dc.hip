// Divide-and-conquer pipeline (Algorithm 1 with the divide of Algorithm 2).
#include "dt_common.hpp"
#include "dt_internal.hpp"
#include "dt_pipeline.hpp"

namespace dtk {
int run_dc(const double*, int64_t, int, int, double, const dt_options&, bool, hipStream_t,
           dt_result*) {
  return DT_E_INVALID_ARG;
}
}  // namespace dtk
