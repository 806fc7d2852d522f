#pragma once
#include "dt_internal.hpp"

namespace dtk {
// Validate and pack row-major points (device pointer) into double4 records.
// pset (nullable): set of each point; duplicates count only inside a set.
// dflag: device word, hflag: pinned host word.
int prep_points(const double* dev_in, const long long* dev_keys, const uint32_t* pset, uint32_t n,
                int D, double4* out, DevBuf& scratch, uint32_t* dflag, uint32_t* hflag,
                hipStream_t st);
}  // namespace dtk
