// gbk_surrogate.h -- private: what the nested sampler needs of the surrogate.
#pragma once
#include <hip/hip_runtime.h>

#include "gbk.h"

namespace gbk {

// Surrogate chi2 of B device rows against the observation of `obs` into
// d_chi2 (device memory, or the device address of pinned, device-mapped host
// memory), enqueued on st.  Calls on one surrogate must be ordered.
gk_status surrogate_chi2(gk_surrogate *s, gk_model *obs, const double *d_params, int B,
                         double *d_chi2, hipStream_t st);

// True when the surrogate was trained on the instrument of m.
bool surrogate_matches(const gk_surrogate *s, const gk_model *m);

int surrogate_device(const gk_surrogate *s);

}  // namespace gbk
