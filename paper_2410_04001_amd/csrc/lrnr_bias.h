// Internal declaration shared by csrc/lrnr_bias.hip and csrc/fastlrnr.hip.
#pragma once

#include "lrnr_internal.h"

namespace lrnr {

// Reduced bias basis of a FastLRNR: rows of the full basis at the indices P
// (host copy for the checks, device copy for the gather).
int32_t bias_gather(const lrnr_bias_basis* full, const int32_t* P_host, const int32_t* P_dev,
                    const lrnr_net* reduced_net, float* B_hat, lrnr_bias_basis* reduced,
                    hipStream_t stream);

}  // namespace lrnr
