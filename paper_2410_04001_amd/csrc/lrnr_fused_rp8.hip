// Instantiation of the fused kernel for rank tile 8.
#include "lrnr_fused_ws.h"

namespace lrnr {
template hipError_t launch_rp<8>(int, const KNet&, const KInst&, const KGrid&, hipStream_t);
}  // namespace lrnr
