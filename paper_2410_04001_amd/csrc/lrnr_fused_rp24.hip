// Instantiation of the fused kernels for rank tile 24.
#include "lrnr_fused_ws.h"

namespace lrnr {
template hipError_t launch_rp<24>(int, const KNet&, const KInst&, const KGrid&, hipStream_t);
template hipError_t launch_table_rp<24>(int, const KTableGrid&, int, hipStream_t);
template int table_grid_rp<24>(int, int);
}  // namespace lrnr
