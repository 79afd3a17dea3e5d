// Instantiation of the fused kernels for rank tile 20.
#include "lrnr_fused_ws.h"

namespace lrnr {
template hipError_t launch_rp<20>(int, const KNet&, const KInst&, const KGrid&, hipStream_t);
template hipError_t launch_table_rp<20>(int, const KTableGrid&, int, hipStream_t);
template int table_grid_rp<20>(int, int);
}  // namespace lrnr
