// Dispatch of the fused kernel over the compiled rank tiles; the kernel body is
// in lrnr_fused_impl.h and each tile is instantiated in its own source file.
#include <algorithm>

#include "lrnr_internal.h"

namespace lrnr {

template <int RP>
hipError_t launch_rp(int mode, const KNet& net, const KInst& inst, const KGrid& grid,
                     hipStream_t stream);
template <int RP>
hipError_t launch_table_rp(int mode, const KTableGrid& tg, int grid, hipStream_t stream);
template <int RP>
int table_grid_rp(int mode, int Wmax_p);

size_t fused_lds_bytes(int RP, int Wmax_p, int n_slabs) {
  const size_t n = (size_t)std::max(1, n_slabs);
  const size_t floats = n * ((size_t)Wmax_p * RP * 3 + Wmax_p + RP) +
                        n * kWaves * ((size_t)Wmax_p + RP) + kWaves * 5;
  return floats * sizeof(float);
}

// Resident layers are worth it where a tile is short (narrow layers, small
// ranks): the per-layer staging costs two or three workgroup barriers per
// layer and sweep.  The budget keeps three workgroups per CU within the
// 160 KB of LDS, so occupancy stays register-bound.
constexpr size_t kResidentLdsMax = 48 * 1024;

int resident_layers(int RP, int Wmax_p, int L) {
  const int n = L - 1;
  if (n < 1 || fused_lds_bytes(RP, Wmax_p, n) > kResidentLdsMax) return 0;
  return n;
}

int padded_rank(int rmax) {
  if (rmax <= 4) return 4;
  if (rmax <= 8) return 8;
  if (rmax <= 16) return 16;
  if (rmax <= 20) return 20;
  if (rmax <= 24) return 24;
  if (rmax <= 32) return 32;
  return -1;
}

hipError_t launch_fused(int RP, int mode, const KNet& net, const KInst& inst,
                        const KGrid& grid, hipStream_t stream) {
  switch (RP) {
    case 4: return launch_rp<4>(mode, net, inst, grid, stream);
    case 8: return launch_rp<8>(mode, net, inst, grid, stream);
    case 16: return launch_rp<16>(mode, net, inst, grid, stream);
    case 20: return launch_rp<20>(mode, net, inst, grid, stream);
    case 24: return launch_rp<24>(mode, net, inst, grid, stream);
    case 32: return launch_rp<32>(mode, net, inst, grid, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_table(int RP, int mode, const KTableGrid& tg, int grid, hipStream_t stream) {
  switch (RP) {
    case 4: return launch_table_rp<4>(mode, tg, grid, stream);
    case 8: return launch_table_rp<8>(mode, tg, grid, stream);
    case 16: return launch_table_rp<16>(mode, tg, grid, stream);
    case 20: return launch_table_rp<20>(mode, tg, grid, stream);
    case 24: return launch_table_rp<24>(mode, tg, grid, stream);
    case 32: return launch_table_rp<32>(mode, tg, grid, stream);
    default: return hipErrorInvalidValue;
  }
}

int table_grid_size(int RP, int mode, int Wmax_p) {
  switch (RP) {
    case 4: return table_grid_rp<4>(mode, Wmax_p);
    case 8: return table_grid_rp<8>(mode, Wmax_p);
    case 16: return table_grid_rp<16>(mode, Wmax_p);
    case 20: return table_grid_rp<20>(mode, Wmax_p);
    case 24: return table_grid_rp<24>(mode, Wmax_p);
    case 32: return table_grid_rp<32>(mode, Wmax_p);
    default: return -1;
  }
}

}  // namespace lrnr
