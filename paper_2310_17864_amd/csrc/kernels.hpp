// Host-side entry points of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace ctca {

bool geometry_supported_one(int W, int M);
bool geometry_supported_pack(int W, int M);
hipError_t launch_one(const Inst& in, hipStream_t st);
hipError_t launch_persistent(const Inst* d_insts, const Pack* d_packs, int npacks, int* d_head,
                             int grid, hipStream_t st);
hipError_t launch_fill(int* p, int n, int v, hipStream_t st);
hipError_t launch_pad(const PadDesc* d_desc, int n, int64_t max_elems, hipStream_t st);
hipError_t launch_pad_one(const PadDesc& pd, hipStream_t st);
int persistent_blocks_per_cu();

}  // namespace ctca
