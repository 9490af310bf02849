// Host-side entry points of the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace ctca {

bool geometry_supported_one(int W, int M);
// single-workgroup layouts only (k_one, k_one_long)
bool geometry_supported_one_wg(int W, int M);
bool geometry_supported_pack(int W, int M);
hipError_t launch_one(const Inst& in, hipStream_t st);
// one long alignment over ceil(W/8) workgroups; xs: its sync region, gen:
// the launch's generation (1 .. kXGens-1, distinct since the last reset)
hipError_t launch_multi(const Inst& in, XSync* xs, uint32_t gen, hipStream_t st);
// sets the whole sync region to -1 (to be complete before the next launch)
hipError_t launch_multi_reset(XSync* xs, hipStream_t st);
hipError_t launch_persistent(const Inst* d_insts, const Pack* d_packs, int npacks, int* d_head,
                             int grid, hipStream_t st, int64_t* d_trace = nullptr);
hipError_t launch_fill(int* p, int n, int v, hipStream_t st);
hipError_t launch_persistent_long(const Inst* d_insts, const int* d_order, int n, int* d_head,
                                  int grid, hipStream_t st);
bool geometry_supported_long_batch(int W, int M);
// the batch's longest chains: one alignment per 8-wave workgroup, M in {4..12}
bool geometry_supported_crit(int W, int M);
hipError_t launch_persistent_crit(const Inst* d_insts, const int* d_order, int n, hipStream_t st);
// the checkpointed long form: one pass (mode kModeCkFirst or kModeCkSeg) of
// an alignment in the multi-workgroup layout, as launch_multi
bool geometry_supported_ck(int W, int M);
hipError_t launch_multi_ck(const Inst& in, XSync* xs, uint32_t gen, const CkArgs& ck, int mode,
                           hipStream_t st);
hipError_t launch_spans(const int32_t* path, const float* scores, int T, int blank, int max_spans,
                        int32_t* tok, int32_t* start, int32_t* end, float* score, int32_t* count,
                        hipStream_t st);
hipError_t launch_pad(const PadDesc* d_desc, int n, int64_t max_elems, hipStream_t st);
hipError_t launch_pad_one(const PadDesc& pd, hipStream_t st);
int persistent_blocks_per_cu();
// resident serving kernel: `grid` 16-wave workgroups serving the mailboxes
// d_box[0..grid) with items d_items[0..grid) (all in mapped host memory)
hipError_t launch_serve(const ServeItem* d_items, ServeBox* d_box, const int32_t* d_stop,
                        uint64_t epoch, int64_t idle_limit, int grid, hipStream_t st);
bool geometry_supported_serve(int W, int M);
// the serving kernel's multi-workgroup parts: W <= 64 segments (8 per
// workgroup), M in {4, 6, 8}
bool geometry_supported_serve_parts(int W, int M);

}  // namespace ctca
