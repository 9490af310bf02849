// Types shared by the host library and the gfx950 kernels.
#pragma once
#include <stdint.h>

namespace ctca {

constexpr int kWave = 64;       // lanes per wavefront (CDNA)
constexpr int kBlk = 32;        // frames per backpointer word
constexpr int kUnroll = 8;      // frames per unrolled group in the forward loop
constexpr int kRing = 8;        // emission rows held in a wave's LDS ring (4 quarters x 2 rows)
constexpr int kBnd = 128;       // boundary values held between two segments
constexpr int kFlowWin = 32;    // frames a segment may run ahead of the one above it
                                // (same workgroup, flow control per 8-frame group)
constexpr int kMaxC = 256;      // largest class count served by the LDS ring
constexpr int kPackWaves = 4;   // waves per workgroup in the persistent kernels

// Device status codes (same values as the public header).
enum : int32_t { kOk = 0, kEinval = 1, kEinfeasible = 2, kEnomem = 3, kEdevice = 4 };

// One alignment as the kernels see it.  The trellis of S = 2L+1 states is cut
// into W segments of 64*M states; segment w runs on one wavefront and lane l
// of it owns states [w*64*M + l*M, w*64*M + (l+1)*M).
struct Inst {
  const float* em;     // [T][stride]: row t at em + t*stride (stride >= C)
  const int32_t* lab;  // [L]
  int32_t* path;       // [T]
  float* scores;       // [T]
  uint32_t* bp;        // backpointer planes, bp_words(T, W, M) words
  float* total;        // nullable
  int32_t* status;     // nullable
  int32_t* notify;     // nullable: host-visible completion flag (fine-grained
                       // pinned host memory), set to the status after every
                       // output of the alignment is written and visible
  int32_t T, C, L, blank;
  int32_t W, M;        // geometry
  int32_t stride;      // emission row stride in HBM and LDS: 32 or 256
  int32_t prio;        // wave issue priority 0..3
};

// Long alignments spread over several workgroups ("multi" layout): segment w
// runs on wave w % kXWaves of workgroup w / kXWaves.  Neighbouring segments in
// different workgroups exchange boundary values through a ring of 64-bit
// slots in global memory, each holding (value bits, tag) so that a reader
// recognises a slot written for the index it wants; all accesses are relaxed
// atomics.  Every word a launch writes carries its tag: the launch's
// generation g (1 .. kXGens-1) in the top bits and the frame index or count
// below, so words left by earlier launches never match and the region needs
// no reset between launches (the host resets it, synchronously, once per
// kXGens-1 launches).  The region lives in uncached device memory (one per
// device).
constexpr int kXWaves = 8;        // waves per workgroup
constexpr int kXMaxGroups = 32;   // workgroups per alignment
constexpr int kXRing = 512;       // slots per cross-workgroup boundary
constexpr int kXIdxBits = 21;     // frame index / count field of a tag
constexpr uint32_t kXIdxMask = (1u << kXIdxBits) - 1;
constexpr int kXGens = 1024;      // generations between resets
constexpr int kXMaxT = (1 << kXIdxBits) - 64;   // longest alignment of the layout
__host__ __device__ constexpr uint32_t x_gen_tag(uint32_t gen) { return gen << kXIdxBits; }
struct XChan {
  uint64_t slot[kXRing];          // (tag | frame index) << 32 | value bits
  int32_t cons;                   // tag | frames the consumer has taken
  int32_t pad[31];
};
struct XSync {
  XChan ch[kXMaxGroups - 1];      // ch[g]: from workgroup g to workgroup g+1
  int32_t done[kXWaves * kXMaxGroups];   // tag | 1 once segment w's backpointers are visible
};
__host__ __device__ constexpr bool geometry_is_multi(int W, int M) { return M <= 16 && W > 4; }

// Checkpointed long form (memory-bounded): a first pass over the whole
// alignment keeps only the column a_t of every K-th frame (t = 0, K, 2K, ...)
// and no backpointers; then, from the last K-frame stretch to the first, each
// stretch is run again from its column with backpointers for its K frames
// only, and backtracked from the state the stretch after it ended on.  The
// same arithmetic in the same order gives the same columns, so the path is
// bitwise the one of the full run.  Columns hold every state slot of the
// layout (W*64*M floats, padding slots included) in state order.
enum : int32_t { kModeFull = 0, kModeCkFirst = 1, kModeCkSeg = 2 };
struct CkArgs {
  float* ck;         // column k (a_{kK}) at ck + k * spad
  int32_t* state;    // [0] state to start the next stretch's backtrack from,
                     // [1] status of the first pass (stretches run only if 0)
  int32_t spad;      // floats per column
  int32_t every;     // K: frames per stretch, a multiple of kBlk
  int32_t col;       // kModeCkSeg: the column this launch starts from
  int32_t pad_;
};

// A workgroup-sized work item of the persistent kernel: wave k runs segment
// seg[k] of instance inst[k] (inst < 0: idle); the W segments of an instance
// sit on consecutive waves starting at first[k].
struct Pack {
  int32_t inst[kPackWaves];
  int16_t seg[kPackWaves];
  int16_t first[kPackWaves];
};

// Row re-layout of one emission into the compiled LDS stride.
struct PadDesc {
  const float* src;   // [T][C]
  float* dst;         // [T][stride]
  int32_t T, C, stride, pad_;
};

// Resident serving kernel: one 16-wave workgroup per CU stays on the device
// and runs work items the host posts to it.  Everything the two sides share
// lives in fine-grained pinned host memory; the device only loads from it
// and stores to it (no read-modify-write), so there is no cross-workgroup
// atomic on the device at all.
constexpr int kServeWaves = 16;
constexpr int kServeMaxParts = 8;   // workgroups one served alignment may span
constexpr int kServePartWaves = 8;  // segments per workgroup of such an alignment (2 waves per SIMD)
enum : int32_t {
  kItemSegments = 0,   // waves run segments of the item's alignments (which/seg/first)
  kItemPart = 1,       // part `part` of `nparts` of inst[0] in the multi-workgroup layout
  kItemReset = 2,      // set every word of the sync region xs to -1
};
struct ServeItem {                // one workgroup's work: up to 16 segments
  Inst inst[kServeWaves];         // the item's alignments
  int8_t which[kServeWaves];      // wave -> index into inst (-1: idle wave)
  int8_t seg[kServeWaves];        // wave -> segment of that alignment
  int8_t first[kServeWaves];      // wave -> first wave of that alignment
  int32_t npad;                   // 1: copy pad.src into pad.dst (inst[0]'s rows) first
  int32_t kind;                   // kItem*
  PadDesc pad;
  XSync* xs;                      // kItemPart / kItemReset: the sync region
  uint32_t xtag;                  // kItemPart: the generation tag of this alignment
  int16_t part, nparts;           // kItemPart: segments 8*part .. 8*part+7
};
static_assert(sizeof(ServeItem) % 8 == 0, "items are copied in 8-byte words");
struct ServeBox {                 // per resident workgroup b (host memory)
  uint64_t mail;                  // host -> device: (sequence << 32) | 0, item in items[b]
  uint64_t ack;                   // device -> host: sequence of the last finished item
  uint64_t live;                  // device -> host: launch epoch once the workgroup runs
  uint64_t pad_[5];               // own 64-byte line
};

// Backpointer layout.  Frames 1..T-1 carry backpointers, in groups of 8
// frames, one bit per state slot and frame.  A blank slot's bit says whether
// it came from the state below.  A label slot's bit says whether it came from
// below at all; which of the two states below it came from is then the bit
// of the blank slot under it in the same frame (that blank already chose the
// better of the same two states, ties to the nearer one), unless the label
// may not skip (it repeats the previous label), in which case it came from
// the state just below.  A lane's P = M bit planes are numbered in the order
// the forward pass produces them (slot pairs from the top down: label, then
// blank) and dealt round-robin over its NQ = ceil(P/4) words (plane p ->
// word p % NQ, position p / NQ), so consecutive planes land in different
// words and their shift-ins do not wait on each other.  Word q holds R_q
// planes interleaved by frame: the plane at position r, frame i of the group
// sits at bit 31 - (R_q*i + r).  Words are stored [segment][group][word][lane].
__host__ __device__ constexpr int bp_planes(int M) { return M; }
__host__ __device__ constexpr int bp_words_per_lane(int M) { return (bp_planes(M) + 3) / 4; }
// groups per segment, rounded up to whole 32-frame blocks (the backtrack
// reads a block's four groups at fixed offsets; the tail is never used)
__host__ __device__ inline int64_t bp_groups(int64_t T) {
  constexpr int64_t per_blk = kBlk / kUnroll;
  return (T - 1 + kBlk - 1) / kBlk * per_blk;
}
__host__ __device__ inline int64_t bp_words(int64_t T, int W, int M) {
  return (int64_t)W * bp_groups(T) * bp_words_per_lane(M) * kWave;
}
// plane index of slot j's bit
__host__ __device__ constexpr int plane_of(int M, int j) { return 2 * (M / 2 - 1 - j / 2) + ((j % 2) ? 0 : 1); }
__host__ __device__ constexpr int planes_in_word(int M, int q) {
  return (bp_planes(M) - q + bp_words_per_lane(M) - 1) / bp_words_per_lane(M);
}
__host__ __device__ constexpr int plane_word(int M, int p) { return p % bp_words_per_lane(M); }
__host__ __device__ constexpr int plane_pos(int M, int p) { return p / bp_words_per_lane(M); }

}  // namespace ctca
