// Internal definitions shared by the HIP translation units of libscsurf.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "scsurf.h"

namespace sc {

constexpr int kBlockVox = 512;             // 8 x 8 x 8 voxels per block
constexpr uint64_t kKeyEmpty = ~0ull;      // never a packed key (bit 63 is clear in every key)
constexpr float kWeightScale = 1024.0f;    // sample weights live on the 2^-10 grid
constexpr float kWeightLimit = 16384.0f;   // 2^14: sums stay exact in FP32 below this
constexpr int kMaxBatchOps = 4096;
// Keyframes per chunk of the integration backward: bounds its per-workgroup
// LDS pose accumulators (3 doubles per keyframe).
constexpr int kAdjChunk = 512;
// Block record in the pool, in floats: D as FP64 at [0, 1024) (Eq. (2)
// amplifies the rounding of a stored D by W / W' when most of a voxel's
// weight is removed, so D is kept in FP64), W as FP32 at [1024, 1536), and
// the colour from 1536 (RGBA8 u32 x 512, or FP64 x 3 x 512 planar).
constexpr int kPoolW = 2 * kBlockVox;
constexpr int kPoolC = 3 * kBlockVox;

// 21 bits per axis, two's complement, x in the high bits.
__host__ __device__ inline uint64_t pack_key(int x, int y, int z)
{
    return ((uint64_t)(x & 0x1FFFFF) << 42) | ((uint64_t)(y & 0x1FFFFF) << 21) | (uint64_t)(z & 0x1FFFFF);
}

__host__ __device__ inline int sext21(uint64_t v)
{
    int x = (int)(v & 0x1FFFFF);
    return (x & 0x100000) ? x - 0x200000 : x;
}

__host__ __device__ inline void unpack_key(uint64_t k, int& x, int& y, int& z)
{
    x = sext21(k >> 42);
    y = sext21(k >> 21);
    z = sext21(k);
}

// Spatial hash of block coordinates (three large primes, XOR), as used by
// voxel hashing; the table size is a power of two.
__host__ __device__ inline uint32_t hash_block(int x, int y, int z)
{
    return ((uint32_t)x * 73856093u) ^ ((uint32_t)y * 19349669u) ^ ((uint32_t)z * 83492791u);
}

// One keyframe operation (integrate or de-integrate a keyframe at a pose):
// everything the voxel pass needs, precomputed on the host.
struct OpDesc {
    // The projection's constants first and contiguous (za at byte 64), so
    // that a pass reads them with a few wide scalar loads.
    const uint4* packed;  // optional interleaved {depth, weight, RGBA8, 0} per pixel (RGBA8 volumes)
    float fx, fy, cx, cy;
    float kin_u, kin_v;   // 1/2 - (2 + |c|) 2^-21 for cx and cy: bound of the pixel rounding test
    float wl, hl, wf;     // width - 1, height - 1 and width as FP32
    int32_t width, height;
    int32_t sign;         // +1 integrate, -1 de-integrate
    int32_t kf;           // keyframe index within the call (for gradients)
    int32_t rec_mode;     // touched-block record, see below
    float za[8][3];       // za[k][row] = fl32(k * a[2][row]): camera step of k voxels along world z
    const float* depth;   // Z*, H x W
    const float* weight;  // W*, H x W
    const void* color;    // RGBA8 (uint32 per pixel) or float x 3
    const float2* cells;  // with packed: {zmin, zmax} of the valid pixels of each 4 x 4 cell
    double R[9];          // camera -> world rotation, row-major
    double t[3];          // camera -> world translation
    float a[3][3];        // a[axis][row] = fl32(s * R[axis][row]): camera step of one voxel along a world axis
    double az[3];         // s * R[axis][2] in FP64: camera-z step per voxel for the continuous distance
    // Touched-block record of this (keyframe, pose): an integration with
    // rec_mode 1 appends every block it touches; a de-integration with
    // rec_mode 2 takes those blocks as its candidates (the same keyframe at
    // the same pose touches the same blocks) when the record did not
    // overflow; rec_mode 0: no record.
    uint64_t* rec_keys;   // rec_cap keys
    uint32_t* rec_count;  // appended so far (may exceed rec_cap: overflowed)
    int32_t rec_cap;
};
static_assert(offsetof(OpDesc, za) == 64, "projection constants of OpDesc: za at byte 64");

// Device view of a volume.
struct VolDev {
    uint64_t* keys;        // n_buckets packed block keys (kKeyEmpty = free)
    int32_t* vals;         // n_buckets pool slots
    uint64_t* slot_keys;   // max_blocks: key of each pool slot
    float* pool;           // max_blocks x stride floats
    uint32_t* n_blocks;    // allocated blocks (pool cursor)
    int32_t* err;          // sticky error word
    uint32_t bucket_mask;
    int32_t max_blocks;
    int32_t stride;        // floats per block: 2048 (RGBA8) or 4608 (F32 mode, colour as double)
    int32_t color_mode;
    float s;               // voxel size
    float mu;              // truncation
};

// Candidate-block table used to deduplicate the blocks that keyframe
// operations may touch (scratch owned by the volume).
struct CandDev {
    uint64_t* keys;       // cand buckets
    uint64_t* mask;       // cand buckets x words: bit o set if operation o proposed the block
    uint32_t* list;       // occupied buckets in insertion order (plain path)
    uint32_t* sorted;     // occupied buckets ordered by operation count (batched path), one per bucket
    uint64_t* skey;       // block key of each sorted entry
    int32_t* sslot;       // pool slot of each sorted entry's block before the pass (-1: not allocated)
    uint32_t* counters;   // [0..1] list length (parity), [2..3] work cursor (parity),
                          // [4] batch candidates, [5] batch work cursor, [6] batch tile cursor
    uint32_t* bins;       // per-operation-count histogram / offsets (batched path)
    uint32_t* cursors;    // two sets (candidate stage, voxel pass) of kCursors work cursors, kCursorStride words apart
    uint32_t* big;        // [0] tiles whose block box exceeds the bit map, then up to kBigCap of their items
    unsigned long long* stats;  // cumulative: candidate blocks, (block, op) pairs, voxel updates, blocks written
    uint32_t mask_bits;   // cand buckets - 1
    uint32_t cap;         // list capacity (plain path)
    int32_t words;        // 64-bit mask words per bucket
};

// Work cursors of the batched passes: a device-wide atomic on one address is
// serviced one at a time, so the items of a pass are split over kCursors
// interleaved ranges, each with its own counter in its own 4 KB page.
constexpr int kCursors = 32;
constexpr int kCursorStride = 1024;  // 32-bit words
constexpr int kCursorDone = 512;     // word of the bit mask of exhausted ranges (its own cache line)
constexpr int kCursorSet = kCursors * kCursorStride;  // words per set
constexpr int kBigCap = 16384;  // listed tiles with an oversized block box (beyond: every tile is redone)

// Batched-update header in device memory, so a captured graph can be
// replayed with a different number of operations.
struct BatchHdr {
    int32_t n_ops;
    int32_t tiles_x, tiles_y;
    int32_t n_tile_ops;              // operations whose candidates come from frustum cells
    int16_t tile_ops[kMaxBatchOps];  // their indices (the others take a touched-block record)
};

inline bool is_pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

}  // namespace sc

// The opaque handle behind the C ABI.
struct sc_volume {
    sc_volume_params p;
    int device;
    sc::VolDev dev;
    sc::CandDev cand;
    sc::OpDesc* d_ops;       // device, max_batch_ops (+ one for the plain path)
    sc::OpDesc* h_ops;       // pinned host staging, two buffers of max_batch_ops
    sc::BatchHdr* d_hdr;     // device
    sc::BatchHdr* h_hdr;     // pinned host staging, two buffers
    uint32_t cand_buckets;
    int parity;              // plain-path candidate counter parity
    hipStream_t cap_stream;  // private stream used for graph capture
    hipEvent_t staged[2];    // recorded after each staging buffer's descriptors were copied to the device
    int stage;               // staging buffer the next chunk fills
    hipGraphExec_t graph_pre[2];  // captured candidate stage (init, candidates, histogram, scan, scatter): pixels, cell ranges
    hipGraphExec_t graph_main[8]; // captured voxel pass per voxels-per-lane choice, unpacked / packed keyframes
    int graph_keys[8];       // schedule the voxel-pass graph of each slot was captured with
    hipEvent_t* timing_ev;   // optional per-launch event pairs (2 * timing_cap)
    int timing_cap, timing_n;
    sc_schedule sched;
    int n_cu;
    int cand_wgs[2];         // resident workgroups per CU of the batched candidate kernel: pixels, cell ranges
    int plain_wgs;           // resident workgroups per CU of the plain update kernel
    double* adj_acc;         // device, 3 x kAdjChunk: pose terms of one backward chunk (zero between calls)
    struct RecordRegistry* rec;  // touched-block records of integrations (host index, device lists)
    struct StreamStore* stream;  // host store of streamed-out blocks (streaming mode)
};
