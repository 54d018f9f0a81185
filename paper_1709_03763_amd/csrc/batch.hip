// Batched surface correction (Sec. 4.3): one pose-graph update applied as
// de-integration of the selected keyframes at their integration poses and
// re-integration at their updated poses, in one graph-captured sequence whose
// voxel work is a single persistent launch.
//
// Sequence (all on the device, replayable):
//   1. reset counters and the histogram
//   2. candidate blocks of every operation (per-pixel frustum cells,
//      deduplicated per tile in LDS, then in a global table whose per-block
//      bit mask records which operations proposed the block)
//   3. histogram of operations per candidate block, descending scan, scatter:
//      the work queue holds the busiest blocks first
//   4. persistent voxel pass: each worker pops a block, loads its voxels once,
//      applies the proposing operations in processing order in registers
//      (the touched test decides per voxel), allocates the block if a
//      re-integration touched it, writes it back once, and clears its
//      candidate entry.
#include <stddef.h>
#include <string.h>

#include <stdio.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "kernels.hpp"

namespace sc {

// Clears the batch's counters, cursors and histogram, and starts an empty
// record for every integration that records its touched blocks; run by one
// workgroup of the first candidate kernel (nothing else that kernel does
// reads them).
__device__ inline void batch_init(const OpDesc* __restrict__ ops, const BatchHdr* hdr, const CandDev& cd, int n_bins)
{
    for (int i = threadIdx.x; i < 8; i += blockDim.x) cd.counters[4 + i] = 0u;
    for (int i = threadIdx.x; i < 2 * kCursors; i += blockDim.x) cd.cursors[i * kCursorStride] = 0u;
    if (threadIdx.x < 2) cd.cursors[threadIdx.x * kCursorSet + kCursorDone] = 0u;
    if (threadIdx.x == 0) cd.big[0] = 0u;
    for (int i = threadIdx.x; i < n_bins; i += blockDim.x) cd.bins[i] = 0u;
    for (int o = threadIdx.x; o < hdr->n_ops; o += blockDim.x)
        if (ops[o].rec_mode == 1) *ops[o].rec_count = 0u;
}

// A de-integration whose touched-block record is complete takes its
// candidates from the record instead of from frustum cells.
__device__ inline bool uses_record(const OpDesc& op)
{
    return op.rec_mode == 2 && *op.rec_count <= (uint32_t)op.rec_cap;
}

// Candidate blocks of de-integrations from their records: every recorded
// block is claimed in the candidate table and marked with the operation's
// bit.  Workgroup (x, y) takes operations y, y + gridDim.y, ... and, of each,
// the keys x * 256 + threadIdx.x + k * gridDim.x * 256.  A record that
// overflowed its capacity is not used: the operation's frustum-cell tiles
// are generated here instead, tile x, x + gridDim.x, ...
__global__ __launch_bounds__(256) void cand_record_kernel(const OpDesc* __restrict__ ops, const BatchHdr* hdr,
                                                          VolDev v, CandDev cd, int n_bins)
{
    if (blockIdx.x == 0 && blockIdx.y == 0) batch_init(ops, hdr, cd, n_bins);
    __shared__ uint64_t lds[CandCfg<kTileBatch, kCellBatch>::lds_set];
    __shared__ uint16_t idx[CandCfg<kTileBatch, kCellBatch>::lds_set];
    const int n_ops = hdr->n_ops;
    const int tiles = hdr->tiles_x * hdr->tiles_y;
    for (int o = blockIdx.y; o < n_ops; o += gridDim.y) {
        const OpDesc& op = ops[o];
        if (op.rec_mode != 2) continue;
        if (!uses_record(op)) {
            for (int tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
                const int ty = tile / hdr->tiles_x;
                const int tx = tile - ty * hdr->tiles_x;
                cand_tile<kTileBatch, kCellBatch>(op, v, cd, nullptr, tx, ty, o, lds, idx);
                __syncthreads();
            }
            continue;
        }
        const uint32_t n = *op.rec_count;
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
            const uint64_t key = op.rec_keys[i];
            int bx, by, bz;
            unpack_key(key, bx, by, bz);
            bool fresh;
            const int gb = cand_claim(cd, v, key, bx, by, bz, fresh);
            if (gb >= 0) cand_mark(cd, gb, o);
        }
    }
}

// Frustum-cell candidates of the operations without a record, one (operation,
// 64 x 64 tile) item at a time.  Tiles differ widely in cost (grazing
// surfaces give large cell boxes), so items are handed out dynamically: item
// i belongs to range i mod kCursors, workgroup b takes item b first (no
// atomic), then kCandPop items at a time from its range's cursor; a
// workgroup that finds its range exhausted marks it in a shared bit mask and
// moves on to a range not yet marked.  One cursor for all items would
// serialise the pops (a device-wide atomic on one address is serviced one at
// a time).
// kFromCells: every operation's keyframe is packed (its cell depth ranges
// stand in for the pixels).
constexpr int kCandPop = 2;
template <bool kFromCells>
__global__ __launch_bounds__(256) void cand_batch_kernel(const OpDesc* __restrict__ ops, const BatchHdr* hdr,
                                                         VolDev v, CandDev cd)
{
    __shared__ uint64_t lds[CandCfg<kTileBatch, kCellBatch>::lds_set];
    __shared__ uint16_t idx[CandCfg<kTileBatch, kCellBatch>::lds_set];
    __shared__ float red[8];
    __shared__ int next;
    const int tiles = hdr->tiles_x * hdr->tiles_y;
    const int items = hdr->n_tile_ops * tiles;
    int r = (int)blockIdx.x % kCursors;
    int k = (int)blockIdx.x / kCursors, end = k + 1;  // index within range r
    for (;;) {
        // with no more items than workgroups every item is a static one
        if (k >= end && items <= (int)gridDim.x) break;
        if (k >= end) {
            __syncthreads();
            if (threadIdx.x == 0) {
                // range r's first indices went to the static first items
                const int base = ((int)gridDim.x - r + kCursors - 1) / kCursors;
                next = base + kCandPop * (int)atomicAdd(cd.cursors + r * kCursorStride, 1u);
            }
            __syncthreads();
            k = next;
            end = k + kCandPop;
        }
        const int it = r + kCursors * k;
        if (it >= items && items <= (int)gridDim.x) break;
        if (it >= items) {
            __syncthreads();
            if (threadIdx.x == 0) {
                const uint32_t m = atomicOr(cd.cursors + kCursorDone, 1u << r) | (1u << r);
                int nr = -1;
                for (int j = 1; j < kCursors && nr < 0; ++j)
                    if (!((m >> ((r + j) % kCursors)) & 1u)) nr = (r + j) % kCursors;
                next = nr;
            }
            __syncthreads();
            if (next < 0) break;
            r = next;
            end = k;  // pop from the new range
            continue;
        }
        const int kk = it / tiles;
        const int o = hdr->tile_ops[kk];
        const int tile = it - kk * tiles;
        const int ty = tile / hdr->tiles_x;
        const int tx = tile - ty * hdr->tiles_x;
        if (kFromCells) {
            // packed keyframes: the tile's bit map; a tile whose box is too
            // large is listed for cand_big_kernel (the hash set)
            if (!cand_tile_bits<kTileBatch>(ops[o], v, cd, tx, ty, o, reinterpret_cast<uint32_t*>(lds), idx, red) &&
                threadIdx.x == 0) {
                const uint32_t pos = atomicAdd(cd.big, 1u);
                if (pos < (uint32_t)kBigCap) cd.big[1 + pos] = (uint32_t)it;
            }
        } else {
            cand_tile<kTileBatch, kCellBatch, false>(ops[o], v, cd, nullptr, tx, ty, o, lds, idx);
        }
        __syncthreads();
        ++k;
    }
}

// The tiles of packed keyframes whose block box exceeds the bit map, on the
// LDS hash set: the listed items, or every item when the list overflowed
// (inserting a tile's candidates twice changes nothing).
__global__ __launch_bounds__(256) void cand_big_kernel(const OpDesc* __restrict__ ops, const BatchHdr* hdr, VolDev v,
                                                       CandDev cd)
{
    __shared__ uint64_t lds[CandCfg<kTileBatch, kCellBatch>::lds_set];
    __shared__ uint16_t idx[CandCfg<kTileBatch, kCellBatch>::lds_set];
    const int tiles = hdr->tiles_x * hdr->tiles_y;
    const int items = hdr->n_tile_ops * tiles;
    const uint32_t nb = cd.big[0];
    const bool all = nb > (uint32_t)kBigCap;
    const int count = all ? items : (int)nb;
    for (int k = blockIdx.x; k < count; k += gridDim.x) {
        const int it = all ? k : (int)cd.big[1 + k];
        const int kk = it / tiles;
        const int o = hdr->tile_ops[kk];
        const int tile = it - kk * tiles;
        const int ty = tile / hdr->tiles_x;
        const int tx = tile - ty * hdr->tiles_x;
        cand_tile<kTileBatch, kCellBatch, true>(ops[o], v, cd, nullptr, tx, ty, o, lds, idx);
        __syncthreads();
    }
}

// Workgroups of cand_batch_kernel that fit on one CU at once (registers and
// LDS); the kernel strides over its items statically, so a grid larger than
// this runs its surplus as a second, mostly idle wave of workgroups.
int cand_batch_resident_wgs(bool from_cells)
{
    int n = 0;
    const hipError_t e =
        from_cells ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, cand_batch_kernel<true>,
                                                                  CandCfg<kTileBatch, kCellBatch>::threads, 0)
                   : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, cand_batch_kernel<false>,
                                                                  CandCfg<kTileBatch, kCellBatch>::threads, 0);
    if (e != hipSuccess) n = 0;
    return std::max(1, std::min(n, 8));
}

__device__ inline int mask_count(const CandDev& cd, uint32_t h)
{
    int c = 0;
    for (int w = 0; w < cd.words; ++w) c += __popcll(cd.mask[(size_t)h * cd.words + w]);
    return c;
}

// Occupied buckets of one wavefront's stretch [base, base + kCollect) of the
// candidate table (clipped at b1), compacted into the wavefront's LDS list in
// bucket order; returns their number.  All key loads issue together, so the
// scans below wait for one load latency per stretch instead of one per
// bucket a lane visits.  Every lane of the wavefront takes part.
constexpr int kCollectPerLane = 8;
constexpr int kCollect = 64 * kCollectPerLane;

__device__ inline int wave_collect(const CandDev& cd, uint32_t base, uint32_t b1, uint32_t* list, int lane)
{
    uint64_t key[kCollectPerLane];
#pragma unroll
    for (int k = 0; k < kCollectPerLane; ++k) {
        const uint32_t i = base + 64u * k + (uint32_t)lane;
        key[k] = i < b1 ? cd.keys[i] : kKeyEmpty;
    }
    int n = 0;
#pragma unroll
    for (int k = 0; k < kCollectPerLane; ++k) {
        const bool occ = key[k] != kKeyEmpty;
        const uint64_t bal = __ballot(occ);
        if (occ) list[n + (int)lanes_below(bal)] = base + 64u * k + (uint32_t)lane;
        n += __popcll(bal);
    }
    wave_lds_sync();
    return n;
}

// Each workgroup takes a contiguous share of the candidate table's buckets,
// so the histogram and the scatter below see the same buckets per workgroup.
__device__ inline void wg_share(uint32_t n, uint32_t& b0, uint32_t& b1)
{
    const uint32_t per = (n + gridDim.x - 1) / gridDim.x;
    b0 = min(n, blockIdx.x * per);
    b1 = min(n, b0 + per);
}

// Histogram of operation counts over the occupied buckets, privatised in LDS
// per workgroup.
__global__ __launch_bounds__(256) void hist_kernel(CandDev cd, int n_bins)
{
    __shared__ uint32_t h[kMaxBatchOps + 1];
    __shared__ uint32_t lst[4][kCollect];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t b0, b1;
    wg_share(cd.mask_bits + 1u, b0, b1);
    for (int c = threadIdx.x; c < n_bins; c += blockDim.x) h[c] = 0u;
    __syncthreads();
    for (uint32_t base = b0 + wave * kCollect; base < b1; base += 4 * kCollect) {
        const int n = wave_collect(cd, base, b1, lst[wave], lane);
        for (int r = lane; r < n; r += 64) atomicAdd(h + min(mask_count(cd, lst[wave][r]), n_bins - 1), 1u);
        wave_lds_sync();
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n_bins; c += blockDim.x)
        if (h[c]) atomicAdd(cd.bins + c, h[c]);
}

// Exclusive scan in descending operation count: offset[c] = #blocks with more
// than c operations; the total is the number of candidate blocks.  One
// workgroup; n_bins <= 4097.
__global__ __launch_bounds__(1024) void scan_kernel(CandDev cd, int n_bins)
{
    __shared__ uint32_t part[1024];
    const int tid = threadIdx.x;
    const int per = (n_bins + 1023) / 1024;
    // thread tid owns bins (descending) [n_bins-1 - tid*per, ...]
    uint32_t sum = 0;
    for (int k = 0; k < per; ++k) {
        const int c = n_bins - 1 - (tid * per + k);
        if (c >= 0) sum += cd.bins[c];
    }
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t x = (tid >= off) ? part[tid - off] : 0u;
        __syncthreads();
        part[tid] += x;
        __syncthreads();
    }
    uint32_t run = (tid > 0) ? part[tid - 1] : 0u;
    for (int k = 0; k < per; ++k) {
        const int c = n_bins - 1 - (tid * per + k);
        if (c >= 0) {
            const uint32_t b = cd.bins[c];
            cd.bins[c] = run;
            run += b;
        }
    }
    if (tid == 1023) {
        cd.counters[4] = part[1023];
        cd.stats[0] += part[1023];  // slot 0 of counter 0
    }
}

// Scatter into operation-count order: each workgroup reserves one range per
// count it holds, then places its buckets inside those ranges, with each
// block's key and current pool slot (looked up here, in parallel, so the
// voxel pass starts a block with one round of independent loads).  Both
// passes over the workgroup's buckets compact the occupied ones first.
__global__ __launch_bounds__(256) void scatter_kernel(CandDev cd, VolDev v, int n_bins)
{
    __shared__ uint32_t h[kMaxBatchOps + 1];
    __shared__ uint32_t lst[4][kCollect];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t b0, b1;
    wg_share(cd.mask_bits + 1u, b0, b1);
    for (int c = threadIdx.x; c < n_bins; c += blockDim.x) h[c] = 0u;
    __syncthreads();
    for (uint32_t base = b0 + wave * kCollect; base < b1; base += 4 * kCollect) {
        const int n = wave_collect(cd, base, b1, lst[wave], lane);
        for (int r = lane; r < n; r += 64) atomicAdd(h + min(mask_count(cd, lst[wave][r]), n_bins - 1), 1u);
        wave_lds_sync();
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n_bins; c += blockDim.x)
        if (h[c]) h[c] = atomicAdd(cd.bins + c, h[c]);
    __syncthreads();
    for (uint32_t base = b0 + wave * kCollect; base < b1; base += 4 * kCollect) {
        const int n = wave_collect(cd, base, b1, lst[wave], lane);
        for (int r = lane; r < n; r += 64) {
            const uint32_t i = lst[wave][r];
            const uint64_t key = cd.keys[i];
            const uint32_t pos = atomicAdd(h + min(mask_count(cd, i), n_bins - 1), 1u);
            int bx, by, bz;
            unpack_key(key, bx, by, bz);
            cd.sorted[pos] = i;
            cd.skey[pos] = key;
            cd.sslot[pos] = vol_find(v, key, bx, by, bz);
        }
        wave_lds_sync();
    }
}

// Voxel state of one lane: VPL voxels along z of the lane's (x, y) column.
template <int CM, int VPL>
struct LaneVox {
    double D[VPL];
    float W[VPL];
    uint32_t C[VPL];       // RGBA8
    double Cf[3][VPL];     // FP32-colour mode (held in FP64)
};

template <int CM, int VPL>
__device__ inline void load_vox(LaneVox<CM, VPL>& s, const float* blk, int lane, int kz0)
{
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
        const int i = lane + 64 * (kz0 + j);
        s.D[j] = reinterpret_cast<const double*>(blk)[i];
        s.W[j] = blk[kPoolW + i];
        if (CM == SC_COLOR_RGBA8) {
            s.C[j] = reinterpret_cast<const uint32_t*>(blk + kPoolC)[i];
        } else {
            const double* Cd = reinterpret_cast<const double*>(blk + kPoolC);
            s.Cf[0][j] = Cd[i];
            s.Cf[1][j] = Cd[512 + i];
            s.Cf[2][j] = Cd[1024 + i];
        }
    }
}

template <int CM, int VPL>
__device__ inline void zero_vox(LaneVox<CM, VPL>& s)
{
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
        s.D[j] = 0.0;
        s.W[j] = 0.0f;
        s.C[j] = 0u;
        s.Cf[0][j] = s.Cf[1][j] = s.Cf[2][j] = 0.0;
    }
}

template <int CM, int VPL>
__device__ inline void store_vox(const LaneVox<CM, VPL>& s, float* blk, int lane, int kz0, uint32_t touched)
{
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
        if (!((touched >> j) & 1u)) continue;
        const int i = lane + 64 * (kz0 + j);
        reinterpret_cast<double*>(blk)[i] = s.D[j];
        blk[kPoolW + i] = s.W[j];
        if (CM == SC_COLOR_RGBA8) {
            reinterpret_cast<uint32_t*>(blk + kPoolC)[i] = s.C[j];
        } else {
            double* Cd = reinterpret_cast<double*>(blk + kPoolC);
            Cd[i] = s.Cf[0][j];
            Cd[512 + i] = s.Cf[1][j];
            Cd[1024 + i] = s.Cf[2][j];
        }
    }
}

// Applies one operation to the lane's voxels.  Updates `touched` (voxels
// changed), `re_touch` (some re-integration touched a voxel) and the error
// flags.  `allocated` says whether the block existed before the batch.
template <int CM, int VPL>
__device__ inline void apply_op(const OpDesc& op, const VolDev& v, int bx, int by, int bz, int lane, int kz0,
                                bool allocated, LaneVox<CM, VPL>& s, uint32_t& touched, bool& re_touch,
                                bool& e_notalloc, bool& e_weight, uint32_t& n_upd)
{
    float q[3];
    double qz;
    block_origin(op, v.s, bx, by, bz, q, qz);
    const float kx = (float)(lane & 7), ky = (float)(lane >> 3);
    float base[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) base[r] = (q[r] + kx * op.a[0][r]) + ky * op.a[1][r];
    const double bz64 = (qz + (double)(lane & 7) * op.az[0]) + (double)(lane >> 3) * op.az[1];
    VoxHits<CM, VPL> h;
    test_voxels<CM, VPL>(op, v.mu, base, kz0, h);
    if (h.hit == 0u) return;
    if (op.sign < 0 && !allocated) {
        e_notalloc = true;
        return;
    }
    if (op.sign > 0) re_touch = true;
    touched |= h.hit;
    n_upd += __popc(h.hit);
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
        if (!((h.hit >> j) & 1u)) continue;
        const double d = distance(h.z[j], bz64 + (double)(kz0 + j) * op.az[2]);
        if (CM == SC_COLOR_RGBA8) {
            e_weight |= !update_rgba8(s.D[j], s.W[j], s.C[j], d, h.w[j], h.c[j], op.sign);
        } else {
            const float* cp = reinterpret_cast<const float*>(op.color) + 3 * h.pix[j];
            const float c[3] = {__ldg(cp), __ldg(cp + 1), __ldg(cp + 2)};
            double C3[3] = {s.Cf[0][j], s.Cf[1][j], s.Cf[2][j]};
            e_weight |= !update_f32(s.D[j], s.W[j], C3, d, h.w[j], c, op.sign);
            s.Cf[0][j] = C3[0];
            s.Cf[1][j] = C3[1];
            s.Cf[2][j] = C3[2];
        }
    }
}

// Persistent voxel pass, one wavefront per block (eight voxels per lane,
// lane = x + 8 y, z in a loop); the wavefronts of a workgroup are independent.
template <int CM>
__global__ __launch_bounds__(256) void batch_main_wave_kernel(const OpDesc* __restrict__ ops, VolDev v, CandDev cd)
{
    constexpr int VPL = 8;
    const int lane = threadIdx.x & 63;
    const uint32_t n = cd.counters[4];
    const uint32_t worker = blockIdx.x * (blockDim.x >> 6) + bcast(threadIdx.x >> 6);
    const uint32_t n_workers = gridDim.x * (blockDim.x >> 6);
    WorkCursor cur;
    cursor_init(cur, worker);
    uint32_t n_upd = 0, n_pairs = 0, n_written = 0;
    for (;;) {
        const uint32_t i = cursor_pop(cur, cd.counters + 5, n_workers, lane);
        if (i >= n) break;
        const uint32_t h = bcast(cd.sorted[i]);
        const uint64_t key = bcast64(cd.skey[i]);
        int slot = (int)bcast((uint32_t)cd.sslot[i]);
        int bx, by, bz;
        unpack_key(key, bx, by, bz);
        LaneVox<CM, VPL> st;
        if (slot >= 0)
            load_vox<CM, VPL>(st, v.pool + (size_t)slot * v.stride, lane, 0);
        else
            zero_vox<CM, VPL>(st);
        uint32_t touched = 0;
        bool re_touch = false, e_na = false, e_w = false;
        for (int w = 0; w < cd.words; ++w) {
            uint64_t m = bcast64(cd.mask[(size_t)h * cd.words + w]);
            n_pairs += __popcll(m);
            while (m) {
                const int b = __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                apply_op<CM, VPL>(ops[w * 64 + b], v, bx, by, bz, lane, 0, slot >= 0, st, touched, re_touch, e_na,
                                  e_w, n_upd);
            }
        }
        const int all = (__ballot(re_touch) ? 1 : 0) | (__ballot(e_na) ? 2 : 0) | (__ballot(e_w) ? 4 : 0);
        if (slot < 0 && (all & 1)) slot = vol_insert_wave(v, key, bx, by, bz, lane);
        if (slot >= 0) store_vox<CM, VPL>(st, v.pool + (size_t)slot * v.stride, lane, 0, touched);
        const bool wrote = __ballot(touched != 0) != 0;
        n_written += (slot >= 0 && wrote) ? 1u : 0u;
        retire_candidate(cd, v, h, all, lane);
    }
    stat_add(cd, 1, worker, n_pairs, lane);
    stat_add(cd, 2, worker, wave_sum(n_upd), lane);
    stat_add(cd, 3, worker, n_written, lane);
}

// LDS bytes per wavefront of the compacting voxel pass: block state
// (D f64, W f32; colour RGBA8 u32 or 3 x f64) and the queue of one part's
// touched voxels (voxel u16; quantised weight, keyframe depth, and RGBA8
// colour or pixel index, 4 bytes each).
template <int CM, int TV>
constexpr int compact_wave_bytes()
{
    return 512 * (8 + 4 + (CM == SC_COLOR_RGBA8 ? 4 : 24)) + 64 * TV * (2 + 4 + 4 + 4);
}

// Persistent voxel pass, compacting: one wavefront per block with the block
// state in LDS.  For each operation the lanes test their own voxels TV at a
// time (a part); the touched ones of a part are gathered into an LDS queue
// (ballot + mbcnt) together with the keyframe samples already loaded for the
// test, and all 64 lanes then update consecutive queue entries.  The update
// work follows the number of touched voxels rather than the number of
// z-slices that hold one, and no keyframe sample is loaded twice.  Per voxel
// the operations still apply in bit order.
template <int CM, int TV>
__global__ __launch_bounds__(256) void batch_compact_kernel(const OpDesc* __restrict__ ops, VolDev v, CandDev cd)
{
    constexpr int Q = 64 * TV;  // queue entries
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = (int)bcast(threadIdx.x >> 6);
    unsigned char* wb = smem + (size_t)wave * compact_wave_bytes<CM, TV>();
    double* sD = reinterpret_cast<double*>(wb);
    float* sW = reinterpret_cast<float*>(sD + 512);
    uint32_t* sC = reinterpret_cast<uint32_t*>(sW + 512);  // RGBA8
    double* sCf = reinterpret_cast<double*>(sW + 512);     // FP32 colour: [3][512]
    float* qw = reinterpret_cast<float*>(wb + 512 * (12 + (CM == SC_COLOR_RGBA8 ? 4 : 24)));
    float* qz = qw + Q;
    uint32_t* qc = reinterpret_cast<uint32_t*>(qz + Q);  // RGBA8 colour, or pixel index (FP32 colour)
    uint16_t* qvox = reinterpret_cast<uint16_t*>(qc + Q);
    const uint32_t n = cd.counters[4];
    const uint32_t worker = blockIdx.x * (blockDim.x >> 6) + (uint32_t)wave;
    const uint32_t n_workers = gridDim.x * (blockDim.x >> 6);
    WorkCursor cur;
    cursor_init(cur, worker);
    uint32_t n_upd = 0, n_pairs = 0, n_written = 0;
    for (;;) {
        const uint32_t i = cursor_pop(cur, cd.counters + 5, n_workers, lane);
        if (i >= n) break;
        const uint32_t h = bcast(cd.sorted[i]);
        const uint64_t key = bcast64(cd.skey[i]);
        int slot = (int)bcast((uint32_t)cd.sslot[i]);
        int bx, by, bz;
        unpack_key(key, bx, by, bz);
        {
            const float* blk = v.pool + (size_t)max(slot, 0) * v.stride;
            const bool have = slot >= 0;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int x = lane + 64 * j;
                sD[x] = have ? reinterpret_cast<const double*>(blk)[x] : 0.0;
                sW[x] = have ? blk[kPoolW + x] : 0.0f;
                if (CM == SC_COLOR_RGBA8) {
                    sC[x] = have ? reinterpret_cast<const uint32_t*>(blk + kPoolC)[x] : 0u;
                } else {
                    const double* Cd = reinterpret_cast<const double*>(blk + kPoolC);
                    sCf[x] = have ? Cd[x] : 0.0;
                    sCf[512 + x] = have ? Cd[512 + x] : 0.0;
                    sCf[1024 + x] = have ? Cd[1024 + x] : 0.0;
                }
            }
        }
        wave_lds_sync();
        uint32_t touched = 0;
        bool re_touch = false, e_na = false, e_w = false;
        for (int w = 0; w < cd.words; ++w) {
            uint64_t m = bcast64(cd.mask[(size_t)h * cd.words + w]);
            n_pairs += __popcll(m);
            while (m) {
                const int b = __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                const OpDesc& op = ops[w * 64 + b];
                float q[3];
                double qz0;
                block_origin(op, v.s, bx, by, bz, q, qz0);
                const float kx = (float)(lane & 7), ky = (float)(lane >> 3);
                float base[3];
#pragma unroll
                for (int r = 0; r < 3; ++r) base[r] = (q[r] + kx * op.a[0][r]) + ky * op.a[1][r];
#pragma unroll
                for (int part = 0; part < 8 / TV; ++part) {
                    VoxHits<CM, TV> hv;
                    test_voxels<CM, TV, true>(op, v.mu, base, part * TV, hv);
                    // gather this part's touched voxels, z-slice by z-slice
                    uint32_t cnt = 0u;
#pragma unroll
                    for (int j = 0; j < TV; ++j) {
                        const bool t = (hv.hit >> j) & 1u;
                        const uint64_t bal = __ballot(t);
                        if (t) {
                            const uint32_t pos = cnt + lanes_below(bal);
                            qvox[pos] = (uint16_t)(lane + 64 * (part * TV + j));
                            qw[pos] = hv.w[j];
                            qz[pos] = hv.z[j];
                            qc[pos] = (CM == SC_COLOR_RGBA8) ? hv.c[j] : (uint32_t)hv.pix[j];
                        }
                        cnt += (uint32_t)__popcll(bal);
                    }
                    if (cnt == 0u) continue;
                    if (op.sign < 0 && slot < 0) {
                        e_na = true;
                        break;
                    }
                    if (op.sign > 0) re_touch = true;
                    touched |= hv.hit << (part * TV);
                    n_upd += __popc(hv.hit);
                    wave_lds_sync();
                    // dense update of the queue, 64 entries per round
                    for (uint32_t r0 = 0; r0 < cnt; r0 += 64) {
                        const uint32_t e = r0 + (uint32_t)lane;
                        if (e < cnt) {
                            const int x = qvox[e];
                            const double pz64 =
                                ((qz0 + (double)(x & 7) * op.az[0]) + (double)((x >> 3) & 7) * op.az[1]) +
                                (double)(x >> 6) * op.az[2];
                            const double d = distance(qz[e], pz64);
                            const float wq = qw[e];
                            double D = sD[x];
                            float W = sW[x];
                            if (CM == SC_COLOR_RGBA8) {
                                uint32_t C = sC[x];
                                e_w |= !update_rgba8(D, W, C, d, wq, qc[e], op.sign);
                                sC[x] = C;
                            } else {
                                const float* cp = reinterpret_cast<const float*>(op.color) + 3 * (size_t)qc[e];
                                const float c[3] = {__ldg(cp), __ldg(cp + 1), __ldg(cp + 2)};
                                double C3[3] = {sCf[x], sCf[512 + x], sCf[1024 + x]};
                                e_w |= !update_f32(D, W, C3, d, wq, c, op.sign);
                                sCf[x] = C3[0];
                                sCf[512 + x] = C3[1];
                                sCf[1024 + x] = C3[2];
                            }
                            sD[x] = D;
                            sW[x] = W;
                        }
                    }
                    wave_lds_sync();
                }
            }
        }
        const int all = (__ballot(re_touch) ? 1 : 0) | (__ballot(e_na) ? 2 : 0) | (__ballot(e_w) ? 4 : 0);
        if (slot < 0 && (all & 1)) slot = vol_insert_wave(v, key, bx, by, bz, lane);
        if (slot >= 0) {
            float* blk = v.pool + (size_t)slot * v.stride;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (!((touched >> j) & 1u)) continue;
                const int x = lane + 64 * j;
                reinterpret_cast<double*>(blk)[x] = sD[x];
                blk[kPoolW + x] = sW[x];
                if (CM == SC_COLOR_RGBA8) {
                    reinterpret_cast<uint32_t*>(blk + kPoolC)[x] = sC[x];
                } else {
                    double* Cd = reinterpret_cast<double*>(blk + kPoolC);
                    Cd[x] = sCf[x];
                    Cd[512 + x] = sCf[512 + x];
                    Cd[1024 + x] = sCf[1024 + x];
                }
            }
        }
        const bool wrote = __ballot(touched != 0) != 0;
        n_written += (slot >= 0 && wrote) ? 1u : 0u;
        retire_candidate(cd, v, h, all, lane);
        wave_lds_sync();
    }
    stat_add(cd, 1, worker, n_pairs, lane);
    stat_add(cd, 2, worker, wave_sum(n_upd), lane);
    stat_add(cd, 3, worker, n_written, lane);
}

// LDS bytes per wavefront of the pipelined pass: the block state (512
// voxels: D f64, W f32, colour RGBA8 u32 or 3 x f64) and a queue of 128
// touched voxels (two z-slices of a lane group).
template <int CM>
constexpr int pipe_wave_bytes()
{
    return 512 * (8 + 4 + (CM == SC_COLOR_RGBA8 ? 4 : 24)) + 128 * (2 + 4 + 4 + 4);
}

// Per-wavefront LDS of the pipelined pass.
struct PipeLds {
    double* sD;      // [512]
    float* sW;       // [512]
    uint32_t* sC;    // [512] RGBA8
    double* sCf;     // [3][512] FP32-colour mode
    float* qw;       // queue: quantised weight,
    float* qz;       // keyframe depth,
    uint32_t* qc;    // RGBA8 colour or pixel index (FP32 colour),
    uint16_t* qvox;  // voxel index in the block
};

template <int CM>
__device__ inline PipeLds pipe_lds(unsigned char* wb)
{
    PipeLds L;
    L.sD = reinterpret_cast<double*>(wb);
    L.sW = reinterpret_cast<float*>(L.sD + 512);
    L.sC = reinterpret_cast<uint32_t*>(L.sW + 512);
    L.sCf = reinterpret_cast<double*>(L.sW + 512);
    L.qw = reinterpret_cast<float*>(wb + 512 * (12 + (CM == SC_COLOR_RGBA8 ? 4 : 24)));
    L.qz = L.qw + 128;
    L.qc = reinterpret_cast<uint32_t*>(L.qz + 128);
    L.qvox = reinterpret_cast<uint16_t*>(L.qc + 128);
    return L;
}

// State of the pipelined pass within one block.  slot is the block's pool
// slot before the pass (-1: not allocated).
struct PipeBlock {
    int bx, by, bz, slot;
    uint32_t touched, n_upd, pairs;
    bool re_touch, e_na, e_w;
    bool pair_any;   // the current operation touched a voxel of the block (ring pass)
    uint32_t n_rec;  // recording integrations that touched the block, not yet appended
    int rec_op;      // lane i < n_rec: the i-th of them
};

// Appends the block to the records of the integrations listed in lanes
// 0 .. n_rec - 1, one atomic per lane on that operation's counter.
__device__ inline void record_flush(const OpDesc* __restrict__ ops, PipeBlock& pb, int lane)
{
    if ((uint32_t)lane < pb.n_rec) {
        const OpDesc& o = ops[pb.rec_op];
        const uint32_t pos = atomicAdd(o.rec_count, 1u);
        if (pos < (uint32_t)o.rec_cap) o.rec_keys[pos] = pack_key(pb.bx, pb.by, pb.bz);
    }
    pb.n_rec = 0u;
}

// Issues the keyframe gathers of (operation `o`, part `part`: z-slices
// 4 part .. 4 part + 3) into `f` and returns the camera z of the block origin
// in `qz`.
template <int CM>
__device__ inline void pipe_fetch(const OpDesc& o, const VolDev& v, const PipeBlock& pb, int part, int lane,
                                  VoxFetch<CM, 4>& f, double& qz)
{
    float q[3], base[3];
    block_origin(o, v.s, pb.bx, pb.by, pb.bz, q, qz);
    const float kx = (float)(lane & 7), ky = (float)(lane >> 3);
#pragma unroll
    for (int r = 0; r < 3; ++r) base[r] = (q[r] + kx * o.a[0][r]) + ky * o.a[1][r];
    fetch_voxels<CM, 4, true>(o, base, part * 4, f);
}

// One step of the pipelined pass: issue the keyframe gathers of the next
// (operation, part) into `nxt`, then decide the current one from `cur` and
// update its touched voxels: two z-slices at a time, gathered with their
// keyframe samples into the LDS queue (ballot + mbcnt) and updated densely
// by all 64 lanes.  The dense phase reads only LDS, so the loads of `nxt`
// stay in flight meanwhile.  Per voxel the operations apply in bit order.
// Returns false when the block has no further step; otherwise op_c /
// part_c / qz_c name the next step.
template <int CM>
__device__ inline bool pipe_step(const OpDesc* __restrict__ ops, const VolDev& v, OpWalk& walk, PipeBlock& pb,
                                 VoxFetch<CM, 4>& cur, VoxFetch<CM, 4>& nxt, int& op_c, int& part_c, double& qz_c,
                                 int lane, const PipeLds& L)
{
    constexpr int TV = 4;
    int op_n, part_n;
    if (part_c == 0) {
        op_n = op_c;
        part_n = 1;
    } else {
        op_n = walk_next(walk);
        part_n = 0;
    }
    double qz_n = 0.0;
    if (op_n >= 0) pipe_fetch<CM>(ops[op_n], v, pb, part_n, lane, nxt, qz_n);
    const OpDesc& op = ops[op_c];
    pb.pairs += (part_c == 0) ? 1u : 0u;
    VoxHits<CM, TV> hv;
    decide_voxels<CM, TV>(cur, v.mu, hv);
    const bool any = __ballot(hv.hit != 0u) != 0ull;
    if (any && op.sign < 0 && pb.slot < 0) {
        pb.e_na = true;
    } else if (any) {
        if (op.sign > 0) pb.re_touch = true;
        pb.touched |= hv.hit << (part_c * TV);
        pb.n_upd += __popc(hv.hit);
#pragma unroll 1
        for (int half = 0; half < 2; ++half) {
            uint32_t cnt = 0u;
#pragma unroll
            for (int jj = 0; jj < 2; ++jj) {
                // slices jj and 2 + jj picked by selects, so no register array is indexed at run time
                const int j = 2 * half + jj;
                const bool t = (hv.hit >> j) & 1u;
                const uint64_t bal = __ballot(t);
                if (t) {
                    const uint32_t pos = cnt + lanes_below(bal);
                    L.qvox[pos] = (uint16_t)(lane + 64 * (part_c * TV + j));
                    L.qw[pos] = half ? hv.w[2 + jj] : hv.w[jj];
                    L.qz[pos] = half ? hv.z[2 + jj] : hv.z[jj];
                    L.qc[pos] = (CM == SC_COLOR_RGBA8) ? (half ? hv.c[2 + jj] : hv.c[jj])
                                                       : (uint32_t)(half ? hv.pix[2 + jj] : hv.pix[jj]);
                }
                cnt += (uint32_t)__popcll(bal);
            }
            if (cnt == 0u) continue;
            wave_lds_sync();
            for (uint32_t r0 = 0; r0 < cnt; r0 += 64) {
                const uint32_t e = r0 + (uint32_t)lane;
                if (e < cnt) {
                    const int x = L.qvox[e];
                    const double pz64 =
                        ((qz_c + (double)(x & 7) * op.az[0]) + (double)((x >> 3) & 7) * op.az[1]) +
                        (double)(x >> 6) * op.az[2];
                    const double d = distance(L.qz[e], pz64);
                    const float wq = L.qw[e];
                    double D = L.sD[x];
                    float W = L.sW[x];
                    if (CM == SC_COLOR_RGBA8) {
                        uint32_t C = L.sC[x];
                        pb.e_w |= !update_rgba8(D, W, C, d, wq, L.qc[e], op.sign);
                        L.sC[x] = C;
                    } else {
                        const float* cp = reinterpret_cast<const float*>(op.color) + 3 * (size_t)L.qc[e];
                        const float c[3] = {__ldg(cp), __ldg(cp + 1), __ldg(cp + 2)};
                        double C3[3] = {L.sCf[x], L.sCf[512 + x], L.sCf[1024 + x]};
                        pb.e_w |= !update_f32(D, W, C3, d, wq, c, op.sign);
                        L.sCf[x] = C3[0];
                        L.sCf[512 + x] = C3[1];
                        L.sCf[1024 + x] = C3[2];
                    }
                    L.sD[x] = D;
                    L.sW[x] = W;
                }
            }
            wave_lds_sync();
        }
    }
    if (op_n < 0) return false;
    op_c = op_n;
    part_c = part_n;
    qz_c = qz_n;
    return true;
}

// Persistent voxel pass, compacting and pipelined: one wavefront per block
// with the block state in LDS; per (operation, part of four z-slices) the
// touched voxels are gathered into an LDS queue with their keyframe samples
// and updated densely, and the gathers of each step are issued one step
// ahead through two fetch buffers used alternately.
template <int CM>
__global__ __launch_bounds__(256) void batch_pipe_kernel(const OpDesc* __restrict__ ops, VolDev v, CandDev cd)
{
    constexpr int TV = 4;
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = (int)bcast(threadIdx.x >> 6);
    const PipeLds L = pipe_lds<CM>(smem + (size_t)wave * pipe_wave_bytes<CM>());
    const uint32_t n = cd.counters[4];
    const uint32_t worker = blockIdx.x * (blockDim.x >> 6) + (uint32_t)wave;
    const uint32_t n_workers = gridDim.x * (blockDim.x >> 6);
    WorkCursor cur;
    cursor_init(cur, worker);
    uint32_t n_upd = 0, n_pairs = 0, n_written = 0;
    for (;;) {
        const uint32_t i = cursor_pop(cur, cd.counters + 5, n_workers, lane);
        if (i >= n) break;
        const uint32_t h = bcast(cd.sorted[i]);
        const uint64_t key = bcast64(cd.skey[i]);
        PipeBlock pb;
        pb.slot = (int)bcast((uint32_t)cd.sslot[i]);
        unpack_key(key, pb.bx, pb.by, pb.bz);
        pb.touched = pb.n_upd = pb.pairs = 0u;
        pb.re_touch = pb.e_na = pb.e_w = false;
        {
            const float* blk = v.pool + (size_t)max(pb.slot, 0) * v.stride;
            const bool have = pb.slot >= 0;
#pragma unroll 4
            for (int j = 0; j < 8; ++j) {
                const int x = lane + 64 * j;
                L.sD[x] = have ? reinterpret_cast<const double*>(blk)[x] : 0.0;
                L.sW[x] = have ? blk[kPoolW + x] : 0.0f;
                if (CM == SC_COLOR_RGBA8) {
                    L.sC[x] = have ? reinterpret_cast<const uint32_t*>(blk + kPoolC)[x] : 0u;
                } else {
                    const double* Cd = reinterpret_cast<const double*>(blk + kPoolC);
                    L.sCf[x] = have ? Cd[x] : 0.0;
                    L.sCf[512 + x] = have ? Cd[512 + x] : 0.0;
                    L.sCf[1024 + x] = have ? Cd[1024 + x] : 0.0;
                }
            }
        }
        wave_lds_sync();
        OpWalk walk;
        walk.mask = cd.mask + (size_t)h * cd.words;
        walk.words = cd.words;
        walk.w = 0;
        walk.m = bcast64(walk.mask[0]);
        int op_c = walk_next(walk);
        if (op_c >= 0) {
            VoxFetch<CM, TV> f0, f1;
            int part_c = 0;
            double qz_c;
            pipe_fetch<CM>(ops[op_c], v, pb, 0, lane, f0, qz_c);
            for (;;) {
                if (!pipe_step<CM>(ops, v, walk, pb, f0, f1, op_c, part_c, qz_c, lane, L)) break;
                if (!pipe_step<CM>(ops, v, walk, pb, f1, f0, op_c, part_c, qz_c, lane, L)) break;
            }
        }
        n_pairs += pb.pairs;
        n_upd += pb.n_upd;
        const int all = (__ballot(pb.re_touch) ? 1 : 0) | (__ballot(pb.e_na) ? 2 : 0) | (__ballot(pb.e_w) ? 4 : 0);
        int slot = pb.slot;
        if (slot < 0 && (all & 1)) slot = vol_insert_wave(v, key, pb.bx, pb.by, pb.bz, lane);
        if (slot >= 0) {
            float* blk = v.pool + (size_t)slot * v.stride;
#pragma unroll 2
            for (int j = 0; j < 8; ++j) {
                if (!((pb.touched >> j) & 1u)) continue;
                const int x = lane + 64 * j;
                reinterpret_cast<double*>(blk)[x] = L.sD[x];
                blk[kPoolW + x] = L.sW[x];
                if (CM == SC_COLOR_RGBA8) {
                    reinterpret_cast<uint32_t*>(blk + kPoolC)[x] = L.sC[x];
                } else {
                    double* Cd = reinterpret_cast<double*>(blk + kPoolC);
                    Cd[x] = L.sCf[x];
                    Cd[512 + x] = L.sCf[512 + x];
                    Cd[1024 + x] = L.sCf[1024 + x];
                }
            }
        }
        const bool wrote = __ballot(pb.touched != 0) != 0;
        n_written += (slot >= 0 && wrote) ? 1u : 0u;
        retire_candidate(cd, v, h, all, lane);
        wave_lds_sync();
    }
    stat_add(cd, 1, worker, n_pairs, lane);
    stat_add(cd, 2, worker, wave_sum(n_upd), lane);
    stat_add(cd, 3, worker, n_written, lane);
}

// ---------------------------------------------------------------------------
// ring-queue voxel pass (schedule compact = 4)
//
// As the pipelined pass, with four changes that cut its instructions per
// voxel test: the touched voxels of an operation collect in a 128-entry LDS
// ring that is updated 64 entries at a time (the pipelined pass updates each
// pair of z-slices separately, so most of its update rounds run half
// empty); the block origin and each lane's column base are computed once per
// (block, operation) instead of once per part; the pixel coordinate uses
// pixel_coord_fast; and the gathers of packed keyframes (pre-quantised
// weight, depth masked to -inf) need no weight test.  The gathers of the
// next step are issued as global (not flat) loads on every step, so the
// wait for the current step's samples leaves them in flight.
// ---------------------------------------------------------------------------

// A block's geometry under one operation: the lane's FP32 camera point of
// voxel (x, y, 0) of its column, and the camera z of the block origin in FP64.
struct RingGeom {
    float base[3];
    double qz;
};

__device__ inline void ring_geom(const OpDesc& o, const VolDev& v, const PipeBlock& pb, int lane, RingGeom& g)
{
    float q[3];
    block_origin(o, v.s, pb.bx, pb.by, pb.bz, q, g.qz);
    const float kx = (float)(lane & 7), ky = (float)(lane >> 3);
#pragma unroll
    for (int r = 0; r < 3; ++r) g.base[r] = (q[r] + kx * o.a[0][r]) + ky * o.a[1][r];
}

typedef __attribute__((address_space(1))) const unsigned char GlobalBytes;
typedef __attribute__((address_space(1))) const float GlobalF32;
typedef __attribute__((address_space(1))) const uint32_t GlobalU32;

// Element `i` of a keyframe array through a 32-bit byte offset from a
// uniform base (a global load with a scalar base and a vector offset).
template <class T, class G>
__device__ inline T kf_load(const void* base, uint32_t i)
{
    return *(G*)((GlobalBytes*)base + i * (uint32_t)sizeof(T));
}

// The lane's voxels in z-slices kz0 .. kz0 + 3 of one (block, operation)
// after their gathers: the camera z (NaN for a voxel outside the image, so
// that its band test fails), the pixel, and the keyframe sample there (pixel
// 0 for a voxel outside the image).
template <int CM>
struct RingFetch {
    float pz[4], wr[4], z[4];
    uint32_t pix[4];
    uint32_t c[4];  // RGBA8 colour at the pixel (RGBA8 mode)
};

// Projections of the lane's voxels in z-slices kz0 .. kz0 + 3 and their
// keyframe gathers: one record per voxel from a packed keyframe, else depth,
// weight and (RGBA8) colour.  The z steps k a_z are the descriptor's
// host-rounded products, equal to the FP32 products of the convention.
template <int CM, bool kPacked>
__device__ inline void ring_fetch(const OpDesc& o, const RingGeom& g, int kz0, RingFetch<CM>& f)
{
    // the operation's constants, read together at the top
    const ProjConst k = proj_const(o);
    float za[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int r = 0; r < 3; ++r) za[j][r] = o.za[kz0 + j][r];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float px = g.base[0] + za[j][0];
        const float py = g.base[1] + za[j][1];
        const float pz = g.base[2] + za[j][2];
        bool in;
        f.pix[j] = pixel_index_fast(k, px, py, pz, in);
        f.pz[j] = in ? pz : __builtin_nanf("");
    }
    if (kPacked) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            // the record's first three words, adjacent: one 12-byte load
            const uint32_t i = 4u * f.pix[j];
            f.z[j] = __uint_as_float(kf_load<uint32_t, GlobalU32>(o.packed, i));
            f.wr[j] = __uint_as_float(kf_load<uint32_t, GlobalU32>(o.packed, i + 1u));
            f.c[j] = kf_load<uint32_t, GlobalU32>(o.packed, i + 2u);
        }
    } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            f.wr[j] = kf_load<float, GlobalF32>(o.weight, f.pix[j]);
            f.z[j] = kf_load<float, GlobalF32>(o.depth, f.pix[j]);
            f.c[j] = (CM == SC_COLOR_RGBA8) ? kf_load<uint32_t, GlobalU32>(o.color, f.pix[j]) : 0u;
        }
    }
}

// Touched decisions of fetched voxels; with kPacked the weight is already
// quantised and the depth of a pixel without weight is -inf.
template <int CM, bool kPacked>
__device__ inline void ring_decide(const RingFetch<CM>& f, float mu, float w[4], bool t[4])
{
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        w[j] = kPacked ? f.wr[j] : qweight(f.wr[j]);
        t[j] = (kPacked || w[j] > 0.0f) && fabsf(f.z[j] - f.pz[j]) <= mu;
    }
}

// The operations of a block in bit order, its mask words held one per lane
// (loaded once per block, so the walk issues no load that a wait could
// confuse with the keyframe gathers in flight).  words <= 64.
struct LaneWalk {
    uint64_t mine;  // mask word `lane`
    uint64_t nz;    // words not yet visited that hold a bit
    uint64_t m;     // remaining bits of the current word
    int w;
};

__device__ inline void lanewalk_init(LaneWalk& k, const uint64_t* mask, int words, int lane)
{
    k.mine = (lane < words) ? mask[lane] : 0ull;
    k.nz = __ballot(k.mine != 0ull);
    k.m = 0ull;
    k.w = 0;
}

__device__ inline int lanewalk_next(LaneWalk& k)
{
    while (k.m == 0ull) {
        if (k.nz == 0ull) return -1;
        k.w = __ffsll((unsigned long long)k.nz) - 1;
        k.nz &= k.nz - 1;
        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)k.mine, k.w);
        const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(k.mine >> 32), k.w);
        k.m = ((uint64_t)hi << 32) | lo;
    }
    const int b = __ffsll((unsigned long long)k.m) - 1;
    k.m &= k.m - 1;
    return k.w * 64 + b;
}

// Ring positions of the queue (uniform): entries [head, tail), modulo 128.
struct Ring {
    uint32_t head, tail;
};

// Updates the n <= 64 oldest queue entries, one per lane (the voxels are
// distinct: they belong to one operation).
template <int CM>
__device__ inline void ring_flush(const OpDesc& op, double qz, Ring& ring, uint32_t n, PipeBlock& pb, int lane,
                                  const PipeLds& L)
{
    wave_lds_sync();
    if ((uint32_t)lane < n) {
        const uint32_t e = (ring.head + (uint32_t)lane) & 127u;
        const int x = L.qvox[e];
        const double pz64 =
            ((qz + (double)(x & 7) * op.az[0]) + (double)((x >> 3) & 7) * op.az[1]) + (double)(x >> 6) * op.az[2];
        const double d = distance(L.qz[e], pz64);
        const float wq = L.qw[e];
        double D = L.sD[x];
        float W = L.sW[x];
        if (CM == SC_COLOR_RGBA8) {
            uint32_t C = L.sC[x];
            pb.e_w |= !update_rgba8_fast(D, W, C, d, wq, L.qc[e], op.sign);
            L.sC[x] = C;
        } else {
            GlobalF32* cp = (GlobalF32*)op.color + 3 * (size_t)L.qc[e];
            const float c[3] = {cp[0], cp[1], cp[2]};
            double C3[3] = {L.sCf[x], L.sCf[512 + x], L.sCf[1024 + x]};
            pb.e_w |= !update_f32(D, W, C3, d, wq, c, op.sign);
            L.sCf[x] = C3[0];
            L.sCf[512 + x] = C3[1];
            L.sCf[1024 + x] = C3[2];
        }
        L.sD[x] = D;
        L.sW[x] = W;
    }
    ring.head += n;
    wave_lds_sync();
}

// One step of the ring pass: geometry and gathers of the next (operation,
// part) first, then the decisions of the current one, its touched voxels
// appended slice by slice to the ring, 64 updated whenever 64 are waiting,
// and the rest when the operation's second part is done.  Returns false
// when the block has no further step.
template <int CM, bool kPacked>
__device__ inline bool ring_step(const OpDesc* __restrict__ ops, const VolDev& v, LaneWalk& walk, PipeBlock& pb,
                                 RingFetch<CM>& cur, RingFetch<CM>& nxt, RingGeom& gc, int& op_c, int& part_c,
                                 int lane, const PipeLds& L, Ring& ring)
{
    int op_n, part_n;
    if (part_c == 0) {
        op_n = op_c;
        part_n = 1;
    } else {
        op_n = lanewalk_next(walk);
        part_n = 0;
    }
    RingGeom gn = gc;
    if (part_n == 0 && op_n >= 0) ring_geom(ops[op_n], v, pb, lane, gn);
    // issued on every step (a block's last step fetches its own part again),
    // so the number of loads in flight is the same on every path
    ring_fetch<CM, kPacked>(ops[op_n >= 0 ? op_n : op_c], gn, 4 * (op_n >= 0 ? part_n : part_c), nxt);
    const OpDesc& op = ops[op_c];
    pb.pairs += (part_c == 0) ? 1u : 0u;
    float w[4];
    bool t[4];
    ring_decide<CM, kPacked>(cur, v.mu, w, t);
    uint64_t bal[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bal[j] = __ballot(t[j]);
    const bool any = ((bal[0] | bal[1]) | (bal[2] | bal[3])) != 0ull;
    pb.pair_any = (part_c == 0) ? any : (pb.pair_any || any);
    if (any && op.sign < 0 && pb.slot < 0) {
        pb.e_na = true;
    } else if (any) {
        if (op.sign > 0) pb.re_touch = true;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            if (bal[j] == 0ull) continue;
            const uint32_t nb = (uint32_t)__popcll(bal[j]);
            pb.touched |= 1u << (part_c * 4 + j);
            pb.n_upd += nb;
            if (t[j]) {
                const uint32_t pos = (ring.tail + lanes_below(bal[j])) & 127u;
                L.qvox[pos] = (uint16_t)(lane + 64 * (part_c * 4 + j));
                L.qw[pos] = w[j];
                L.qz[pos] = cur.z[j];
                L.qc[pos] = (CM == SC_COLOR_RGBA8) ? cur.c[j] : cur.pix[j];
            }
            ring.tail += nb;
            if (ring.tail - ring.head >= 64u) ring_flush<CM>(op, gc.qz, ring, 64u, pb, lane, L);
        }
    }
    if (part_c == 1 && ring.tail != ring.head) ring_flush<CM>(op, gc.qz, ring, ring.tail - ring.head, pb, lane, L);
    if (part_c == 1 && op.rec_mode == 1 && pb.pair_any) {
        // the integration touched the block: lane n_rec remembers the
        // operation, and the block's record appends are issued together
        // when the block is done (no atomic waits while gathers are in
        // flight); a 65th operation flushes the list first
        if (pb.n_rec == 64u) {
            record_flush(ops, pb, lane);
        }
        pb.rec_op = (lane == (int)pb.n_rec) ? op_c : pb.rec_op;
        pb.n_rec += 1u;
    }
    if (op_n < 0) return false;
    op_c = op_n;
    part_c = part_n;
    gc = gn;
    return true;
}

// Persistent voxel pass with the ring queue: one wavefront per block, block
// state in LDS, the same LDS footprint as the pipelined pass.  Its
// PipeBlock counts (touched z-slices, updates) are uniform over the
// wavefront.  kPacked: every
// operation's keyframe carries its packed copy (RGBA8 volumes).
template <int CM, bool kPacked>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void batch_ring_kernel(const OpDesc* __restrict__ ops, VolDev v, CandDev cd)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63;
    const int wave = (int)bcast(threadIdx.x >> 6);
    const PipeLds L = pipe_lds<CM>(smem + (size_t)wave * pipe_wave_bytes<CM>());
    const uint32_t n = cd.counters[4];
    const uint32_t worker = blockIdx.x * (blockDim.x >> 6) + (uint32_t)wave;
    const uint32_t n_workers = gridDim.x * (blockDim.x >> 6);
    RangeCursor cur;
    range_init(cur, worker);
    uint32_t* const cursors = cd.cursors + kCursorSet;  // the voxel pass's set
    uint32_t n_upd = 0, n_pairs = 0, n_written = 0;
    for (;;) {
        const uint32_t i = range_pop(cur, cursors, n, n_workers, lane);
        if (i >= n) break;
        const uint32_t h = bcast(cd.sorted[i]);
        const uint64_t key = bcast64(cd.skey[i]);
        PipeBlock pb;
        pb.slot = (int)bcast((uint32_t)cd.sslot[i]);
        unpack_key(key, pb.bx, pb.by, pb.bz);
        pb.touched = pb.n_upd = pb.pairs = 0u;
        pb.re_touch = pb.e_na = pb.e_w = false;
        pb.n_rec = 0u;
        pb.rec_op = 0;
        // the operation mask first, then the block state into registers;
        // the first operation's gathers are issued before the state goes to
        // LDS, so the two round trips overlap
        LaneWalk walk;
        lanewalk_init(walk, cd.mask + (size_t)h * cd.words, cd.words, lane);
        const float* blk = v.pool + (size_t)max(pb.slot, 0) * v.stride;
        const bool have = pb.slot >= 0;
        double rD[8];
        float rW[8];
        uint32_t rC[8];
        if (CM == SC_COLOR_RGBA8) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int x = lane + 64 * j;
                rD[j] = have ? reinterpret_cast<const double*>(blk)[x] : 0.0;
                rW[j] = have ? blk[kPoolW + x] : 0.0f;
                rC[j] = have ? reinterpret_cast<const uint32_t*>(blk + kPoolC)[x] : 0u;
            }
        } else {
            // FP32 colour: 24 bytes of colour per voxel, written to LDS as read
#pragma unroll 4
            for (int j = 0; j < 8; ++j) {
                const int x = lane + 64 * j;
                L.sD[x] = have ? reinterpret_cast<const double*>(blk)[x] : 0.0;
                L.sW[x] = have ? blk[kPoolW + x] : 0.0f;
                const double* Cd = reinterpret_cast<const double*>(blk + kPoolC);
                L.sCf[x] = have ? Cd[x] : 0.0;
                L.sCf[512 + x] = have ? Cd[512 + x] : 0.0;
                L.sCf[1024 + x] = have ? Cd[1024 + x] : 0.0;
            }
        }
        int op_c = lanewalk_next(walk);
        RingFetch<CM> f0, f1;
        RingGeom gc;
        if (op_c >= 0) {
            ring_geom(ops[op_c], v, pb, lane, gc);
            ring_fetch<CM, kPacked>(ops[op_c], gc, 0, f0);
        }
        if (CM == SC_COLOR_RGBA8) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int x = lane + 64 * j;
                L.sD[x] = rD[j];
                L.sW[x] = rW[j];
                L.sC[x] = rC[j];
            }
        }
        wave_lds_sync();
        if (op_c >= 0) {
            Ring ring;
            ring.head = ring.tail = 0u;
            int part_c = 0;
            for (;;) {
                if (!ring_step<CM, kPacked>(ops, v, walk, pb, f0, f1, gc, op_c, part_c, lane, L, ring)) break;
                if (!ring_step<CM, kPacked>(ops, v, walk, pb, f1, f0, gc, op_c, part_c, lane, L, ring)) break;
            }
        }
        if (pb.n_rec) record_flush(ops, pb, lane);
        n_pairs += pb.pairs;
        n_upd += pb.n_upd;
        const int all = (__ballot(pb.re_touch) ? 1 : 0) | (__ballot(pb.e_na) ? 2 : 0) | (__ballot(pb.e_w) ? 4 : 0);
        int slot = pb.slot;
        if (slot < 0 && (all & 1)) slot = vol_insert_wave(v, key, pb.bx, pb.by, pb.bz, lane);
        if (slot >= 0) {
            float* blk = v.pool + (size_t)slot * v.stride;
#pragma unroll 2
            for (int j = 0; j < 8; ++j) {
                // every slice with a touched voxel is written whole (the
                // voxels the operations left keep the values read above)
                if (!((pb.touched >> j) & 1u)) continue;
                const int x = lane + 64 * j;
                reinterpret_cast<double*>(blk)[x] = L.sD[x];
                blk[kPoolW + x] = L.sW[x];
                if (CM == SC_COLOR_RGBA8) {
                    reinterpret_cast<uint32_t*>(blk + kPoolC)[x] = L.sC[x];
                } else {
                    double* Cd = reinterpret_cast<double*>(blk + kPoolC);
                    Cd[x] = L.sCf[x];
                    Cd[512 + x] = L.sCf[512 + x];
                    Cd[1024 + x] = L.sCf[1024 + x];
                }
            }
        }
        n_written += (slot >= 0 && pb.touched != 0u) ? 1u : 0u;
        retire_candidate(cd, v, h, all, lane);
        wave_lds_sync();
    }
    stat_add(cd, 1, worker, n_pairs, lane);
    stat_add(cd, 2, worker, n_upd, lane);
    stat_add(cd, 3, worker, n_written, lane);
}

// Persistent voxel pass, one workgroup of G = 8 / VPL wavefronts per block
// (wavefront w owns z in [w VPL, (w+1) VPL)).  Wavefront 0 pops and
// allocates; the others learn the results through LDS after a barrier.  The
// wavefront index is made uniform with readfirstlane, so every branch on it
// is a scalar branch.
template <int CM, int VPL>
__global__ __launch_bounds__(512) void batch_main_group_kernel(const OpDesc* __restrict__ ops, VolDev v, CandDev cd)
{
    __shared__ uint32_t s_item;
    __shared__ int s_slot;
    __shared__ int s_flags;
    const int lane = threadIdx.x & 63;
    const int wave = (int)bcast(threadIdx.x >> 6);
    const int kz0 = wave * VPL;
    const uint32_t n = cd.counters[4];
    WorkCursor cur;  // used by wavefront 0
    cursor_init(cur, blockIdx.x);
    uint32_t n_upd = 0, n_pairs = 0, n_written = 0;
    for (;;) {
        if (wave == 0) {
            const uint32_t it = cursor_pop(cur, cd.counters + 5, gridDim.x, lane);
            s_item = it;
            s_flags = 0;
        }
        __syncthreads();
        const uint32_t i = bcast(s_item);
        if (i >= n) break;
        const uint32_t h = bcast(cd.sorted[i]);
        const uint64_t key = bcast64(cd.skey[i]);
        int slot = (int)bcast((uint32_t)cd.sslot[i]);
        int bx, by, bz;
        unpack_key(key, bx, by, bz);
        LaneVox<CM, VPL> st;
        if (slot >= 0)
            load_vox<CM, VPL>(st, v.pool + (size_t)slot * v.stride, lane, kz0);
        else
            zero_vox<CM, VPL>(st);
        uint32_t touched = 0;
        bool re_touch = false, e_na = false, e_w = false;
        for (int w = 0; w < cd.words; ++w) {
            uint64_t m = bcast64(cd.mask[(size_t)h * cd.words + w]);
            n_pairs += __popcll(m);
            while (m) {
                const int b = __ffsll((unsigned long long)m) - 1;
                m &= m - 1;
                apply_op<CM, VPL>(ops[w * 64 + b], v, bx, by, bz, lane, kz0, slot >= 0, st, touched, re_touch, e_na,
                                  e_w, n_upd);
            }
        }
        const int f = (__ballot(re_touch) ? 1 : 0) | (__ballot(e_na) ? 2 : 0) | (__ballot(e_w) ? 4 : 0) |
                      (__ballot(touched != 0) ? 8 : 0);
        if (f) atomicOr(&s_flags, f);
        __syncthreads();
        const int all = (int)bcast((uint32_t)s_flags);
        if (slot < 0 && (all & 1)) {
            if (wave == 0) {
                const int sl = vol_insert_wave(v, key, bx, by, bz, lane);
                s_slot = sl;
            }
            __syncthreads();
            slot = (int)bcast((uint32_t)s_slot);
        }
        if (slot >= 0) store_vox<CM, VPL>(st, v.pool + (size_t)slot * v.stride, lane, kz0, touched);
        n_written += (slot >= 0 && (all & 8)) ? 1u : 0u;
        if (wave == 0) retire_candidate(cd, v, h, all, lane);
        __syncthreads();
    }
    stat_add(cd, 2, blockIdx.x * (blockDim.x >> 6) + (uint32_t)wave, wave_sum(n_upd), lane);
    if (wave == 0) {
        stat_add(cd, 1, blockIdx.x, n_pairs, lane);
        stat_add(cd, 3, blockIdx.x, n_written, lane);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static bool schedule_ok(const sc_schedule& s)
{
    if (s.vpl != 8 && s.vpl != 4 && s.vpl != 2 && s.vpl != 1) return false;
    if (s.compact < 0 || s.compact > 4) return false;
    if (s.compact && (s.vpl != 8 || (s.waves_per_wg != 1 && s.waves_per_wg != 2 && s.waves_per_wg != 4)))
        return false;
    return s.wgs_per_cu >= 1 && s.wgs_per_cu <= 32;
}

// Candidate stage: clears the per-batch counters, generates the candidate
// blocks with their operation masks, and orders them by operation count.
static void launch_candidates(sc_volume* vol, bool from_cells, hipStream_t s)
{
    const int n_bins = vol->p.max_batch_ops + 1;
    // first the recorded candidates (their kernel also clears the batch's
    // counters), then the frustum tiles
    // 16 workgroups per operation: about one recorded key per thread
    cand_record_kernel<<<dim3(16, (unsigned)std::min(vol->p.max_batch_ops, 256)), 256, 0, s>>>(
        vol->d_ops, vol->d_hdr, vol->dev, vol->cand, n_bins);
    const int threads = CandCfg<kTileBatch, kCellBatch>::threads;
    if (from_cells) {
        cand_batch_kernel<true><<<vol->n_cu * vol->cand_wgs[1], threads, 0, s>>>(vol->d_ops, vol->d_hdr, vol->dev,
                                                                                 vol->cand);
        cand_big_kernel<<<vol->n_cu, threads, 0, s>>>(vol->d_ops, vol->d_hdr, vol->dev, vol->cand);
    } else
        cand_batch_kernel<false><<<vol->n_cu * vol->cand_wgs[0], threads, 0, s>>>(vol->d_ops, vol->d_hdr, vol->dev,
                                                                                  vol->cand);
    // two workgroups per CU: fewer of them meet on the global bins of the
    // common operation counts (28 -> 22 us and 40 -> 37 us against four)
    hist_kernel<<<vol->n_cu * 2, 256, 0, s>>>(vol->cand, n_bins);
    scan_kernel<<<1, 1024, 0, s>>>(vol->cand, n_bins);
    scatter_kernel<<<vol->n_cu * 2, 256, 0, s>>>(vol->cand, vol->dev, n_bins);
}

// The persistent voxel pass with schedule `sch`; `packed`: every operation
// of the chunk has a packed keyframe (RGBA8 volumes).
static void launch_voxel_pass(sc_volume* vol, const sc_schedule& sch, bool packed, hipStream_t s)
{
    const bool rgba = vol->p.color_mode == SC_COLOR_RGBA8;
    const int grid = vol->n_cu * sch.wgs_per_cu;
    if (sch.compact) {
        const int threads = 64 * sch.waves_per_wg;
        const size_t w = sch.waves_per_wg;
        if (sch.compact == 4) {
            if (rgba && packed)
                batch_ring_kernel<SC_COLOR_RGBA8, true><<<grid, threads, w * pipe_wave_bytes<SC_COLOR_RGBA8>(), s>>>(
                    vol->d_ops, vol->dev, vol->cand);
            else if (rgba)
                batch_ring_kernel<SC_COLOR_RGBA8, false><<<grid, threads, w * pipe_wave_bytes<SC_COLOR_RGBA8>(), s>>>(
                    vol->d_ops, vol->dev, vol->cand);
            else
                batch_ring_kernel<SC_COLOR_F32, false><<<grid, threads, w * pipe_wave_bytes<SC_COLOR_F32>(), s>>>(
                    vol->d_ops, vol->dev, vol->cand);
        } else if (sch.compact == 3) {
            if (rgba)
                batch_pipe_kernel<SC_COLOR_RGBA8><<<grid, threads, w * pipe_wave_bytes<SC_COLOR_RGBA8>(), s>>>(
                    vol->d_ops, vol->dev, vol->cand);
            else
                batch_pipe_kernel<SC_COLOR_F32><<<grid, threads, w * pipe_wave_bytes<SC_COLOR_F32>(), s>>>(
                    vol->d_ops, vol->dev, vol->cand);
        } else if (sch.compact == 1) {
            if (rgba)
                batch_compact_kernel<SC_COLOR_RGBA8, 8><<<grid, threads, w * compact_wave_bytes<SC_COLOR_RGBA8, 8>(),
                                                          s>>>(vol->d_ops, vol->dev, vol->cand);
            else
                batch_compact_kernel<SC_COLOR_F32, 8><<<grid, threads, w * compact_wave_bytes<SC_COLOR_F32, 8>(),
                                                        s>>>(vol->d_ops, vol->dev, vol->cand);
        } else {
            if (rgba)
                batch_compact_kernel<SC_COLOR_RGBA8, 4><<<grid, threads, w * compact_wave_bytes<SC_COLOR_RGBA8, 4>(),
                                                          s>>>(vol->d_ops, vol->dev, vol->cand);
            else
                batch_compact_kernel<SC_COLOR_F32, 4><<<grid, threads, w * compact_wave_bytes<SC_COLOR_F32, 4>(),
                                                        s>>>(vol->d_ops, vol->dev, vol->cand);
        }
        return;
    }
    const int threads = (sch.vpl == 8) ? 256 : 64 * (8 / sch.vpl);
    switch (sch.vpl) {
    case 8:
        if (rgba)
            batch_main_wave_kernel<SC_COLOR_RGBA8><<<grid, threads, 0, s>>>(vol->d_ops, vol->dev, vol->cand);
        else
            batch_main_wave_kernel<SC_COLOR_F32><<<grid, threads, 0, s>>>(vol->d_ops, vol->dev, vol->cand);
        break;
    case 4:
        if (rgba)
            batch_main_group_kernel<SC_COLOR_RGBA8, 4><<<grid, threads, 0, s>>>(vol->d_ops, vol->dev, vol->cand);
        else
            batch_main_group_kernel<SC_COLOR_F32, 4><<<grid, threads, 0, s>>>(vol->d_ops, vol->dev, vol->cand);
        break;
    case 2:
        if (rgba)
            batch_main_group_kernel<SC_COLOR_RGBA8, 2><<<grid, threads, 0, s>>>(vol->d_ops, vol->dev, vol->cand);
        else
            batch_main_group_kernel<SC_COLOR_F32, 2><<<grid, threads, 0, s>>>(vol->d_ops, vol->dev, vol->cand);
        break;
    default:
        if (rgba)
            batch_main_group_kernel<SC_COLOR_RGBA8, 1><<<grid, threads, 0, s>>>(vol->d_ops, vol->dev, vol->cand);
        else
            batch_main_group_kernel<SC_COLOR_F32, 1><<<grid, threads, 0, s>>>(vol->d_ops, vol->dev, vol->cand);
        break;
    }
}

static int sched_index(const sc_schedule& s)
{
    const int v = (s.vpl == 8) ? 0 : (s.vpl == 4) ? 1 : (s.vpl == 2) ? 2 : 3;
    return v;
}

// Captures the work that `launch` enqueues on the private capture stream and
// instantiates it.  Returns null on failure (after clearing HIP's last error).
template <class F>
static hipGraphExec_t capture(sc_volume* vol, F&& launch)
{
    hipStream_t cs = vol->cap_stream;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    launch(cs);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(cs, &g) != hipSuccess || !g) {
        (void)hipGetLastError();
        return nullptr;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return ex;
}

// Returns the voxel-pass graph for the current schedule and keyframe form,
// capturing it on first use.
static bool graphs_for(sc_volume* vol, bool packed, hipGraphExec_t& main)
{
    const int vi = sched_index(vol->sched) + (packed ? 4 : 0);
    const int key = (vol->sched.compact * 8 + vol->sched.waves_per_wg) * 64 + vol->sched.wgs_per_cu;
    if (vol->graph_main[vi] && vol->graph_keys[vi] != key) {
        (void)hipGraphExecDestroy(vol->graph_main[vi]);
        vol->graph_main[vi] = nullptr;
    }
    if (!vol->graph_main[vi]) {
        const sc_schedule sch = vol->sched;
        vol->graph_main[vi] = capture(vol, [&](hipStream_t cs) { launch_voxel_pass(vol, sch, packed, cs); });
        vol->graph_keys[vi] = key;
    }
    main = vol->graph_main[vi];
    return main != nullptr;
}

// Copies one chunk of staged operations to the device and runs the captured
// candidate stage over them: afterwards the candidate table holds each
// candidate block's operation mask and the work list orders the blocks by
// operation count, heaviest first.
sc_status run_candidates(sc_volume* vol, const OpDesc* ops, int n_ops, const sc_intrinsics* in, hipStream_t s)
{
    BatchHdr* hdr = stage_hdr(vol);
    hdr->n_ops = n_ops;
    hdr->tiles_x = (in->width + kTileBatch - 1) / kTileBatch;
    hdr->tiles_y = (in->height + kTileBatch - 1) / kTileBatch;
    hdr->n_tile_ops = 0;
    // the frustum-cell operations read cell depth ranges when every one of
    // them has a packed keyframe
    bool from_cells = true;
    for (int o = 0; o < n_ops; ++o)
        if (ops[o].rec_mode != 2) {
            hdr->tile_ops[hdr->n_tile_ops++] = (int16_t)o;
            from_cells = from_cells && ops[o].cells != nullptr;
        }
    const size_t hdr_bytes = offsetof(BatchHdr, tile_ops) + sizeof(int16_t) * (size_t)std::max(hdr->n_tile_ops, 1);
    if (hipMemcpyAsync(vol->d_ops, ops, sizeof(OpDesc) * n_ops, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(vol->d_hdr, hdr, hdr_bytes, hipMemcpyHostToDevice, s) != hipSuccess)
        return SC_EDEVICE;
    // the staging buffer may be refilled once these copies have run
    const sc_status st = stage_end(vol, s);
    if (st != SC_OK) return st;
    hipGraphExec_t& pre = vol->graph_pre[from_cells ? 1 : 0];
    if (!pre) pre = capture(vol, [&](hipStream_t cs) { launch_candidates(vol, from_cells, cs); });
    if (!pre || hipGraphLaunch(pre, s) != hipSuccess) return SC_EDEVICE;
    return SC_OK;
}

// Runs one chunk of staged operations: the candidate stage, then the voxel
// pass.  With timing enabled, an event pair brackets the voxel pass on the
// stream.
static sc_status run_chunk(sc_volume* vol, const OpDesc* ops, int n_ops, const sc_intrinsics* in, hipStream_t s)
{
    sc_status st = run_candidates(vol, ops, n_ops, in, s);
    if (st != SC_OK) return st;
    st = stream_in_batch(vol, s);
    if (st != SC_OK) return st;
    bool packed = vol->p.color_mode == SC_COLOR_RGBA8;
    for (int i = 0; i < n_ops && packed; ++i) packed = ops[i].packed != nullptr;
    hipGraphExec_t main = nullptr;
    if (!graphs_for(vol, packed, main)) return SC_EDEVICE;
    const bool timed = vol->timing_n < vol->timing_cap;
    if (timed && hipEventRecord(vol->timing_ev[2 * vol->timing_n], s) != hipSuccess) return SC_EDEVICE;
    if (hipGraphLaunch(main, s) != hipSuccess) return SC_EDEVICE;
    if (timed) {
        if (hipEventRecord(vol->timing_ev[2 * vol->timing_n + 1], s) != hipSuccess) return SC_EDEVICE;
        vol->timing_n++;
    }
    return SC_OK;
}

static bool intr_valid(const sc_intrinsics* in)
{
    return in && in->width > 0 && in->height > 0 && in->fx > 0.0f && in->fy > 0.0f && in->width <= 16384 &&
           in->height <= 16384;
}

sc_status batch_update(sc_volume* vol, const sc_keyframe* kfs, int32_t n_kf, const sc_intrinsics* in,
                       const sc_pose* T_int, const sc_pose* T_new, const int32_t* order, int32_t ns, hipStream_t s)
{
    const int cap = vol->p.max_batch_ops;
    // processing order: every de-integration, then every re-integration
    int total = 2 * ns, done = 0;
    while (done < total) {
        const int cnt = std::min(cap, total - done);
        OpDesc* ops = stage_begin(vol);
        if (!ops) return SC_EDEVICE;
        for (int j = 0; j < cnt; ++j) {
            const int g = done + j;
            const int k = order[g < ns ? g : g - ns];
            if (g < ns) {
                make_op(vol, &kfs[k], in, &T_int[k], -1, k, &ops[j]);
                rec_for_deintegration(vol, &kfs[k], in, &T_int[k], &ops[j]);
            } else {
                make_op(vol, &kfs[k], in, &T_new[k], +1, k, &ops[j]);
                rec_for_integration(vol, &kfs[k], in, &T_new[k], vol->sched.compact == 4, &ops[j]);
            }
        }
        const sc_status st = run_chunk(vol, ops, cnt, in, s);
        if (st != SC_OK) {
            rec_commit(vol);
            return st;
        }
        done += cnt;
    }
    rec_commit(vol);
    return SC_OK;
}

}  // namespace sc

using namespace sc;

extern "C" {

// A schedule is usable on a volume if it is valid and its LDS fits in 64 KiB
// per workgroup.
// The autotuner's results of this process (see sc_autotune).
static std::mutex g_tune_mu;
static std::map<std::string, std::pair<sc_schedule, float>> g_tune;

static bool schedule_fits(const sc_volume* vol, const sc_schedule& s)
{
    if (!schedule_ok(s)) return false;
    if (!s.compact) return true;
    const bool rgba = vol->p.color_mode == SC_COLOR_RGBA8;
    const int per = (s.compact == 1)   ? (rgba ? compact_wave_bytes<SC_COLOR_RGBA8, 8>() : compact_wave_bytes<SC_COLOR_F32, 8>())
                    : (s.compact == 2) ? (rgba ? compact_wave_bytes<SC_COLOR_RGBA8, 4>() : compact_wave_bytes<SC_COLOR_F32, 4>())
                                       : (rgba ? pipe_wave_bytes<SC_COLOR_RGBA8>() : pipe_wave_bytes<SC_COLOR_F32>());
    return s.waves_per_wg * per <= 65536;
}

sc_status sc_set_schedule(sc_volume* vol, const sc_schedule* sched)
{
    if (!vol || !sched || !schedule_fits(vol, *sched)) return SC_EINVAL;
    vol->sched = *sched;
    if (!sched->compact) vol->sched.waves_per_wg = (vol->sched.vpl == 8) ? 4 : 8 / vol->sched.vpl;
    return SC_OK;
}

sc_status sc_batch_timing(sc_volume* vol, int32_t capacity)
{
    if (!vol || capacity < 0 || capacity > (1 << 20)) return SC_EINVAL;
    if (hipDeviceSynchronize() != hipSuccess) return SC_EDEVICE;
    for (int i = 0; i < 2 * vol->timing_cap; ++i) (void)hipEventDestroy(vol->timing_ev[i]);
    delete[] vol->timing_ev;
    vol->timing_ev = nullptr;
    vol->timing_cap = vol->timing_n = 0;
    if (capacity == 0) return SC_OK;
    vol->timing_ev = new (std::nothrow) hipEvent_t[2 * capacity];
    if (!vol->timing_ev) return SC_ENOMEM;
    for (int i = 0; i < 2 * capacity; ++i)
        if (hipEventCreate(&vol->timing_ev[i]) != hipSuccess) return SC_EDEVICE;
    vol->timing_cap = capacity;
    return SC_OK;
}

sc_status sc_batch_timing_read(sc_volume* vol, float* ms, int32_t* n)
{
    if (!vol || !n || (vol->timing_n > 0 && !ms)) return SC_EINVAL;
    for (int i = 0; i < vol->timing_n; ++i) {
        if (hipEventSynchronize(vol->timing_ev[2 * i + 1]) != hipSuccess) return SC_EDEVICE;
        if (hipEventElapsedTime(&ms[i], vol->timing_ev[2 * i], vol->timing_ev[2 * i + 1]) != hipSuccess)
            return SC_EDEVICE;
    }
    *n = vol->timing_n;
    return SC_OK;
}

sc_status sc_volume_stats(sc_volume* vol, void* stream, int64_t* stats)
{
    if (!vol || !stats) return SC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int64_t slots[4 * kStatSlots];
    if (hipMemcpyAsync(slots, vol->cand.stats, sizeof(slots), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SC_EDEVICE;
    for (int k = 0; k < 4; ++k) {
        stats[k] = 0;
        for (int j = 0; j < kStatSlots; ++j) stats[k] += slots[k * kStatSlots + j];
    }
    return SC_OK;
}

sc_status sc_get_schedule(sc_volume* vol, sc_schedule* sched)
{
    if (!vol || !sched) return SC_EINVAL;
    *sched = vol->sched;
    return SC_OK;
}

sc_status reintegrate_batch(sc_volume* vol, const sc_keyframe* kfs, int32_t n_kf, const sc_intrinsics* intr,
                            sc_pose* T_integrated, const sc_pose* T_new, int32_t m, int32_t mode,
                            int32_t* selected_out, int32_t* n_selected, void* stream)
{
    if (!vol || !kfs || n_kf <= 0 || !T_integrated || !T_new || !intr_valid(intr)) return SC_EINVAL;
    for (int i = 0; i < n_kf; ++i)
        if (!keyframe_ok(&kfs[i])) return SC_EINVAL;
    std::vector<int32_t> order(n_kf);
    const int32_t ns = sc_select(T_integrated, T_new, n_kf, m, mode, order.data(), nullptr);
    if (ns < 0) return ns;
    const sc_status st = batch_update(vol, kfs, n_kf, intr, T_integrated, T_new, order.data(), ns, (hipStream_t)stream);
    if (st != SC_OK) return st;
    if (hipGetLastError() != hipSuccess) return SC_EDEVICE;
    for (int j = 0; j < ns; ++j) T_integrated[order[j]] = T_new[order[j]];
    if (selected_out) memcpy(selected_out, order.data(), sizeof(int32_t) * ns);
    if (n_selected) *n_selected = ns;
    return SC_OK;
}

sc_status tsdf_integrate_batch(sc_volume* vol, const sc_keyframe* kfs, int32_t n_kf, const sc_intrinsics* intr,
                               const sc_pose* T, void* stream)
{
    if (!vol || !kfs || n_kf <= 0 || !T || !intr_valid(intr)) return SC_EINVAL;
    for (int i = 0; i < n_kf; ++i)
        if (!keyframe_ok(&kfs[i])) return SC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int cap = vol->p.max_batch_ops;
    for (int done = 0; done < n_kf;) {
        const int cnt = std::min(cap, n_kf - done);
        OpDesc* ops = stage_begin(vol);
        if (!ops) return SC_EDEVICE;
        for (int j = 0; j < cnt; ++j) {
            const int k = done + j;
            make_op(vol, &kfs[k], intr, &T[k], +1, k, &ops[j]);
            rec_for_integration(vol, &kfs[k], intr, &T[k], vol->sched.compact == 4, &ops[j]);
        }
        const sc_status st = run_chunk(vol, ops, cnt, intr, s);
        rec_commit(vol);
        if (st != SC_OK) return st;
        done += cnt;
    }
    return hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
}

// Copies the state of `src` into `dst` (same parameters), on stream s.
static sc_status clone_state(sc_volume* dst, sc_volume* src, hipStream_t s)
{
    int64_t nb = 0, nt = 0;
    sc_status st = sc_volume_query(src, s, &nb, nullptr);
    if (st == SC_OK) st = sc_volume_query(dst, s, &nt, nullptr);
    if (st != SC_OK) return st;
    const VolDev& a = src->dev;
    const VolDev& b = dst->dev;
    bool ok = true;
    ok &= hipMemcpyAsync(b.keys, a.keys, sizeof(uint64_t) * src->p.n_buckets, hipMemcpyDeviceToDevice, s) == hipSuccess;
    ok &= hipMemcpyAsync(b.vals, a.vals, sizeof(int32_t) * src->p.n_buckets, hipMemcpyDeviceToDevice, s) == hipSuccess;
    if (nb > 0) {
        ok &= hipMemcpyAsync(b.slot_keys, a.slot_keys, sizeof(uint64_t) * nb, hipMemcpyDeviceToDevice, s) == hipSuccess;
        ok &= hipMemcpyAsync(b.pool, a.pool, sizeof(float) * (size_t)a.stride * nb, hipMemcpyDeviceToDevice, s) ==
              hipSuccess;
    }
    // blocks [nb, nt) of dst hold data from an earlier trial: clear them
    if (nt > nb) fill_u32(reinterpret_cast<uint32_t*>(b.pool + (size_t)b.stride * nb), 0u, (size_t)b.stride * (nt - nb), s);
    ok &= hipMemcpyAsync(b.n_blocks, a.n_blocks, sizeof(uint32_t), hipMemcpyDeviceToDevice, s) == hipSuccess;
    ok &= hipMemcpyAsync(b.err, a.err, sizeof(int32_t), hipMemcpyDeviceToDevice, s) == hipSuccess;
    return ok ? SC_OK : SC_EDEVICE;
}

sc_status sc_autotune(sc_volume* vol, const sc_keyframe* kfs, int32_t n_kf, const sc_intrinsics* intr,
                      const sc_pose* T_integrated, const sc_pose* T_new, int32_t m, int32_t mode, sc_schedule* best,
                      float* best_ms, void* stream)
{
    if (!vol || !kfs || n_kf <= 0 || !T_integrated || !T_new || !intr_valid(intr)) return SC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    std::vector<int32_t> order(n_kf);
    const int32_t ns = sc_select(T_integrated, T_new, n_kf, m, mode, order.data(), nullptr);
    if (ns < 0) return ns;
    // tuning cache: one entry per (architecture, image size, operations per
    // chunk, keyframe form, volume parameters); a hit sets the schedule
    // without timing anything
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, vol->device) != hipSuccess) return SC_EDEVICE;
    bool packed = vol->p.color_mode == SC_COLOR_RGBA8;
    for (int j = 0; j < ns && packed; ++j) packed = kfs[order[j]].packed != nullptr;
    char key[256];
    snprintf(key, sizeof(key), "%s|%dx%d|%d|%d|%g|%g|%d|%d|%lld", prop.gcnArchName, intr->width, intr->height,
             std::min(2 * ns, vol->p.max_batch_ops), (int)packed, (double)vol->p.voxel_size, (double)vol->p.trunc,
             vol->p.color_mode, vol->p.max_batch_ops, (long long)vol->p.n_buckets);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            vol->sched = it->second.first;
            if (best) *best = it->second.first;
            if (best_ms) *best_ms = it->second.second;
            return SC_OK;
        }
    }
    sc_volume* tmp = nullptr;
    sc_status st = sc_volume_create(&vol->p, &tmp);
    if (st != SC_OK) return st;
    static const sc_schedule cands[] = {{8, 4, 2, 0}, {8, 4, 4, 0}, {8, 4, 8, 0}, {4, 2, 8, 0}, {4, 2, 16, 0},
                                        {2, 4, 4, 0}, {2, 4, 8, 0}, {1, 8, 2, 0}, {1, 8, 4, 0}, {8, 4, 2, 1},
                                        {8, 4, 4, 1}, {8, 2, 4, 1},  {8, 2, 8, 1},  {8, 1, 16, 1}, {8, 4, 4, 2},
                                        {8, 2, 8, 2}, {8, 1, 16, 2}, {8, 4, 4, 3},  {8, 2, 8, 3},  {8, 1, 16, 3},
                                        {8, 4, 4, 4}, {8, 2, 8, 4},  {8, 1, 16, 4}};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        sc_volume_destroy(tmp);
        return SC_EDEVICE;
    }
    float bms = 3.0e38f;
    sc_schedule bs = vol->sched;
    for (const sc_schedule& c : cands) {
        if (!schedule_fits(vol, c)) continue;
        tmp->sched = c;
        float tbest = 3.0e38f;
        for (int rep = 0; rep < 3 && st == SC_OK; ++rep) {
            st = clone_state(tmp, vol, s);
            if (st != SC_OK) break;
            if (hipEventRecord(e0, s) != hipSuccess) st = SC_EDEVICE;
            if (st == SC_OK) st = batch_update(tmp, kfs, n_kf, intr, T_integrated, T_new, order.data(), ns, s);
            if (st == SC_OK && hipEventRecord(e1, s) != hipSuccess) st = SC_EDEVICE;
            if (st == SC_OK && hipEventSynchronize(e1) != hipSuccess) st = SC_EDEVICE;
            float ms = 0.0f;
            if (st == SC_OK && hipEventElapsedTime(&ms, e0, e1) == hipSuccess && rep > 0) tbest = std::min(tbest, ms);
        }
        if (st != SC_OK) break;
        int64_t nb = 0;
        int32_t err = 0;
        st = sc_volume_query(tmp, s, &nb, &err);
        if (st != SC_OK) break;
        if (err != SC_OK) {
            st = err;
            break;
        }
        if (tbest < bms) {
            bms = tbest;
            bs = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    sc_volume_destroy(tmp);
    if (st != SC_OK) return st;
    vol->sched = bs;
    if (best) *best = bs;
    if (best_ms) *best_ms = bms;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[key] = std::make_pair(bs, bms);
    }
    return SC_OK;
}

void sc_autotune_clear(void)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.clear();
}

}  // extern "C"
