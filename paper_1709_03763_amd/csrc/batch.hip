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
#include <string.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "common.hpp"
#include "internal.hpp"
#include "kernels.hpp"

namespace sc {

__global__ void batch_init_kernel(CandDev cd, int n_bins)
{
    for (int i = threadIdx.x; i < 8; i += blockDim.x) cd.counters[4 + i] = 0u;
    for (int i = threadIdx.x; i < n_bins; i += blockDim.x) cd.bins[i] = 0u;
}

__global__ __launch_bounds__(256) void cand_batch_kernel(const OpDesc* __restrict__ ops, const BatchHdr* hdr,
                                                         VolDev v, CandDev cd)
{
    __shared__ uint64_t lds[kLdsSet];
    const int tiles = hdr->tiles_x * hdr->tiles_y;
    const int items = hdr->n_ops * tiles;
    for (int it = blockIdx.x; it < items; it += gridDim.x) {
        const int o = it / tiles;
        const int tile = it - o * tiles;
        const int ty = tile / hdr->tiles_x;
        const int tx = tile - ty * hdr->tiles_x;
        cand_tile(ops[o], v, cd, cd.counters + 4, tx, ty, o, lds);
        __syncthreads();
    }
}

__device__ inline int mask_count(const CandDev& cd, uint32_t h)
{
    int c = 0;
    for (int w = 0; w < cd.words; ++w) c += __popcll(cd.mask[(size_t)h * cd.words + w]);
    return c;
}

__global__ void hist_kernel(CandDev cd)
{
    const uint32_t n = min(cd.counters[4], cd.cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        atomicAdd(cd.bins + mask_count(cd, cd.list[i]), 1u);
}

// Exclusive scan in descending operation count: offset[c] = #blocks with more
// than c operations.  One workgroup; n_bins <= 4097.
__global__ __launch_bounds__(1024) void scan_kernel(CandDev cd, int n_bins)
{
    __shared__ uint32_t part[1024];
    const int tid = threadIdx.x;
    if (tid == 0) cd.stats[0] += min(cd.counters[4], cd.cap);
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
}

__global__ void scatter_kernel(CandDev cd)
{
    const uint32_t n = min(cd.counters[4], cd.cap);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t h = cd.list[i];
        const uint32_t pos = atomicAdd(cd.bins + mask_count(cd, h), 1u);
        cd.sorted[pos] = h;
    }
}

// Voxel state of one lane: VPL voxels along z of the lane's (x, y) column.
template <int CM, int VPL>
struct LaneVox {
    float D[VPL], W[VPL];
    uint32_t C[VPL];       // RGBA8
    double Cf[3][VPL];     // FP32-colour mode (held in FP64)
};

template <int CM, int VPL>
__device__ inline void load_vox(LaneVox<CM, VPL>& s, const float* blk, int lane, int kz0)
{
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
        const int i = lane + 64 * (kz0 + j);
        s.D[j] = blk[i];
        s.W[j] = blk[512 + i];
        if (CM == SC_COLOR_RGBA8) {
            s.C[j] = reinterpret_cast<const uint32_t*>(blk)[1024 + i];
        } else {
            const double* Cd = reinterpret_cast<const double*>(blk + 1024);
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
        s.D[j] = 0.0f;
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
        blk[i] = s.D[j];
        blk[512 + i] = s.W[j];
        if (CM == SC_COLOR_RGBA8) {
            reinterpret_cast<uint32_t*>(blk)[1024 + i] = s.C[j];
        } else {
            double* Cd = reinterpret_cast<double*>(blk + 1024);
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
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
        const float fz = (float)(kz0 + j);
        const float px = base[0] + fz * op.a[2][0];
        const float py = base[1] + fz * op.a[2][1];
        const float pz = base[2] + fz * op.a[2][2];
        int pix;
        float w, z;
        if (!touch(op, v.mu, px, py, pz, pix, w, z)) continue;
        const float d = distance(z, bz64 + (double)(kz0 + j) * op.az[2]);
        if (op.sign < 0 && !allocated) {
            e_notalloc = true;
            continue;
        }
        if (op.sign > 0) re_touch = true;
        touched |= 1u << j;
        ++n_upd;
        if (CM == SC_COLOR_RGBA8) {
            const uint32_t c = __ldg(reinterpret_cast<const uint32_t*>(op.color) + pix);
            e_weight |= !update_rgba8(s.D[j], s.W[j], s.C[j], d, w, c, op.sign);
        } else {
            const float* cp = reinterpret_cast<const float*>(op.color) + 3 * pix;
            const float c[3] = {__ldg(cp), __ldg(cp + 1), __ldg(cp + 2)};
            double C3[3] = {s.Cf[0][j], s.Cf[1][j], s.Cf[2][j]};
            e_weight |= !update_f32(s.D[j], s.W[j], C3, d, w, c, op.sign);
            s.Cf[0][j] = C3[0];
            s.Cf[1][j] = C3[1];
            s.Cf[2][j] = C3[2];
        }
    }
}

// Finishes a block: allocation flags, errors and clearing the candidate
// entry; executed by every lane of one wavefront (branch-free).
__device__ inline void retire_candidate(const CandDev& cd, const VolDev& v, uint32_t h, int all, int lane)
{
    if (all & 2) set_error(v.err, SC_ENOTALLOC);
    if (all & 4) set_error(v.err, SC_EWEIGHT);
    cd.mask[(size_t)h * cd.words + min(lane, cd.words - 1)] = 0ull;  // words <= 64
    cd.keys[h] = kKeyEmpty;
}

// Persistent voxel pass, one wavefront per block (eight voxels per lane,
// lane = x + 8 y, z in a loop); the wavefronts of a workgroup are independent.
template <int CM>
__global__ __launch_bounds__(256) void batch_main_wave_kernel(const OpDesc* __restrict__ ops, VolDev v, CandDev cd)
{
    constexpr int VPL = 8;
    const int lane = threadIdx.x & 63;
    const uint32_t n = min(cd.counters[4], cd.cap);
    uint32_t n_upd = 0, n_pairs = 0, n_written = 0;
    for (;;) {
        const uint32_t i = wave_fetch_add1(cd.counters + 5, lane);
        if (i >= n) break;
        const uint32_t h = bcast(cd.sorted[i]);
        const uint64_t key = bcast64(cd.keys[h]);
        int bx, by, bz;
        unpack_key(key, bx, by, bz);
        int slot = (int)bcast((uint32_t)vol_find(v, key, bx, by, bz));
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
    atomicAdd(cd.stats + 1, (unsigned long long)(lane == 0 ? n_pairs : 0u));
    atomicAdd(cd.stats + 2, (unsigned long long)n_upd);
    atomicAdd(cd.stats + 3, (unsigned long long)(lane == 0 ? n_written : 0u));
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
    const uint32_t n = min(cd.counters[4], cd.cap);
    uint32_t n_upd = 0, n_pairs = 0, n_written = 0;
    for (;;) {
        if (wave == 0) {
            const uint32_t it = wave_fetch_add1(cd.counters + 5, lane);
            s_item = it;
            s_flags = 0;
        }
        __syncthreads();
        const uint32_t i = bcast(s_item);
        if (i >= n) break;
        const uint32_t h = bcast(cd.sorted[i]);
        const uint64_t key = bcast64(cd.keys[h]);
        int bx, by, bz;
        unpack_key(key, bx, by, bz);
        int slot = (int)bcast((uint32_t)vol_find(v, key, bx, by, bz));
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
    atomicAdd(cd.stats + 2, (unsigned long long)n_upd);
    if (wave == 0) {
        atomicAdd(cd.stats + 1, (unsigned long long)(lane == 0 ? n_pairs : 0u));
        atomicAdd(cd.stats + 3, (unsigned long long)(lane == 0 ? n_written : 0u));
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

static bool schedule_ok(const sc_schedule& s)
{
    if (s.vpl != 8 && s.vpl != 4 && s.vpl != 2 && s.vpl != 1) return false;
    return s.wgs_per_cu >= 1 && s.wgs_per_cu <= 32;
}

static void launch_sequence(sc_volume* vol, const sc_schedule& sch, hipStream_t s, bool events)
{
    const int n_bins = vol->p.max_batch_ops + 1;
    batch_init_kernel<<<1, 1024, 0, s>>>(vol->cand, n_bins);
    cand_batch_kernel<<<vol->n_cu * 16, 256, 0, s>>>(vol->d_ops, vol->d_hdr, vol->dev, vol->cand);
    hist_kernel<<<vol->n_cu * 4, 256, 0, s>>>(vol->cand);
    scan_kernel<<<1, 1024, 0, s>>>(vol->cand, n_bins);
    scatter_kernel<<<vol->n_cu * 4, 256, 0, s>>>(vol->cand);
    if (events) (void)hipEventRecordWithFlags(vol->tev[0], s, hipEventRecordExternal);
    const bool rgba = vol->p.color_mode == SC_COLOR_RGBA8;
    const int grid = vol->n_cu * sch.wgs_per_cu;
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
    if (events) (void)hipEventRecordWithFlags(vol->tev[1], s, hipEventRecordExternal);
}

static int sched_index(const sc_schedule& s)
{
    const int v = (s.vpl == 8) ? 0 : (s.vpl == 4) ? 1 : (s.vpl == 2) ? 2 : 3;
    return v;
}

// Returns the graph for the current schedule, capturing it on first use.  The
// capture records two events around the voxel pass; their nodes are kept so
// that each launch can record per-launch timing events instead.
static hipGraphExec_t graph_for(sc_volume* vol)
{
    const int vi = sched_index(vol->sched);
    const int key = vol->sched.waves_per_wg * 64 + vol->sched.wgs_per_cu;
    if (vol->graph[vi][0] && vol->graph_keys[vi] == key) return vol->graph[vi][0];
    if (vol->graph[vi][0]) {
        (void)hipGraphExecDestroy(vol->graph[vi][0]);
        vol->graph[vi][0] = nullptr;
    }
    if (vol->graph_src[vi]) {
        (void)hipGraphDestroy(vol->graph_src[vi]);
        vol->graph_src[vi] = nullptr;
    }
    hipStream_t cs = vol->cap_stream;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
    launch_sequence(vol, vol->sched, cs, true);
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(cs, &g) != hipSuccess || !g) return nullptr;
    // locate the two event-record nodes (in capture order)
    size_t nn = 0;
    if (hipGraphGetNodes(g, nullptr, &nn) != hipSuccess) return nullptr;
    std::vector<hipGraphNode_t> nodes(nn);
    if (nn && hipGraphGetNodes(g, nodes.data(), &nn) != hipSuccess) return nullptr;
    vol->ev_node[vi][0] = vol->ev_node[vi][1] = nullptr;
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType ty;
        if (hipGraphNodeGetType(nd, &ty) != hipSuccess || ty != hipGraphNodeTypeEventRecord) continue;
        hipEvent_t e = nullptr;
        if (hipGraphEventRecordNodeGetEvent(nd, &e) != hipSuccess) continue;
        if (e == vol->tev[0]) vol->ev_node[vi][0] = nd;
        if (e == vol->tev[1]) vol->ev_node[vi][1] = nd;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return nullptr;
    }
    vol->graph[vi][0] = ex;
    vol->graph_src[vi] = g;
    vol->graph_keys[vi] = key;
    return ex;
}

// Stages and runs one chunk of operations (ops already in vol->h_ops).
static sc_status run_chunk(sc_volume* vol, int n_ops, const sc_intrinsics* in, hipStream_t s)
{
    vol->h_hdr->n_ops = n_ops;
    vol->h_hdr->tiles_x = (in->width + kTile - 1) / kTile;
    vol->h_hdr->tiles_y = (in->height + kTile - 1) / kTile;
    if (hipMemcpyAsync(vol->d_ops, vol->h_ops, sizeof(OpDesc) * n_ops, hipMemcpyHostToDevice, s) != hipSuccess ||
        hipMemcpyAsync(vol->d_hdr, vol->h_hdr, sizeof(BatchHdr), hipMemcpyHostToDevice, s) != hipSuccess)
        return SC_EDEVICE;
    hipGraphExec_t g = graph_for(vol);
    if (!g) return SC_EDEVICE;
    const int vi = sched_index(vol->sched);
    if (vol->ev_node[vi][0] && vol->ev_node[vi][1]) {
        hipEvent_t e0 = vol->tev[0], e1 = vol->tev[1];
        if (vol->timing_n < vol->timing_cap) {
            e0 = vol->timing_ev[2 * vol->timing_n];
            e1 = vol->timing_ev[2 * vol->timing_n + 1];
            vol->timing_n++;
        }
        if (hipGraphExecEventRecordNodeSetEvent(g, vol->ev_node[vi][0], e0) != hipSuccess ||
            hipGraphExecEventRecordNodeSetEvent(g, vol->ev_node[vi][1], e1) != hipSuccess)
            return SC_EDEVICE;
    }
    if (hipGraphLaunch(g, s) != hipSuccess) return SC_EDEVICE;
    // the staging buffers may be rewritten only after the copies have run
    if (hipEventRecord(vol->staged, s) != hipSuccess) return SC_EDEVICE;
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
        if (hipEventSynchronize(vol->staged) != hipSuccess) return SC_EDEVICE;
        for (int j = 0; j < cnt; ++j) {
            const int g = done + j;
            const int k = order[g < ns ? g : g - ns];
            if (g < ns)
                make_op(vol, &kfs[k], in, &T_int[k], -1, k, &vol->h_ops[j]);
            else
                make_op(vol, &kfs[k], in, &T_new[k], +1, k, &vol->h_ops[j]);
        }
        const sc_status st = run_chunk(vol, cnt, in, s);
        if (st != SC_OK) return st;
        done += cnt;
    }
    return SC_OK;
}

}  // namespace sc

using namespace sc;

extern "C" {

sc_status sc_set_schedule(sc_volume* vol, const sc_schedule* sched)
{
    if (!vol || !sched || !schedule_ok(*sched)) return SC_EINVAL;
    vol->sched = *sched;
    vol->sched.waves_per_wg = (vol->sched.vpl == 8) ? 4 : 8 / vol->sched.vpl;
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
    if (hipMemcpyAsync(stats, vol->cand.stats, sizeof(int64_t) * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return SC_EDEVICE;
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
    for (int j = 0; j < ns; ++j) T_integrated[order[j]] = T_new[order[j]];
    if (selected_out) memcpy(selected_out, order.data(), sizeof(int32_t) * ns);
    if (n_selected) *n_selected = ns;
    return SC_OK;
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
    sc_volume* tmp = nullptr;
    sc_status st = sc_volume_create(&vol->p, &tmp);
    if (st != SC_OK) return st;
    static const sc_schedule cands[] = {{8, 4, 2}, {8, 4, 4}, {8, 4, 8}, {4, 2, 8}, {4, 2, 16},
                                        {2, 4, 4}, {2, 4, 8}, {1, 8, 2}, {1, 8, 4}};
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        sc_volume_destroy(tmp);
        return SC_EDEVICE;
    }
    float bms = 3.0e38f;
    sc_schedule bs = vol->sched;
    for (const sc_schedule& c : cands) {
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
    return SC_OK;
}

}  // extern "C"
