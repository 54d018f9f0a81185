// Voxel-hashed TSDF volume (Sec. 3, "SDF volume"): lifecycle, block
// allocation, and the plain per-keyframe integration (running weighted
// average) and de-integration (Sec. 4.3, Eq. 2).
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <unordered_map>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "internal.hpp"

namespace sc {

// ---------------------------------------------------------------------------
// small kernels
// ---------------------------------------------------------------------------

__global__ void fill_u64_kernel(uint64_t* p, uint64_t v, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

void fill_u64(uint64_t* p, uint64_t v, size_t n, hipStream_t s)
{
    if (n == 0) return;
    const int grid = (int)std::min<size_t>((n + 255) / 256, 8192);
    fill_u64_kernel<<<grid, 256, 0, s>>>(p, v, n);
}

void fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s)
{
    if (n == 0) return;
    const int grid = (int)std::min<size_t>((n + 255) / 256, 8192);
    fill_u32_kernel<<<grid, 256, 0, s>>>(p, v, n);
}

// ---------------------------------------------------------------------------
// hash_alloc: wavefront ballot deduplication (one round per distinct key),
// CAS insert, LDS-staged queue of new blocks and one pool reservation per
// workgroup
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void hash_alloc_kernel(VolDev v, const int32_t* xyz, int64_t n)
{
    __shared__ uint32_t q_bucket[256];
    __shared__ uint32_t q_n;
    __shared__ uint32_t q_base;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    if (tid == 0) q_n = 0;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + tid;
    const bool have = i < n;
    int bx = 0, by = 0, bz = 0;
    uint64_t key = kKeyEmpty;
    if (have) {
        bx = xyz[3 * i];
        by = xyz[3 * i + 1];
        bz = xyz[3 * i + 2];
        key = pack_key(bx, by, bz);
    }
    __syncthreads();
    // one leader per distinct key within each wavefront, by ballot: the
    // lowest lane still undecided takes its key, every lane holding that key
    // is decided; one round per distinct key of the wavefront
    bool leader = false;
    uint64_t todo = __ballot(have);
    while (todo) {
        const int l = __ffsll((unsigned long long)todo) - 1;
        const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)key, l);
        const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(key >> 32), l);
        const uint64_t k = ((uint64_t)hi << 32) | lo;
        leader = leader || lane == l;
        todo &= ~__ballot(key == k);
    }
    if (leader) {
        uint32_t h = hash_block(bx, by, bz) & v.bucket_mask;
        bool done = false;
        for (uint32_t probe = 0; probe <= v.bucket_mask; ++probe) {
            const uint64_t old = atomicCAS((unsigned long long*)(v.keys + h), (unsigned long long)kKeyEmpty,
                                           (unsigned long long)key);
            if (old == kKeyEmpty) {
                const uint32_t q = atomicAdd(&q_n, 1u);
                q_bucket[q] = h;
                done = true;
                break;
            }
            if (old == key) {
                done = true;
                break;
            }
            h = (h + 1) & v.bucket_mask;
        }
        if (!done) set_error(v.err, SC_EHASHFULL);
    }
    __syncthreads();
    if (tid == 0) q_base = q_n ? atomicAdd(v.n_blocks, q_n) : 0u;
    __syncthreads();
    for (uint32_t j = tid; j < q_n; j += blockDim.x) {
        const uint32_t slot = q_base + j;
        const uint32_t h = q_bucket[j];
        if (slot >= (uint32_t)v.max_blocks) {
            v.vals[h] = -1;
            set_error(v.err, SC_EPOOLFULL);
        } else {
            v.slot_keys[slot] = v.keys[h];
            v.vals[h] = (int)slot;
        }
    }
}

__global__ void hash_lookup_kernel(VolDev v, const int32_t* xyz, int64_t n, int32_t* slots)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int bx = xyz[3 * i], by = xyz[3 * i + 1], bz = xyz[3 * i + 2];
    slots[i] = vol_find(v, pack_key(bx, by, bz), bx, by, bz);
}

// ---------------------------------------------------------------------------
// plain path: one keyframe operation
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void cand_plain_kernel(OpDesc op, VolDev v, CandDev cd, int parity)
{
    __shared__ uint64_t lds[CandCfg<kTilePlain, kCellPlain>::lds_set];
    __shared__ uint16_t idx[CandCfg<kTilePlain, kCellPlain>::lds_set];
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
        cd.counters[1 - parity] = 0u;
        cd.counters[2 + (1 - parity)] = 0u;
    }
    cand_tile<kTilePlain, kCellPlain>(op, v, cd, cd.counters + parity, blockIdx.x, blockIdx.y, -1, lds, idx);
}

// Applies one operation to one candidate block with one wavefront, eight
// voxels per lane (lane = x + 8 y, loop over z), coalesced in brick order.
template <int CM>
__device__ void block_one_op(const OpDesc& op, const VolDev& v, uint64_t key, int lane)
{
    int bx, by, bz;
    unpack_key(key, bx, by, bz);
    float q[3];
    double qz;
    block_origin(op, v.s, bx, by, bz, q, qz);
    const float kx = (float)(lane & 7), ky = (float)(lane >> 3);
    float base[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) base[r] = (q[r] + kx * op.a[0][r]) + ky * op.a[1][r];
    const double bz64 = (qz + (double)(lane & 7) * op.az[0]) + (double)(lane >> 3) * op.az[1];
    VoxHits<CM, 8> hv;
    test_voxels<CM, 8>(op, v.mu, base, 0, hv);
    const uint32_t tmask = hv.hit;
    if (__ballot(tmask != 0) == 0) return;
    if (op.rec_mode == 1 && lane == 0) {
        // the integration's touched-block record: one append by one lane
        const uint32_t pos = atomicAdd(op.rec_count, 1u);
        if (pos < (uint32_t)op.rec_cap) op.rec_keys[pos] = key;
    }
    const int slot = (op.sign > 0) ? vol_insert_wave(v, key, bx, by, bz, lane) : (int)bcast((uint32_t)vol_find(v, key, bx, by, bz));
    if (slot < 0) {
        if (op.sign < 0) set_error(v.err, SC_ENOTALLOC);
        return;
    }
    float* blk = v.pool + (size_t)slot * v.stride;
    bool bad = false;
#pragma unroll
    for (int kz = 0; kz < 8; ++kz) {
        if (!((tmask >> kz) & 1u)) continue;
        const int i = lane + 64 * kz;
        double* Dp = reinterpret_cast<double*>(blk);
        double D = Dp[i];
        float W = blk[kPoolW + i];
        const double dd = distance(hv.z[kz], bz64 + (double)kz * op.az[2]);
        if (CM == SC_COLOR_RGBA8) {
            uint32_t* Cp = reinterpret_cast<uint32_t*>(blk + kPoolC);
            uint32_t C = Cp[i];
            bad |= !update_rgba8(D, W, C, dd, hv.w[kz], hv.c[kz], op.sign);
            Cp[i] = C;
        } else {
            double* Cd = reinterpret_cast<double*>(blk + kPoolC);
            double C[3] = {Cd[i], Cd[512 + i], Cd[1024 + i]};
            const float* cp = reinterpret_cast<const float*>(op.color) + 3 * hv.pix[kz];
            const float c[3] = {cp[0], cp[1], cp[2]};
            bad |= !update_f32(D, W, C, dd, hv.w[kz], c, op.sign);
            Cd[i] = C[0];
            Cd[512 + i] = C[1];
            Cd[1024 + i] = C[2];
        }
        Dp[i] = D;
        blk[kPoolW + i] = W;
    }
    if (__ballot(bad) != 0) set_error(v.err, SC_EWEIGHT);
}

// Persistent: each wavefront pops candidate blocks until the list is
// exhausted (no lane-dependent branches in the loop).
template <int CM>
__global__ __launch_bounds__(256) void update_plain_kernel(OpDesc op, VolDev v, CandDev cd, int parity)
{
    const int lane = threadIdx.x & 63;
    const uint32_t n = min(cd.counters[parity], cd.cap);
    WorkCursor cur;
    cursor_init(cur, blockIdx.x * (blockDim.x >> 6) + bcast(threadIdx.x >> 6));
    const uint32_t n_workers = gridDim.x * (blockDim.x >> 6);
    for (;;) {
        const uint32_t i = cursor_pop(cur, cd.counters + 2 + parity, n_workers, lane);
        if (i >= n) break;
        const uint32_t h = bcast(cd.list[i]);
        const uint64_t key = bcast64(cd.keys[h]);
        block_one_op<CM>(op, v, key, lane);
        cd.keys[h] = kKeyEmpty;
    }
}

// Writes imported block records into their pool slots (D widened to FP64;
// FP32 colour widened to the FP64 planes).
__global__ void import_kernel(VolDev v, const int32_t* __restrict__ slots, int64_t n, const float* __restrict__ D,
                              const float* __restrict__ W, const void* __restrict__ C)
{
    const int64_t b = blockIdx.x;
    if (b >= n) return;
    const int slot = slots[b];
    if (slot < 0) return;
    float* blk = v.pool + (size_t)slot * v.stride;
    for (int i = threadIdx.x; i < kBlockVox; i += blockDim.x) {
        const size_t g = (size_t)b * kBlockVox + i;
        reinterpret_cast<double*>(blk)[i] = D ? (double)D[g] : 0.0;
        blk[kPoolW + i] = W ? W[g] : 0.0f;
        if (v.color_mode == SC_COLOR_RGBA8) {
            reinterpret_cast<uint32_t*>(blk + kPoolC)[i] = C ? reinterpret_cast<const uint32_t*>(C)[g] : 0u;
        } else {
            const float* Cf = reinterpret_cast<const float*>(C) + (size_t)b * 3 * kBlockVox;
            double* Cd = reinterpret_cast<double*>(blk + kPoolC);
            Cd[i] = C ? (double)Cf[i] : 0.0;
            Cd[512 + i] = C ? (double)Cf[512 + i] : 0.0;
            Cd[1024 + i] = C ? (double)Cf[1024 + i] : 0.0;
        }
    }
}

__global__ void export_kernel(VolDev v, int64_t n, int32_t* xyz, float* D, float* W, void* C)
{
    const int64_t b = blockIdx.x;
    if (b >= n) return;
    const float* blk = v.pool + (size_t)b * v.stride;
    for (int i = threadIdx.x; i < kBlockVox; i += blockDim.x) {
        if (D) D[b * kBlockVox + i] = (float)reinterpret_cast<const double*>(blk)[i];
        if (W) W[b * kBlockVox + i] = blk[kPoolW + i];
        if (C) {
            if (v.color_mode == SC_COLOR_RGBA8) {
                reinterpret_cast<uint32_t*>(C)[b * kBlockVox + i] = reinterpret_cast<const uint32_t*>(blk + kPoolC)[i];
            } else {
                const double* Cd = reinterpret_cast<const double*>(blk + kPoolC);
                float* Cf = reinterpret_cast<float*>(C) + b * 3 * kBlockVox;
                Cf[i] = (float)Cd[i];
                Cf[512 + i] = (float)Cd[512 + i];
                Cf[1024 + i] = (float)Cd[1024 + i];
            }
        }
    }
    if (xyz && threadIdx.x == 0) {
        int x, y, z;
        unpack_key(v.slot_keys[b], x, y, z);
        xyz[3 * b] = x;
        xyz[3 * b + 1] = y;
        xyz[3 * b + 2] = z;
    }
}

// Packed record of a pixel: the quantised weight, and the depth only where
// that weight is positive (-inf elsewhere, which fails every band test).
__global__ void pack_kernel(const float* depth, const float* weight, const uint32_t* color, uint4* out, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float w = qweight(weight[i]);
        const float z = (w > 0.0f) ? depth[i] : -__builtin_inff();
        out[i] = make_uint4(__float_as_uint(z), __float_as_uint(w), color[i], 0u);
    }
}

// Depth range {zmin, zmax} of the valid pixels (positive quantised weight,
// 0 < depth < 1e30) of each 4 x 4 cell, {+inf, -inf} without one: the
// candidate stage's per-cell test without reading the pixels.
__global__ void pack_cells_kernel(const float* depth, const float* weight, float2* cells, int width, int height,
                                  int cells_w, int64_t n_cells)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n_cells;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int cy = (int)(c / cells_w), cx = (int)(c - (int64_t)cy * cells_w);
        float zmin = __builtin_inff(), zmax = -__builtin_inff();
        for (int q = 0; q < 16; ++q) {
            const int u = 4 * cx + (q & 3), v = 4 * cy + (q >> 2);
            if (u >= width || v >= height) continue;
            const int64_t pix = (int64_t)v * width + u;
            const float z = depth[pix];
            if (qweight(weight[pix]) > 0.0f && z > 0.0f && z < 1.0e30f) {
                zmin = fminf(zmin, z);
                zmax = fmaxf(zmax, z);
            }
        }
        cells[c] = make_float2(zmin, zmax);
    }
}

// ---------------------------------------------------------------------------
// host helpers
// ---------------------------------------------------------------------------

void make_op(const sc_volume* vol, const sc_keyframe* kf, const sc_intrinsics* in, const sc_pose* T, int sign,
             int kf_index, OpDesc* op)
{
    memset(op, 0, sizeof(*op));
    op->depth = kf->depth;
    op->weight = kf->weight;
    op->color = kf->color;
    op->packed = (vol->p.color_mode == SC_COLOR_RGBA8) ? reinterpret_cast<const uint4*>(kf->packed) : nullptr;
    // the cell depth ranges follow the width x height records
    op->cells = op->packed ? reinterpret_cast<const float2*>(op->packed + (size_t)in->width * in->height) : nullptr;
    op->width = in->width;
    op->height = in->height;
    op->fx = in->fx;
    op->fy = in->fy;
    op->cx = in->cx;
    op->cy = in->cy;
    memcpy(op->R, T->R, sizeof(op->R));
    memcpy(op->t, T->t, sizeof(op->t));
    const double s = (double)vol->p.voxel_size;
    for (int c = 0; c < 3; ++c) {
        for (int r = 0; r < 3; ++r) op->a[c][r] = (float)(s * T->R[3 * c + r]);
        op->az[c] = s * T->R[3 * c + 2];
    }
    for (int k = 0; k < 8; ++k)
        for (int r = 0; r < 3; ++r) op->za[k][r] = (float)k * op->a[2][r];  // one FP32 rounding, as on the device
    op->wl = (float)(in->width - 1);
    op->hl = (float)(in->height - 1);
    op->wf = (float)in->width;
    // one extra 2^-21 covers the rounding of the bound itself to FP32
    op->kin_u = (float)(0.5 - (2.0 + fabs((double)in->cx)) * 0x1p-21);
    op->kin_v = (float)(0.5 - (2.0 + fabs((double)in->cy)) * 0x1p-21);
    op->sign = sign;
    op->kf = kf_index;
}

// Host staging of operation descriptors, double-buffered: a buffer is
// refilled only after the copy that last read it has run, so the host can
// prepare the next chunk while the device still works on the previous one.
OpDesc* stage_begin(sc_volume* vol)
{
    if (hipEventSynchronize(vol->staged[vol->stage]) != hipSuccess) return nullptr;
    return vol->h_ops + (size_t)vol->stage * vol->p.max_batch_ops;
}

BatchHdr* stage_hdr(sc_volume* vol) { return vol->h_hdr + vol->stage; }

// Records the current buffer's copies on `s` and switches buffers.
sc_status stage_end(sc_volume* vol, hipStream_t s)
{
    if (hipEventRecord(vol->staged[vol->stage], s) != hipSuccess) return SC_EDEVICE;
    vol->stage ^= 1;
    return SC_OK;
}

static bool intr_ok(const sc_intrinsics* in)
{
    return in && in->width > 0 && in->height > 0 && in->fx > 0.0f && in->fy > 0.0f && in->width <= 16384 &&
           in->height <= 16384;
}

bool keyframe_ok(const sc_keyframe* kf)
{
    return kf && kf->depth && kf->weight && kf->color && ((uintptr_t)kf->packed & 15u) == 0u;
}

// ---------------------------------------------------------------------------
// touched-block records
//
// A keyframe integrated at a pose touches a set of blocks that depends only
// on the keyframe and the pose; de-integrating it at that pose (Eq. 2)
// touches exactly the same set.  Integrations therefore append the blocks
// they touch to a record keyed by (keyframe buffers, intrinsics, pose), and
// a later de-integration of the same key takes the record as its candidate
// blocks instead of generating frustum candidates.  A record is dropped when
// as many de-integrations as integrations of its key have been applied, on
// reset and on import; a record that overflowed its capacity is ignored on
// the device (frustum candidates are generated instead).
// ---------------------------------------------------------------------------

}  // namespace sc

struct RecordRegistry {
    struct Entry {
        int slot;
        int refs;
    };
    std::unordered_map<std::string, Entry> map;
    std::vector<int> free_slots;
    std::vector<int> pending;  // slots released by de-integrations of the call in flight
    uint64_t* d_keys = nullptr;
    uint32_t* d_count = nullptr;
    int slots = 0, cap = 0;
    bool failed = false;
};

namespace sc {

constexpr int kRecSlots = 1024;   // records held at once
constexpr int kRecCap = 16384;    // blocks per record
constexpr int kRecCountStride = 32;  // one record counter per 128 bytes, so appends to different records do not meet

static std::string rec_fingerprint(const sc_keyframe* kf, const sc_intrinsics* in, const sc_pose* T)
{
    std::string f;
    f.reserve(4 * sizeof(void*) + sizeof(sc_intrinsics) + sizeof(sc_pose));
    const void* ptrs[4] = {kf->depth, kf->weight, kf->color, kf->packed};
    f.append(reinterpret_cast<const char*>(ptrs), sizeof(ptrs));
    f.append(reinterpret_cast<const char*>(in), sizeof(*in));
    f.append(reinterpret_cast<const char*>(T), sizeof(*T));
    return f;
}

static bool rec_ready(sc_volume* vol)
{
    if (!vol->rec) vol->rec = new (std::nothrow) RecordRegistry();
    RecordRegistry* r = vol->rec;
    if (!r || r->failed) return false;
    if (r->d_keys) return true;
    const int cap = (int)std::min<int64_t>(kRecCap, vol->p.max_blocks);
    if (hipMalloc(&r->d_keys, sizeof(uint64_t) * (size_t)kRecSlots * cap) != hipSuccess ||
        hipMalloc(&r->d_count, kRecCountStride * sizeof(uint32_t) * kRecSlots) != hipSuccess) {
        (void)hipGetLastError();
        hipFree(r->d_keys);
        r->d_keys = nullptr;
        r->failed = true;
        return false;
    }
    r->slots = kRecSlots;
    r->cap = cap;
    r->free_slots.clear();
    for (int i = kRecSlots - 1; i >= 0; --i) r->free_slots.push_back(i);
    return true;
}

void rec_clear(sc_volume* vol)
{
    RecordRegistry* r = vol->rec;
    if (!r || !r->d_keys) return;
    r->map.clear();
    r->pending.clear();
    r->free_slots.clear();
    for (int i = r->slots - 1; i >= 0; --i) r->free_slots.push_back(i);
}

void rec_destroy(sc_volume* vol)
{
    RecordRegistry* r = vol->rec;
    if (!r) return;
    hipFree(r->d_keys);
    hipFree(r->d_count);
    delete r;
    vol->rec = nullptr;
}

// An integration of kf at T: an existing record of the key only gains a
// reference (the same keyframe at the same pose touches the same blocks, so
// the record still holds them); otherwise, with `records` (the kernel that
// will run appends the touched blocks), the op fills a fresh record (rec_mode
// 1; its count is cleared on the device before the pass).
void rec_for_integration(sc_volume* vol, const sc_keyframe* kf, const sc_intrinsics* in, const sc_pose* T,
                         bool records, OpDesc* op)
{
    if (!rec_ready(vol)) return;
    RecordRegistry* r = vol->rec;
    const std::string f = rec_fingerprint(kf, in, T);
    auto it = r->map.find(f);
    if (!records) {
        if (it != r->map.end()) it->second.refs += 1;
        return;
    }
    if (it != r->map.end()) {
        // the same keyframe at the same pose touches the same blocks: the
        // record stands as it is (so a slot being recorded is always a fresh
        // one, never one a de-integration of the same batch reads)
        it->second.refs += 1;
        return;
    }
    if (r->free_slots.empty()) return;
    const int slot = r->free_slots.back();
    r->free_slots.pop_back();
    r->map.emplace(f, RecordRegistry::Entry{slot, 1});
    op->rec_keys = r->d_keys + (size_t)slot * r->cap;
    op->rec_count = r->d_count + (size_t)kRecCountStride * slot;
    op->rec_cap = r->cap;
    op->rec_mode = 1;
}

// A de-integration of kf at T: takes the key's record when there is one
// (rec_mode 2) and releases one reference to it; the slot becomes free once
// the call's work is enqueued (rec_commit).
void rec_for_deintegration(sc_volume* vol, const sc_keyframe* kf, const sc_intrinsics* in, const sc_pose* T,
                           OpDesc* op)
{
    RecordRegistry* r = vol->rec;
    if (!r || !r->d_keys) return;
    auto it = r->map.find(rec_fingerprint(kf, in, T));
    if (it == r->map.end()) return;
    const int slot = it->second.slot;
    op->rec_keys = r->d_keys + (size_t)slot * r->cap;
    op->rec_count = r->d_count + (size_t)kRecCountStride * slot;
    op->rec_cap = r->cap;
    op->rec_mode = 2;
    if (--it->second.refs == 0) {
        r->pending.push_back(slot);
        r->map.erase(it);
    }
}

// Frees the slots released during a call, once all its work is enqueued:
// later work on the stream runs after it.
void rec_commit(sc_volume* vol)
{
    RecordRegistry* r = vol->rec;
    if (!r) return;
    for (int slot : r->pending) r->free_slots.push_back(slot);
    r->pending.clear();
}

sc_status plain_op(sc_volume* vol, const sc_keyframe* kf, const sc_intrinsics* in, const sc_pose* T, int sign,
                   hipStream_t s)
{
    if (!vol || !keyframe_ok(kf) || !intr_ok(in) || !T) return SC_EINVAL;
    OpDesc op;
    make_op(vol, kf, in, T, sign, 0, &op);
    if (sign > 0) {
        rec_for_integration(vol, kf, in, T, true, &op);
        if (op.rec_mode == 1) fill_u32(op.rec_count, 0u, 1, s);
    } else {
        // the plain de-integration generates its own candidates: only the
        // reference is released
        OpDesc tmp = op;
        rec_for_deintegration(vol, kf, in, T, &tmp);
    }
    const int p = vol->parity;
    vol->parity ^= 1;
    dim3 tiles((in->width + kTilePlain - 1) / kTilePlain, (in->height + kTilePlain - 1) / kTilePlain);
    cand_plain_kernel<<<tiles, CandCfg<kTilePlain, kCellPlain>::threads, 0, s>>>(op, vol->dev, vol->cand, p);
    const sc_status sst = stream_in_plain(vol, p, s);
    if (sst != SC_OK) {
        rec_commit(vol);
        return sst;
    }
    const int grid = vol->n_cu * vol->plain_wgs;  // resident at once: the first items are assigned statically
    if (vol->p.color_mode == SC_COLOR_RGBA8)
        update_plain_kernel<SC_COLOR_RGBA8><<<grid, 256, 0, s>>>(op, vol->dev, vol->cand, p);
    else
        update_plain_kernel<SC_COLOR_F32><<<grid, 256, 0, s>>>(op, vol->dev, vol->cand, p);
    rec_commit(vol);
    return hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
}

}  // namespace sc

using namespace sc;

#define HIP_TRY(x)                                \
    do {                                          \
        if ((x) != hipSuccess) return SC_EDEVICE; \
    } while (0)

extern "C" {

const char* sc_version(void) { return "scsurf 0.1 (gfx950)"; }

sc_status sc_volume_create(const sc_volume_params* p, sc_volume** out)
{
    if (!out) return SC_EINVAL;
    *out = nullptr;
    if (!p || !(p->voxel_size > 0.0f) || !(p->trunc > 0.0f) || !is_pow2(p->n_buckets) || p->n_buckets > (1ll << 30) ||
        p->max_blocks <= 0 || p->max_blocks > (1ll << 30) ||
        (p->color_mode != SC_COLOR_RGBA8 && p->color_mode != SC_COLOR_F32) || p->max_batch_ops <= 0 ||
        p->max_batch_ops > kMaxBatchOps)
        return SC_EINVAL;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return SC_ENOLIB;
    sc_volume* vol = new (std::nothrow) sc_volume();
    if (!vol) return SC_ENOMEM;
    memset(vol, 0, sizeof(*vol));
    vol->p = *p;
    vol->device = dev;
    vol->n_cu = prop.multiProcessorCount;
    vol->cand_wgs[0] = cand_batch_resident_wgs(false);
    vol->cand_wgs[1] = cand_batch_resident_wgs(true);
    {
        int n = 0;
        const hipError_t e = (p->color_mode == SC_COLOR_RGBA8)
                                 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, update_plain_kernel<SC_COLOR_RGBA8>,
                                                                               256, 0)
                                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, update_plain_kernel<SC_COLOR_F32>,
                                                                               256, 0);
        vol->plain_wgs = (e == hipSuccess) ? std::max(1, std::min(n, 4)) : 1;
    }
    // default voxel-pass schedule: RGBA8 volumes take the ring pass (two
    // wavefronts per workgroup, eight workgroups per CU), the fastest measured
    // on a 400-operation update of 200 keyframes at 640x480, which also keeps
    // touched-block records for later de-integrations; FP32-colour volumes
    // the per-lane pass
    vol->sched.vpl = 8;
    if (p->color_mode == SC_COLOR_RGBA8) {
        vol->sched.waves_per_wg = 2;
        vol->sched.wgs_per_cu = 8;
        vol->sched.compact = 4;
    } else {
        vol->sched.waves_per_wg = 4;
        vol->sched.wgs_per_cu = 4;
    }
    VolDev& d = vol->dev;
    d.bucket_mask = (uint32_t)(p->n_buckets - 1);
    d.max_blocks = (int32_t)p->max_blocks;
    d.stride = (p->color_mode == SC_COLOR_RGBA8) ? 4 * kBlockVox : 9 * kBlockVox;
    d.color_mode = p->color_mode;
    d.s = p->voxel_size;
    d.mu = p->trunc;
    // candidate table: as many buckets as the volume, capped; one mask word per 64 batch operations
    uint64_t cb = (uint64_t)std::min<int64_t>(std::max<int64_t>(p->n_buckets, 1 << 16), 1 << 23);
    vol->cand_buckets = (uint32_t)cb;
    CandDev& c = vol->cand;
    c.mask_bits = (uint32_t)(cb - 1);
    c.cap = (uint32_t)(cb / 2);
    c.words = (p->max_batch_ops + 63) / 64;
    bool ok = true;
    ok &= hipMalloc(&d.keys, sizeof(uint64_t) * p->n_buckets) == hipSuccess;
    ok &= hipMalloc(&d.vals, sizeof(int32_t) * p->n_buckets) == hipSuccess;
    ok &= hipMalloc(&d.slot_keys, sizeof(uint64_t) * p->max_blocks) == hipSuccess;
    ok &= hipMalloc(&d.pool, sizeof(float) * (size_t)d.stride * p->max_blocks) == hipSuccess;
    ok &= hipMalloc(&d.n_blocks, 64) == hipSuccess;
    ok &= hipMalloc(&d.err, 64) == hipSuccess;
    ok &= hipMalloc(&c.keys, sizeof(uint64_t) * cb) == hipSuccess;
    ok &= hipMalloc(&c.mask, sizeof(uint64_t) * cb * c.words) == hipSuccess;
    ok &= hipMalloc(&c.list, sizeof(uint32_t) * c.cap) == hipSuccess;
    ok &= hipMalloc(&c.sorted, sizeof(uint32_t) * cb) == hipSuccess;  // every bucket may be a candidate
    ok &= hipMalloc(&c.skey, sizeof(uint64_t) * cb) == hipSuccess;
    ok &= hipMalloc(&c.sslot, sizeof(int32_t) * cb) == hipSuccess;
    ok &= hipMalloc(&c.counters, 64 * sizeof(uint32_t)) == hipSuccess;
    ok &= hipMalloc(&c.bins, sizeof(uint32_t) * (kMaxBatchOps + 2)) == hipSuccess;
    ok &= hipMalloc(&c.cursors, sizeof(uint32_t) * 2 * kCursorSet) == hipSuccess;
    ok &= hipMalloc(&c.big, sizeof(uint32_t) * (kBigCap + 1)) == hipSuccess;
    ok &= hipMalloc(&c.stats, sizeof(unsigned long long) * 4 * kStatSlots) == hipSuccess;
    ok &= hipMalloc(&vol->d_ops, sizeof(OpDesc) * p->max_batch_ops) == hipSuccess;
    ok &= hipMalloc(&vol->adj_acc, sizeof(double) * 3 * kAdjChunk) == hipSuccess;
    ok &= hipHostMalloc((void**)&vol->h_ops, 2 * sizeof(OpDesc) * p->max_batch_ops, hipHostMallocDefault) ==
          hipSuccess;
    ok &= hipMalloc(&vol->d_hdr, sizeof(BatchHdr)) == hipSuccess;
    ok &= hipHostMalloc((void**)&vol->h_hdr, 2 * sizeof(BatchHdr), hipHostMallocDefault) == hipSuccess;
    ok &= hipStreamCreateWithFlags(&vol->cap_stream, hipStreamNonBlocking) == hipSuccess;
    ok &= hipEventCreateWithFlags(&vol->staged[0], hipEventDisableTiming) == hipSuccess;
    ok &= hipEventCreateWithFlags(&vol->staged[1], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        sc_volume_destroy(vol);
        return SC_ENOMEM;
    }
    hipStream_t s = 0;
    sc_status st = sc_volume_reset(vol, s);
    for (int b = 0; b < 2; ++b)
        if (st == SC_OK && hipEventRecord(vol->staged[b], s) != hipSuccess) st = SC_EDEVICE;
    if (st != SC_OK || hipStreamSynchronize(s) != hipSuccess) {
        sc_volume_destroy(vol);
        return SC_EDEVICE;
    }
    *out = vol;
    return SC_OK;
}

void sc_volume_destroy(sc_volume* vol)
{
    if (!vol) return;
    hipDeviceSynchronize();
    for (hipGraphExec_t g : vol->graph_pre)
        if (g) hipGraphExecDestroy(g);
    for (auto& g : vol->graph_main)
        if (g) hipGraphExecDestroy(g);
    for (int i = 0; i < 2 * vol->timing_cap; ++i) hipEventDestroy(vol->timing_ev[i]);
    delete[] vol->timing_ev;
    hipFree(vol->cand.stats);
    hipFree(vol->cand.skey);
    hipFree(vol->cand.sslot);
    hipFree(vol->dev.keys);
    hipFree(vol->dev.vals);
    hipFree(vol->dev.slot_keys);
    hipFree(vol->dev.pool);
    hipFree(vol->dev.n_blocks);
    hipFree(vol->dev.err);
    hipFree(vol->cand.keys);
    hipFree(vol->cand.mask);
    hipFree(vol->cand.list);
    hipFree(vol->cand.sorted);
    hipFree(vol->cand.counters);
    hipFree(vol->cand.bins);
    hipFree(vol->cand.cursors);
    hipFree(vol->cand.big);
    hipFree(vol->d_ops);
    hipFree(vol->adj_acc);
    hipFree(vol->d_hdr);
    if (vol->h_ops) hipHostFree(vol->h_ops);
    if (vol->h_hdr) hipHostFree(vol->h_hdr);
    if (vol->cap_stream) hipStreamDestroy(vol->cap_stream);
    for (hipEvent_t e : vol->staged)
        if (e) hipEventDestroy(e);
    rec_destroy(vol);
    stream_destroy(vol);
    delete vol;
}

sc_status sc_volume_reset(sc_volume* vol, void* stream)
{
    if (!vol) return SC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    fill_u64(vol->dev.keys, kKeyEmpty, (size_t)vol->p.n_buckets, s);
    fill_u32(reinterpret_cast<uint32_t*>(vol->dev.vals), 0xFFFFFFFFu, (size_t)vol->p.n_buckets, s);
    fill_u32(reinterpret_cast<uint32_t*>(vol->dev.pool), 0u, (size_t)vol->dev.stride * vol->p.max_blocks, s);
    fill_u32(vol->dev.n_blocks, 0u, 16, s);
    fill_u32(reinterpret_cast<uint32_t*>(vol->dev.err), 0u, 16, s);
    const CandDev& c = vol->cand;
    fill_u64(c.keys, kKeyEmpty, vol->cand_buckets, s);
    fill_u64(c.mask, 0ull, (size_t)vol->cand_buckets * c.words, s);
    fill_u32(c.counters, 0u, 64, s);
    fill_u32(c.bins, 0u, kMaxBatchOps + 2, s);
    fill_u32(c.cursors, 0u, (size_t)2 * kCursorSet, s);
    fill_u32(c.big, 0u, 1, s);
    fill_u64(reinterpret_cast<uint64_t*>(c.stats), 0ull, 4 * kStatSlots, s);
    fill_u64(reinterpret_cast<uint64_t*>(vol->adj_acc), 0ull, 3 * kAdjChunk, s);
    vol->parity = 0;
    rec_clear(vol);
    stream_clear(vol);
    return hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
}

sc_status sc_volume_query(sc_volume* vol, void* stream, int64_t* n_blocks, int32_t* sticky_error)
{
    if (!vol) return SC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    uint32_t nb = 0;
    int32_t e = 0;
    HIP_TRY(hipMemcpyAsync(&nb, vol->dev.n_blocks, sizeof(nb), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&e, vol->dev.err, sizeof(e), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (n_blocks) *n_blocks = std::min<int64_t>((int64_t)nb, vol->p.max_blocks);
    if (sticky_error) *sticky_error = e;
    return SC_OK;
}

sc_status sc_volume_export(sc_volume* vol, void* stream, int32_t* block_xyz, float* D, float* W, void* C, int64_t cap,
                           int64_t* n_out)
{
    if (!vol || cap < 0) return SC_EINVAL;
    int64_t nb = 0;
    sc_status st = sc_volume_query(vol, stream, &nb, nullptr);
    if (st != SC_OK) return st;
    const int64_t n = std::min(nb, cap);
    hipStream_t s = (hipStream_t)stream;
    if (n > 0) export_kernel<<<(unsigned)n, 256, 0, s>>>(vol->dev, n, block_xyz, D, W, C);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(s));
    if (n_out) *n_out = nb;
    return SC_OK;
}

sc_status sc_volume_import(sc_volume* vol, void* stream, const int32_t* block_xyz, const float* D, const float* W,
                           const void* C, int64_t n)
{
    if (!vol || n < 0 || (n > 0 && !block_xyz) || n > vol->p.max_blocks || stream_host_blocks(vol) > 0)
        return SC_EINVAL;
    if (n == 0) return SC_OK;
    hipStream_t s = (hipStream_t)stream;
    int32_t* slots = nullptr;
    HIP_TRY(hipMalloc(&slots, sizeof(int32_t) * (size_t)n));
    sc_status st = hash_alloc(vol, block_xyz, n, slots, stream);
    if (st == SC_OK) {
        import_kernel<<<(unsigned)n, 256, 0, s>>>(vol->dev, slots, n, D, W, C);
        st = hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
    }
    int64_t nb = 0;
    int32_t sticky = 0;
    if (st == SC_OK) st = sc_volume_query(vol, stream, &nb, &sticky);
    (void)hipFree(slots);
    if (st != SC_OK) return st;
    return sticky;
}

int64_t sc_keyframe_pack_bytes(int32_t width, int32_t height)
{
    if (width <= 0 || height <= 0 || width > 16384 || height > 16384) return 0;
    const int64_t cells = (int64_t)((width + 3) / 4) * ((height + 3) / 4);
    return (int64_t)width * height * 16 + cells * 8;
}

sc_status sc_keyframe_pack(const sc_keyframe* kf, int32_t width, int32_t height, void* packed, int64_t packed_bytes,
                           void* stream)
{
    const int64_t need = sc_keyframe_pack_bytes(width, height);
    if (!kf || !kf->depth || !kf->weight || !kf->color || !packed || ((uintptr_t)packed & 15u) || need == 0 ||
        packed_bytes < need)
        return SC_EINVAL;
    const int64_t n = (int64_t)width * height;
    const int grid = (int)std::min<int64_t>((n + 255) / 256, 65536);
    pack_kernel<<<grid, 256, 0, (hipStream_t)stream>>>(kf->depth, kf->weight,
                                                        reinterpret_cast<const uint32_t*>(kf->color),
                                                        reinterpret_cast<uint4*>(packed), n);
    const int cells_w = (width + 3) / 4;
    const int64_t n_cells = (int64_t)cells_w * ((height + 3) / 4);
    pack_cells_kernel<<<(int)std::min<int64_t>((n_cells + 255) / 256, 65536), 256, 0, (hipStream_t)stream>>>(
        kf->depth, kf->weight, reinterpret_cast<float2*>(reinterpret_cast<uint4*>(packed) + n), width, height, cells_w,
        n_cells);
    return hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
}

sc_status hash_alloc(sc_volume* vol, const int32_t* block_xyz, int64_t n, int32_t* slots_out, void* stream)
{
    if (!vol || n < 0 || (n > 0 && !block_xyz) || stream_host_blocks(vol) > 0) return SC_EINVAL;
    if (n == 0) return SC_OK;
    hipStream_t s = (hipStream_t)stream;
    const unsigned grid = (unsigned)((n + 255) / 256);
    hash_alloc_kernel<<<grid, 256, 0, s>>>(vol->dev, block_xyz, n);
    if (slots_out) hash_lookup_kernel<<<grid, 256, 0, s>>>(vol->dev, block_xyz, n, slots_out);
    return hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
}

sc_status tsdf_integrate(sc_volume* vol, const sc_keyframe* kf, const sc_intrinsics* intr, const sc_pose* T,
                         void* stream)
{
    return plain_op(vol, kf, intr, T, +1, (hipStream_t)stream);
}

sc_status tsdf_deintegrate(sc_volume* vol, const sc_keyframe* kf, const sc_intrinsics* intr, const sc_pose* T,
                           void* stream)
{
    return plain_op(vol, kf, intr, T, -1, (hipStream_t)stream);
}

sc_status reintegrate_plain(sc_volume* vol, const sc_keyframe* kfs, int32_t n_kf, const sc_intrinsics* intr,
                            sc_pose* T_integrated, const sc_pose* T_new, int32_t m, int32_t mode,
                            int32_t* selected_out, int32_t* n_selected, void* stream)
{
    if (!vol || !kfs || n_kf <= 0 || !T_integrated || !T_new || !intr_ok(intr)) return SC_EINVAL;
    for (int i = 0; i < n_kf; ++i)
        if (!keyframe_ok(&kfs[i])) return SC_EINVAL;
    int32_t* order = new (std::nothrow) int32_t[n_kf];
    if (!order) return SC_ENOMEM;
    const int32_t ns = sc_select(T_integrated, T_new, n_kf, m, mode, order, nullptr);
    if (ns < 0) {
        delete[] order;
        return ns;
    }
    hipStream_t s = (hipStream_t)stream;
    sc_status st = SC_OK;
    for (int j = 0; j < ns && st == SC_OK; ++j) st = plain_op(vol, &kfs[order[j]], intr, &T_integrated[order[j]], -1, s);
    for (int j = 0; j < ns && st == SC_OK; ++j) st = plain_op(vol, &kfs[order[j]], intr, &T_new[order[j]], +1, s);
    if (st == SC_OK) {
        for (int j = 0; j < ns; ++j) T_integrated[order[j]] = T_new[order[j]];
        if (selected_out) memcpy(selected_out, order, sizeof(int32_t) * ns);
        if (n_selected) *n_selected = ns;
    }
    delete[] order;
    return st;
}

}  // extern "C"
