// Device code shared by the plain and batched voxel passes: the decision
// convention (camera point, nearest pixel, touched test), the voxel updates
// of integration (Sec. 3, running weighted average) and de-integration
// (Sec. 4.3, Eq. 2), the block hash and the candidate-block generation.
//
// Compiled with -ffp-contract=off: every FP32/FP64 expression below is
// evaluated with correctly rounded IEEE operations in the written order.
#pragma once

#include "common.hpp"

namespace sc {

__device__ inline void set_error(int32_t* err, int32_t code) { atomicCAS(err, 0, code); }

// ---------------------------------------------------------------------------
// wavefront-level helpers for persistent loops
//
// Inside persistent loops no branch depends on the lane id: a region executed
// by lane 0 only, next to the loop's back edge, can be restructured by the
// compiler into nested loops that separate lane 0 from the other lanes, after
// which cross-lane reads see the wrong lanes.  Single-lane side effects are
// therefore issued branch-free by every lane, and values are broadcast with
// readfirstlane only at the top level of the loop body, where every lane of
// the wavefront is active.
// ---------------------------------------------------------------------------

constexpr uint64_t kKeyNever = ~1ull;  // has bit 63 set: never a key, never empty

__device__ inline uint32_t bcast(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ inline uint64_t bcast64(uint64_t x)
{
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Adds one to *ctr once per wavefront; every lane receives the old value.
__device__ inline uint32_t wave_fetch_add1(uint32_t* ctr, int lane)
{
    const uint32_t r = atomicAdd(ctr, lane == 0 ? 1u : 0u);
    return bcast(r);
}

// ---------------------------------------------------------------------------
// decision convention
// ---------------------------------------------------------------------------

// Camera-frame position of block (bx, by, bz)'s origin: R^T (8 s b - t) in
// FP64, rounded once to FP32 for the decisions; its z also returned in FP64
// for the continuous distance.
__device__ inline void block_origin(const OpDesc& op, float s, int bx, int by, int bz, float q[3], double& qz)
{
    const double s8 = 8.0 * (double)s;
    const double e0 = s8 * (double)bx - op.t[0];
    const double e1 = s8 * (double)by - op.t[1];
    const double e2 = s8 * (double)bz - op.t[2];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const double v = (op.R[r] * e0 + op.R[3 + r] * e1) + op.R[6 + r] * e2;
        q[r] = (float)v;
        if (r == 2) qz = v;
    }
}

// Nearest pixel of the pinhole projection; false if behind the camera or
// outside the image.
__device__ inline bool nearest_pixel(const OpDesc& op, float px, float py, float pz, int& pix)
{
    if (!(pz > 0.0f)) return false;
    const float u = (op.fx * px) / pz + op.cx;
    const float v = (op.fy * py) / pz + op.cy;
    const float fu = floorf(u + 0.5f);
    const float fv = floorf(v + 0.5f);
    if (!(fu >= 0.0f && fu <= (float)(op.width - 1) && fv >= 0.0f && fv <= (float)(op.height - 1))) return false;
    pix = (int)fv * op.width + (int)fu;
    return true;
}

__device__ inline float qweight(float w) { return rintf(w * kWeightScale) * (1.0f / kWeightScale); }

// Touched test of one voxel whose FP32 camera point is (px, py, pz).  On
// success returns the pixel, the quantised weight w and the keyframe depth z
// there (the band test uses fl32(z - pz)).
__device__ inline bool touch(const OpDesc& op, float mu, float px, float py, float pz, int& pix, float& w, float& z)
{
    if (!nearest_pixel(op, px, py, pz, pix)) return false;
    w = qweight(__ldg(op.weight + pix));
    if (!(w > 0.0f)) return false;
    z = __ldg(op.depth + pix);
    return fabsf(z - pz) <= mu;
}

// Continuous projective distance d = Z*(pixel) - p_z with p_z in FP64.
__device__ inline float distance(float z, double pz64) { return (float)((double)z - pz64); }

// ---------------------------------------------------------------------------
// voxel updates
// ---------------------------------------------------------------------------

// Round-half-to-even of N / M (exact rational), clamped to 255.
// N < 2^32, 0 < M < 2^24.  An FP32 estimate is corrected with the exact
// integer residual, so the result is the exact rounding.
__device__ inline uint32_t rne_div_255(uint32_t N, uint32_t M, float rcpM)
{
    const float qf = (float)N * rcpM;
    if (qf >= 256.5f) return 255u;
    int q = (int)rintf(qf);
    int twice = 2 * (int)(N - (uint32_t)q * M);  // |residual| < 0.51 M, so no overflow
    const int m = (int)M;
    if (twice > m) {
        q += 1;
        twice -= 2 * m;
    } else if (twice < -m) {
        q -= 1;
        twice += 2 * m;
    }
    if (twice == m && (q & 1)) q += 1;
    else if (twice == -m && (q & 1)) q -= 1;
    return (uint32_t)min(max(q, 0), 255);
}

// One RGBA8 colour channel after (de-)integration: the exact rational
// (C Wq +- c wq) / W'q on the 2^-10 weight grid, rounded, clamped to [0,255].
__device__ inline uint32_t mix_channel(uint32_t C, uint32_t c, uint32_t Wq, uint32_t wq, uint32_t W1q, float rcp,
                                       int sign)
{
    int64_t N = (int64_t)C * Wq + (int64_t)sign * (int64_t)c * wq;
    if (N <= 0) return 0u;
    return rne_div_255((uint32_t)N, W1q, rcp);
}

// Integrate (sign +1) or de-integrate (sign -1, Eq. 2) one sample into an
// RGBA8 voxel held in registers.  Returns false on a weight error.
__device__ inline bool update_rgba8(float& D, float& W, uint32_t& C, float d, float w, uint32_t c, int sign)
{
    const float W1 = (sign > 0) ? W + w : W - w;  // exact on the 2^-10 grid
    if (sign > 0 ? !(W1 < kWeightLimit) : (W1 < 0.0f)) return false;
    if (W1 == 0.0f) {
        D = 0.0f;
        W = 0.0f;
        C = 0u;
        return true;
    }
    const float rcp = __builtin_amdgcn_rcpf(W1);
    D = (sign > 0 ? (D * W + d * w) : (D * W - d * w)) * rcp;
    const uint32_t Wq = (uint32_t)(W * kWeightScale);
    const uint32_t wq = (uint32_t)(w * kWeightScale);
    const uint32_t W1q = (uint32_t)(W1 * kWeightScale);
    const float rcpq = __builtin_amdgcn_rcpf((float)W1q);
    const uint32_t r = mix_channel(C & 0xFFu, c & 0xFFu, Wq, wq, W1q, rcpq, sign);
    const uint32_t g = mix_channel((C >> 8) & 0xFFu, (c >> 8) & 0xFFu, Wq, wq, W1q, rcpq, sign);
    const uint32_t b = mix_channel((C >> 16) & 0xFFu, (c >> 16) & 0xFFu, Wq, wq, W1q, rcpq, sign);
    C = r | (g << 8) | (b << 16);
    W = W1;
    return true;
}

// FP32-colour mode: keyframe colour FP32 in [0,1]; the voxel colour is held
// in FP64, because Eq. (2) amplifies the rounding of the stored colour by
// W / W' when most of a voxel's weight is removed.
__device__ inline bool update_f32(float& D, float& W, double C[3], float d, float w, const float c[3], int sign)
{
    const float W1 = (sign > 0) ? W + w : W - w;
    if (sign > 0 ? !(W1 < kWeightLimit) : (W1 < 0.0f)) return false;
    if (W1 == 0.0f) {
        D = 0.0f;
        W = 0.0f;
        C[0] = C[1] = C[2] = 0.0;
        return true;
    }
    const float rcp = __builtin_amdgcn_rcpf(W1);
    D = (sign > 0 ? (D * W + d * w) : (D * W - d * w)) * rcp;
    const double Wd = (double)W, wd = (double)w, W1d = (double)W1;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        C[k] = (sign > 0 ? (C[k] * Wd + (double)c[k] * wd) : (C[k] * Wd - (double)c[k] * wd)) / W1d;
    W = W1;
    return true;
}

// ---------------------------------------------------------------------------
// block hash
// ---------------------------------------------------------------------------

// Finds the pool slot of a block, or -1.
__device__ inline int vol_find(const VolDev& v, uint64_t key, int bx, int by, int bz)
{
    uint32_t h = hash_block(bx, by, bz) & v.bucket_mask;
    for (uint32_t probe = 0; probe <= v.bucket_mask; ++probe) {
        const uint64_t k = v.keys[h];
        if (k == key) return v.vals[h];
        if (k == kKeyEmpty) return -1;
        h = (h + 1) & v.bucket_mask;
    }
    return -1;
}

// Inserts a block that no other thread inserts concurrently and returns its
// slot; on a full table or pool sets the sticky error and returns -1.
__device__ inline int vol_insert_unique(const VolDev& v, uint64_t key, int bx, int by, int bz)
{
    uint32_t h = hash_block(bx, by, bz) & v.bucket_mask;
    for (uint32_t probe = 0; probe <= v.bucket_mask; ++probe) {
        const uint64_t old = atomicCAS((unsigned long long*)(v.keys + h), (unsigned long long)kKeyEmpty,
                                       (unsigned long long)key);
        if (old == key) return v.vals[h];
        if (old == kKeyEmpty) {
            const uint32_t slot = atomicAdd(v.n_blocks, 1u);
            if (slot >= (uint32_t)v.max_blocks) {
                v.vals[h] = -1;
                set_error(v.err, SC_EPOOLFULL);
                return -1;
            }
            v.slot_keys[slot] = key;
            v.vals[h] = (int)slot;
            return (int)slot;
        }
        h = (h + 1) & v.bucket_mask;
    }
    set_error(v.err, SC_EHASHFULL);
    return -1;
}

// Wavefront-cooperative insert of a block no other wavefront inserts
// concurrently: every lane issues the CAS, lanes other than 0 compare against
// a value that never occurs, so only lane 0 can write; lane 0's view decides.
__device__ inline int vol_insert_wave(const VolDev& v, uint64_t key, int bx, int by, int bz, int lane)
{
    const unsigned long long cmp = (lane == 0) ? (unsigned long long)kKeyEmpty : (unsigned long long)kKeyNever;
    uint32_t h = hash_block(bx, by, bz) & v.bucket_mask;
    for (uint32_t probe = 0; probe <= v.bucket_mask; ++probe) {
        const uint64_t old =
            bcast64(atomicCAS((unsigned long long*)(v.keys + h), cmp, (unsigned long long)key));
        if (old == kKeyEmpty) {
            const uint32_t slot = wave_fetch_add1(v.n_blocks, lane);
            if (slot >= (uint32_t)v.max_blocks) {
                v.vals[h] = -1;
                set_error(v.err, SC_EPOOLFULL);
                return -1;
            }
            v.slot_keys[slot] = key;
            v.vals[h] = (int)slot;
            return (int)slot;
        }
        if (old == key) return (int)bcast((uint32_t)v.vals[h]);
        h = (h + 1) & v.bucket_mask;
    }
    set_error(v.err, SC_EHASHFULL);
    return -1;
}

// ---------------------------------------------------------------------------
// candidate blocks
// ---------------------------------------------------------------------------

constexpr int kTile = 16;     // candidate generation works on 16 x 16 pixel tiles
constexpr int kLdsSet = 1024; // LDS hash set per tile

// Conservative world-space block range of one pixel's frustum cell
// (u +- 0.55, v +- 0.55) between depths z - mu and z + mu, padded so that
// FP32 rounding in the decision convention cannot escape it.
__device__ inline bool pixel_block_range(const OpDesc& op, float s, float mu, int u, int v, float z, int lo[3],
                                         int hi[3])
{
    const float zl = fmaxf(z - mu - 1e-3f, 0.0f);
    const float zh = z + mu + 1e-3f;
    const float xl = ((float)u - 0.55f - op.cx) / op.fx, xh = ((float)u + 0.55f - op.cx) / op.fx;
    const float yl = ((float)v - 0.55f - op.cy) / op.fy, yh = ((float)v + 0.55f - op.cy) / op.fy;
    float mn[3], mx[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        mn[r] = 3.0e38f;
        mx[r] = -3.0e38f;
    }
#pragma unroll
    for (int iz = 0; iz < 2; ++iz) {
        const float zz = iz ? zh : zl;
        const float cxm = 0.5f * (xl + xh) * zz, hx = 0.5f * (xh - xl) * zz;
        const float cym = 0.5f * (yl + yh) * zz, hy = 0.5f * (yh - yl) * zz;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const float r0 = (float)op.R[3 * r + 0], r1 = (float)op.R[3 * r + 1], r2 = (float)op.R[3 * r + 2];
            const float c = r0 * cxm + r1 * cym + r2 * zz + (float)op.t[r];
            const float e = fabsf(r0) * hx + fabsf(r1) * hy;
            mn[r] = fminf(mn[r], c - e);
            mx[r] = fmaxf(mx[r], c + e);
        }
    }
    bool ok = true;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float pad = 2e-3f + 2e-5f * fmaxf(fabsf(mn[r]), fabsf(mx[r]));
        const float flo = ceilf((mn[r] - pad) / s);
        const float fhi = floorf((mx[r] + pad) / s);
        // keys hold 21-bit block coordinates; a cell wider than 16 blocks means
        // a depth far beyond the voxel scale and is rejected
        ok = ok && (flo > -8.0e6f) && (fhi < 8.0e6f) && (fhi - flo < 128.0f);
        lo[r] = ok ? ((int)flo >> 3) : 0;  // arithmetic shift: floor division by 8
        hi[r] = ok ? ((int)fhi >> 3) : -1;
    }
    return ok;
}

// Inserts a candidate block into the deduplicating candidate table; returns
// its bucket, or -1 if the table is full (sticky error set).
__device__ inline int cand_insert(const CandDev& cd, const VolDev& v, uint64_t key, int bx, int by, int bz,
                                  uint32_t* count)
{
    uint32_t h = hash_block(bx, by, bz) & cd.mask_bits;
    for (uint32_t probe = 0; probe <= cd.mask_bits; ++probe) {
        const uint64_t old = atomicCAS((unsigned long long*)(cd.keys + h), (unsigned long long)kKeyEmpty,
                                       (unsigned long long)key);
        if (old == key) return (int)h;
        if (old == kKeyEmpty) {
            const uint32_t idx = atomicAdd(count, 1u);
            if (idx < cd.cap) {
                cd.list[idx] = h;
            } else {
                set_error(v.err, SC_EHASHFULL);
            }
            return (int)h;
        }
        h = (h + 1) & cd.mask_bits;
    }
    set_error(v.err, SC_EHASHFULL);
    return -1;
}

// Candidate generation for one 16 x 16 tile of one keyframe operation
// (256 threads): per-pixel conservative block ranges, deduplicated in an
// LDS hash set, then inserted once per tile into the global candidate table.
// With op_bit >= 0 the operation's bit is set in the block's mask.
__device__ inline void cand_tile(const OpDesc& op, const VolDev& v, const CandDev& cd, uint32_t* count, int tx,
                                 int ty, int op_bit, uint64_t* lds)
{
    const int tid = threadIdx.x;
    for (int i = tid; i < kLdsSet; i += blockDim.x) lds[i] = kKeyEmpty;
    __syncthreads();
    const int u = tx * kTile + (tid & (kTile - 1));
    const int vv = ty * kTile + (tid >> 4);
    if (u < op.width && vv < op.height) {
        const int pix = vv * op.width + u;
        const float w = qweight(op.weight[pix]);
        const float z = op.depth[pix];
        if (w > 0.0f && z > 0.0f && z < 1.0e30f) {
            int lo[3], hi[3];
            if (!pixel_block_range(op, v.s, v.mu, u, vv, z, lo, hi)) set_error(v.err, SC_ERANGE);
            for (int bx = lo[0]; bx <= hi[0]; ++bx)
                for (int by = lo[1]; by <= hi[1]; ++by)
                    for (int bz = lo[2]; bz <= hi[2]; ++bz) {
                        const uint64_t key = pack_key(bx, by, bz);
                        uint32_t h = hash_block(bx, by, bz) & (kLdsSet - 1);
                        bool placed = false;
                        for (int probe = 0; probe < 32; ++probe) {
                            const uint64_t old = atomicCAS((unsigned long long*)(lds + h),
                                                           (unsigned long long)kKeyEmpty, (unsigned long long)key);
                            if (old == kKeyEmpty || old == key) {
                                placed = true;
                                break;
                            }
                            h = (h + 1) & (kLdsSet - 1);
                        }
                        if (!placed) {
                            const int gb = cand_insert(cd, v, key, bx, by, bz, count);
                            if (gb >= 0 && op_bit >= 0)
                                atomicOr((unsigned long long*)(cd.mask + (size_t)gb * cd.words + (op_bit >> 6)),
                                         1ull << (op_bit & 63));
                        }
                    }
        }
    }
    __syncthreads();
    for (int i = tid; i < kLdsSet; i += blockDim.x) {
        const uint64_t key = lds[i];
        if (key == kKeyEmpty) continue;
        int bx, by, bz;
        unpack_key(key, bx, by, bz);
        const int gb = cand_insert(cd, v, key, bx, by, bz, count);
        if (gb >= 0 && op_bit >= 0)
            atomicOr((unsigned long long*)(cd.mask + (size_t)gb * cd.words + (op_bit >> 6)), 1ull << (op_bit & 63));
    }
}

}  // namespace sc
