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

// Number of set bits of the wavefront mask m below this lane.
__device__ inline uint32_t lanes_below(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Orders this wavefront's LDS accesses: the lanes that write a list or queue
// entry or a voxel are not the lanes that read it next.
__device__ inline void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Adds k to *ctr once per wavefront; every lane receives the old value.
__device__ inline uint32_t wave_fetch_add(uint32_t* ctr, uint32_t k, int lane)
{
    const uint32_t r = atomicAdd(ctr, lane == 0 ? k : 0u);
    return bcast(r);
}

__device__ inline uint32_t wave_fetch_add1(uint32_t* ctr, int lane) { return wave_fetch_add(ctr, 1u, lane); }

// Sum over the wavefront.
__device__ inline uint32_t wave_sum(uint32_t x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Work distribution of the persistent passes.  A device-wide atomic on one
// address is serviced one at a time, so a queue that pops one item per
// atomic is bounded by that service rate.  Instead each worker (wavefront or
// workgroup) takes item `id` first, without an atomic (the queue is ordered
// heaviest first, so the heaviest items spread over all workers), then
// claims kPopBatch consecutive items per atomic.  Used in uniform control
// flow only.
constexpr uint32_t kPopBatch = 4;

struct WorkCursor {
    uint32_t next, end;
};

__device__ inline void cursor_init(WorkCursor& c, uint32_t id)
{
    c.next = id;
    c.end = id + 1u;
}

__device__ inline uint32_t cursor_pop(WorkCursor& c, uint32_t* ctr, uint32_t n_workers, int lane)
{
    if (c.next >= c.end) {
        // single items through the heavy front of the queue, so that no
        // worker holds several heavy items at once; batches after it
        const uint32_t k = (c.next < 2u * n_workers) ? 1u : kPopBatch;
        c.next = n_workers + wave_fetch_add(ctr, k, lane);
        c.end = c.next + k;
    }
    return c.next++;
}

// The same distribution over kCursors interleaved ranges (item i in range
// i mod kCursors, each range with its own counter in its own page), so that
// the claims of many wavefronts do not queue on one address: worker w takes
// item w first, then claims from its range (single items through the heavy
// front, kRangePop after it); a worker that finds its range exhausted marks
// it in a shared bit mask and moves on to a range not yet marked.  Returns
// n when every range is exhausted.  Used in uniform control flow only.
static_assert(kCursors == 32, "the exhausted-range mask is one 32-bit word");
constexpr uint32_t kRangePop = 8;  // items per claim past the heavy front

struct RangeCursor {
    uint32_t next, end;  // indices [next, end) within range r held
    int r;
};

__device__ inline void range_init(RangeCursor& c, uint32_t worker)
{
    c.r = (int)(worker % kCursors);
    c.next = worker / kCursors;
    c.end = c.next + 1u;
}

__device__ inline uint32_t range_pop(RangeCursor& c, uint32_t* cursors, uint32_t n, uint32_t n_workers, int lane)
{
    for (;;) {
        // indices below `base` of range r are the workers' static first items
        const uint32_t base = (n_workers + kCursors - 1u - (uint32_t)c.r) / kCursors;
        // a pass with no more items than workers has only static items
        if (c.next >= c.end && n <= n_workers) return n;
        if (c.next >= c.end) {
            const uint32_t k = (c.end < 2u * base) ? 1u : kRangePop;
            c.next = base + bcast(atomicAdd(cursors + c.r * kCursorStride, lane == 0 ? k : 0u));
            c.end = c.next + k;
        }
        const uint32_t item = (uint32_t)c.r + kCursors * c.next;
        if (item < n) {
            c.next++;
            return item;
        }
        if (n <= n_workers) return n;
        const uint32_t m =
            bcast(atomicOr(cursors + kCursorDone, lane == 0 ? (1u << c.r) : 0u)) | (1u << c.r);
        if (m == ~0u) return n;
        int nr = c.r;
        for (int j = 1; j < kCursors; ++j) {
            const int q = (c.r + j) % kCursors;
            if (!((m >> q) & 1u)) {
                nr = q;
                break;
            }
        }
        c.r = nr;
        c.next = c.end = 0u;
    }
}

// Per-pass statistics are added into kStatSlots slots per counter so that the
// workers' final atomics do not all meet on one address.
constexpr int kStatSlots = 64;

__device__ inline void stat_add(const CandDev& cd, int counter, uint32_t worker, uint64_t x, int lane)
{
    atomicAdd(cd.stats + counter * kStatSlots + (worker % kStatSlots), (unsigned long long)(lane == 0 ? x : 0ull));
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
// Pixel coordinate floor(fl32(fl32(t + c) + 0.5)) of t = fl32(a / z) (a
// correctly rounded division), given r = rcp(z) with at most one ulp of
// error.  fl32(a * r) is within |a r| 2^-21 of t, so t lies in
// [a r - e, a r + e] with e = |a r| 2^-20 (+2^-60 for tiny values); the map
// t -> floor(fl32(fl32(t + c) + 0.5)) is monotone, so when both ends of the
// interval give the same integer that is the exact result, and when both lie
// beyond the same image border the pixel is outside either way.  Only the
// remaining cases take the correctly rounded division.
__device__ inline float pixel_coord(float a, float z, float r, float c, float limit)
{
    const float tq = a * r;
    const float e = fabsf(tq) * 0x1p-20f + 0x1p-60f;
    const float lo = floorf(((tq - e) + c) + 0.5f);
    const float hi = floorf(((tq + e) + c) + 0.5f);
    if (lo == hi) return lo;
    if (hi < 0.0f || lo > limit) return -1.0f;
    return floorf(((a / z) + c) + 0.5f);
}

// The same pixel coordinate with one rounding test instead of two: with
// tq = fl32(a r), |tq - t| <= |tq| 2^-22 (one ulp of rcp and two roundings),
// and the two additions of the convention round by at most one ulp of their
// results on either side, so the convention's f = fl32(fl32(t + c) + 1/2)
// and fq = fl32(yq + 1/2), yq = fl32(tq + c), differ by at most
// |tq| 2^-22 + |yq| 2^-22 + 2^-24.  yq - floor(fq) equals fq - floor(fq) - 1/2
// to within |yq| 2^-24 + 2^-24, so when it lies inside (-1/2, 1/2) by more
// than m = (|tq| + |yq|) 2^-21 + 2^-21 (which covers both terms), f and fq
// have the same floor.  The rare lanes nearer a half-integer take the
// interval test of pixel_coord.
__device__ inline float pixel_coord_fast(float a, float z, float r, float c, float limit)
{
    const float tq = a * r;
    const float yq = tq + c;
    const float fl = floorf(yq + 0.5f);
    const float inner = fmaf(fabsf(tq) + fabsf(yq), -0x1p-21f, 0.5f - 0x1p-21f);
    if (fabsf(yq - fl) < inner) return fl;
    return pixel_coord(a, z, r, c, limit);
}

// nearest_pixel with pixel_coord_fast.
__device__ inline bool nearest_pixel_fast(const OpDesc& op, float px, float py, float pz, int& pix)
{
    if (!(pz > 0.0f)) return false;
    const float r = __builtin_amdgcn_rcpf(pz);
    const float wl = (float)(op.width - 1), hl = (float)(op.height - 1);
    const float fu = pixel_coord_fast(op.fx * px, pz, r, op.cx, wl);
    const float fv = pixel_coord_fast(op.fy * py, pz, r, op.cy, hl);
    if (!(fu >= 0.0f && fu <= wl && fv >= 0.0f && fv <= hl)) return false;
    pix = (int)fv * op.width + (int)fu;
    return true;
}

// The pixel coordinate of pixel_coord_fast with a cheaper test.  For
// |yq| < 2^22 the convention's fl32(y + 1/2) is exact, so its floor is the
// nearest integer to y = fl32(t + c) away from half-integers, and rint(yq)
// stands in for floor(fl32(yq + 1/2)).  |y - yq| <= |tq| 2^-22 +
// (|y| + |yq|) 2^-24, below (2 |tq| + |c|) 2^-21 + 2^-21 >= (|tq| + |yq|)
// 2^-21 + 2^-21; so when yq lies inside (-1/2, 1/2) of rint(yq) by more
// than that, y lies in the same interval and floor(y + 1/2) = rint(yq).
// kin <= 1/2 - (1 + |c|) 2^-21 comes with the operation.  A coordinate with
// |yq| >= 2^22 is far outside the image either way.  Other lanes take the
// interval test of pixel_coord.
__device__ inline float pixel_coord_rint(float a, float z, float r, float c, float kin, float limit)
{
    const float tq = a * r;
    const float yq = tq + c;
    const float fl = rintf(yq);
    if (fabsf(yq - fl) < fmaf(fabsf(tq), -0x1p-20f, kin)) return fl;
    return pixel_coord(a, z, r, c, limit);
}

// The projection constants of one operation, read together.
struct ProjConst {
    float fx, fy, cx, cy, kin_u, kin_v, wl, hl, wf;
};

__device__ inline ProjConst proj_const(const OpDesc& op)
{
    return {op.fx, op.fy, op.cx, op.cy, op.kin_u, op.kin_v, op.wl, op.hl, op.wf};
}

// The nearest pixel without branches around it, with pixel_coord_rint: the
// pixel index (0 when `in` is false: behind the camera or outside the
// image).  A lane behind the camera projects with z = 1 so that its
// coordinates stay finite.  The index fv W + fu is an integer below 2^24, so
// one FP32 fma forms it exactly.
__device__ inline uint32_t pixel_index_fast(const ProjConst& k, float px, float py, float pz, bool& in)
{
    const bool front = pz > 0.0f;
    const float zs = front ? pz : 1.0f;
    const float r = __builtin_amdgcn_rcpf(zs);
    const float fu = pixel_coord_rint(k.fx * px, zs, r, k.cx, k.kin_u, k.wl);
    const float fv = pixel_coord_rint(k.fy * py, zs, r, k.cy, k.kin_v, k.hl);
    // bitwise, not short-circuit: no branches
    in = front & (fu >= 0.0f) & (fu <= k.wl) & (fv >= 0.0f) & (fv <= k.hl);
    const uint32_t p = (uint32_t)fmaf(fv, k.wf, fu);
    return in ? p : 0u;
}

// Nearest pixel of the FP32 camera point (px, py, pz); false if behind the
// camera or outside the image.
__device__ inline bool nearest_pixel(const OpDesc& op, float px, float py, float pz, int& pix)
{
    if (!(pz > 0.0f)) return false;
    const float r = __builtin_amdgcn_rcpf(pz);
    const float wl = (float)(op.width - 1), hl = (float)(op.height - 1);
    const float fu = pixel_coord(op.fx * px, pz, r, op.cx, wl);
    const float fv = pixel_coord(op.fy * py, pz, r, op.cy, hl);
    if (!(fu >= 0.0f && fu <= wl && fv >= 0.0f && fv <= hl)) return false;
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
__device__ inline double distance(float z, double pz64) { return (double)z - pz64; }

// What one lane learns about its VPL voxels (z = kz0 .. kz0 + VPL - 1 of its
// column) from one operation.
template <int CM, int VPL>
struct VoxHits {
    uint32_t hit;   // bit j: voxel j is touched
    int pix[VPL];
    float w[VPL], z[VPL];
    uint32_t c[VPL]; // RGBA8 colour at the pixel (RGBA8 mode)
};

// Projections and keyframe samples of a lane's VPL voxels for one operation
// (the loads are issued, not waited for: the caller decides later).
template <int CM, int VPL>
struct VoxFetch {
    uint32_t in;  // bit j: voxel j projects into the image
    int pix[VPL];
    float pz[VPL], wr[VPL], z[VPL];
    uint32_t c[VPL];  // RGBA8 colour at the pixel (RGBA8 mode)
};

template <int CM, int VPL, bool kColor>
__device__ inline void fetch_voxels(const OpDesc& op, const float base[3], int kz0, VoxFetch<CM, VPL>& f)
{
    f.in = 0u;
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
        const float fz = (float)(kz0 + j);
        const float px = base[0] + fz * op.a[2][0];
        const float py = base[1] + fz * op.a[2][1];
        const float pz = base[2] + fz * op.a[2][2];
        int p = 0;
        const bool in = nearest_pixel(op, px, py, pz, p);
        f.in |= in ? (1u << j) : 0u;
        f.pix[j] = in ? p : 0;
        f.pz[j] = pz;
    }
    if (CM == SC_COLOR_RGBA8 && op.packed) {
#pragma unroll
        for (int j = 0; j < VPL; ++j) {
            const uint4 r = __ldg(op.packed + f.pix[j]);
            f.z[j] = __uint_as_float(r.x);
            f.wr[j] = __uint_as_float(r.y);
            f.c[j] = r.z;
        }
    } else {
#pragma unroll
        for (int j = 0; j < VPL; ++j) {
            f.wr[j] = __ldg(op.weight + f.pix[j]);
            f.z[j] = __ldg(op.depth + f.pix[j]);
            f.c[j] = (kColor && CM == SC_COLOR_RGBA8)
                         ? __ldg(reinterpret_cast<const uint32_t*>(op.color) + f.pix[j])
                         : 0u;
        }
    }
}

// The touched decisions of fetched voxels.
template <int CM, int VPL>
__device__ inline void decide_voxels(const VoxFetch<CM, VPL>& f, float mu, VoxHits<CM, VPL>& h)
{
    h.hit = 0u;
#pragma unroll
    for (int j = 0; j < VPL; ++j) {
        h.pix[j] = f.pix[j];
        h.z[j] = f.z[j];
        h.c[j] = f.c[j];
        h.w[j] = qweight(f.wr[j]);
        const bool t = ((f.in >> j) & 1u) && h.w[j] > 0.0f && fabsf(h.z[j] - f.pz[j]) <= mu;
        h.hit |= t ? (1u << j) : 0u;
    }
}

// Touched tests of a lane's VPL voxels: every projection first, then every
// keyframe load (voxels outside the image read pixel 0, so the loads need no
// branch and are issued together), then the decisions.
template <int CM, int VPL, bool kColor = true>
__device__ inline void test_voxels(const OpDesc& op, float mu, const float base[3], int kz0, VoxHits<CM, VPL>& h)
{
    VoxFetch<CM, VPL> f;
    fetch_voxels<CM, VPL, kColor>(op, base, kz0, f);
    decide_voxels<CM, VPL>(f, mu, h);
}

// ---------------------------------------------------------------------------
// voxel updates
// ---------------------------------------------------------------------------

// One RGBA8 channel: round-half-to-even of the exact rational N / M, clamped
// to [0, 255].  N and M are integers below 2^53 held exactly in FP64 and rM
// is 1/M to about 2^-52.  For a quotient below 256, N rM misses N / M by
// less than 2^-43 while a quotient that is not a tie lies at least 1/(2M) >=
// 2^-25 from every half-integer, so rint(N rM) is the correct rounding except
// at exact ties, which the exact residual N - q M identifies.
__device__ inline uint32_t mix_channel(double N, double M, double rM)
{
    const double Np = fmax(N, 0.0);
    const double q = fmin(rint(Np * rM), 256.0);
    const double two = 2.0 * fma(-q, M, Np);  // exact for q < 256: integers below 2^53
    const int k = (int)q;
    const bool tie = (two == M || two == -M) && (k & 1);
    return (uint32_t)min(k + (tie ? ((two > 0.0) ? 1 : -1) : 0), 255);
}

// Integrate (sign +1) or de-integrate (sign -1, Eq. 2) one sample into an
// RGBA8 voxel held in registers; on a weight error the voxel is left as it
// was and false is returned.  The colour is the exact rational
// (C Wq +- c wq) / W'q on the 2^-10 weight grid (every product below 2^32,
// so exact in FP64), rounded half to even.  D is the running mean in FP64:
// (D W +- d w) times the refined reciprocal of W' (the colour's reciprocal
// of W' 2^10, rescaled exactly), within two FP64 ulps of the quotient.
// Branch-free.
__device__ inline bool update_rgba8(double& D, float& W, uint32_t& C, double d, float w, uint32_t c, int sign)
{
    const float sw = (sign > 0) ? w : -w;
    const float W1 = W + sw;  // exact on the 2^-10 grid
    const bool bad = !(W1 < kWeightLimit) || W1 < 0.0f;
    const bool zero = W1 == 0.0f;
    const double M = (double)W1 * (double)kWeightScale;
    const double Wq = (double)W * (double)kWeightScale;
    const double swq = (double)sw * (double)kWeightScale;
    double rM = __builtin_amdgcn_rcp(M);
    rM = fma(rM, fma(-M, rM, 1.0), rM);
    rM = fma(rM, fma(-M, rM, 1.0), rM);
    const double D1 = (D * (double)W + d * (double)sw) * (rM * (double)kWeightScale);
    uint32_t C1 = 0u;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double N = (double)((C >> (8 * k)) & 0xFFu) * Wq + (double)((c >> (8 * k)) & 0xFFu) * swq;
        C1 |= mix_channel(N, M, rM) << (8 * k);
    }
    D = bad ? D : (zero ? 0.0 : D1);
    C = bad ? C : (zero ? 0u : C1);
    W = bad ? W : (zero ? 0.0f : W1);
    return !bad;
}

// update_rgba8 with each colour channel's quotient y = N / M first estimated
// in FP32: y' = fl(fl(c swq + fl(C Wq)) fl32(1/M)).  Below the weight limit
// Wq, swq and M are integers below 2^24, and
// |y' - y| <= 2^-24 (C Wq / M + 3 |y|) (1 + 2^-20), which is below
// E = 2^-22 (255 Wq / M + |y'| + 1).  When |y' - rint(y')| + E <= 1/2 the
// exact quotient lies strictly inside the same rounding interval, so
// rint(y') clamped to [0, 255] is the exact result; a lane with a channel
// nearer a rounding boundary (exact ties among them) takes update_rgba8's
// FP64 path.  The same results as update_rgba8, bit for bit.
__device__ inline bool update_rgba8_fast(double& D, float& W, uint32_t& C, double d, float w, uint32_t c, int sign)
{
    const float sw = (sign > 0) ? w : -w;
    const float W1 = W + sw;  // exact on the 2^-10 grid
    const bool bad = !(W1 < kWeightLimit) || W1 < 0.0f;
    const bool zero = W1 == 0.0f;
    const double M = (double)W1 * (double)kWeightScale;
    double rM = __builtin_amdgcn_rcp(M);
    rM = fma(rM, fma(-M, rM, 1.0), rM);
    rM = fma(rM, fma(-M, rM, 1.0), rM);
    const double D1 = (D * (double)W + d * (double)sw) * (rM * (double)kWeightScale);
    const float Wq = W * kWeightScale, swq = sw * kWeightScale;
    const float rMf = (float)rM;
    const float E0 = fmaf(Wq * rMf, 255.0f * 0x1p-22f, 0x1p-22f);
    uint32_t C1 = 0u;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float Ck = (float)((C >> (8 * k)) & 0xFFu), ck = (float)((c >> (8 * k)) & 0xFFu);
        const float y = fmaf(ck, swq, Ck * Wq) * rMf;
        const float q = rintf(y);
        ok = ok && (fabsf(y - q) + fmaf(fabsf(y), 0x1p-22f, E0) <= 0.5f);
        C1 |= (uint32_t)fminf(fmaxf(q, 0.0f), 255.0f) << (8 * k);
    }
    if (!(ok || bad || zero)) {
        const double Wqd = (double)Wq, swqd = (double)swq;
        C1 = 0u;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double N = (double)((C >> (8 * k)) & 0xFFu) * Wqd + (double)((c >> (8 * k)) & 0xFFu) * swqd;
            C1 |= mix_channel(N, M, rM) << (8 * k);
        }
    }
    D = bad ? D : (zero ? 0.0 : D1);
    C = bad ? C : (zero ? 0u : C1);
    W = bad ? W : (zero ? 0.0f : W1);
    return !bad;
}

// FP32-colour mode: keyframe colour FP32 in [0,1]; the voxel colour is held
// in FP64, because Eq. (2) amplifies the rounding of the stored colour by
// W / W' when most of a voxel's weight is removed (as for D).
__device__ inline bool update_f32(double& D, float& W, double C[3], double d, float w, const float c[3], int sign)
{
    const float W1 = (sign > 0) ? W + w : W - w;
    if (sign > 0 ? !(W1 < kWeightLimit) : (W1 < 0.0f)) return false;
    if (W1 == 0.0f) {
        D = 0.0;
        W = 0.0f;
        C[0] = C[1] = C[2] = 0.0;
        return true;
    }
    const double Wd = (double)W, wd = (double)w, W1d = (double)W1;
    D = (sign > 0 ? (D * Wd + d * wd) : (D * Wd - d * wd)) / W1d;
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

// Operations of a block in bit order, read word by word from its mask.
struct OpWalk {
    const uint64_t* mask;
    int words, w;
    uint64_t m;
};

__device__ inline int walk_next(OpWalk& k)
{
    while (k.m == 0ull) {
        if (++k.w >= k.words) return -1;
        k.m = bcast64(k.mask[k.w]);
    }
    const int b = __ffsll((unsigned long long)k.m) - 1;
    k.m &= k.m - 1;
    return k.w * 64 + b;
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


// Candidate generation works on square pixel tiles with one CELL x CELL pixel
// cell per thread: 64 x 64 tiles of 4 x 4 cells for the batched path, where
// many operations fill the GPU, and 32 x 32 tiles of 2 x 2 quads for the one
// operation of a plain-path call (256 threads either way).
constexpr int kTileBatch = 64, kCellBatch = 4;
constexpr int kTilePlain = 32, kCellPlain = 2;
// A merged cell widens the depth band of each of its pixels by the cell's
// depth spread; these bounds (in units of mu) keep the extra candidates few.
constexpr float kCellSpread = 1.0f, kQuadSpread = 2.0f;

template <int TILE, int CELL>
struct CandCfg {
    static constexpr int threads = (TILE / CELL) * (TILE / CELL);
    static constexpr int lds_set = 2048;  // LDS hash set entries per tile
};

// Frustum cell of a pixel rectangle [u0, u1] x [v0, v1], widened by 0.55 px
// on every side: normalised image coordinates x in [xm - hx, xm + hx] and
// y in [ym - hy, ym + hy], camera depth in [zl, zh] (the band
// [zlo - mu, zhi + mu], padded so that FP32 rounding in the decision
// convention cannot escape it).  The reciprocals ifx = 1/fx and ify = 1/fy
// may carry a few ulps of error: the 0.05 px padding exceeds their effect by
// orders of magnitude.
struct CellGeom {
    float xm, ym, hx, hy, zl, zh;
};

__device__ inline CellGeom cell_geom(const OpDesc& op, float ifx, float ify, float mu, int u0, int u1, int v0, int v1,
                                     float zlo, float zhi)
{
    CellGeom c;
    const float xl = ((float)u0 - 0.55f - op.cx) * ifx, xh = ((float)u1 + 0.55f - op.cx) * ifx;
    const float yl = ((float)v0 - 0.55f - op.cy) * ify, yh = ((float)v1 + 0.55f - op.cy) * ify;
    c.xm = 0.5f * (xl + xh);
    c.hx = 0.5f * (xh - xl);
    c.ym = 0.5f * (yl + yh);
    c.hy = 0.5f * (yh - yl);
    c.zl = fmaxf(zlo - mu - 1e-3f, 0.0f);
    c.zh = zhi + mu + 1e-3f;
    return c;
}

// Conservative world-space block range of a cell's frustum (the box of its
// eight corners, padded); false if the cell spans 16 blocks or more along an
// axis (a depth far beyond the voxel scale) or leaves the key range.
__device__ inline bool cell_block_range(const OpDesc& op, float is, const CellGeom& c, int lo[3], int hi[3])
{
    float mn[3], mx[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        mn[r] = 3.0e38f;
        mx[r] = -3.0e38f;
    }
#pragma unroll
    for (int iz = 0; iz < 2; ++iz) {
        const float zz = iz ? c.zh : c.zl;
        const float cxm = c.xm * zz, hx = c.hx * zz;
        const float cym = c.ym * zz, hy = c.hy * zz;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const float r0 = (float)op.R[3 * r + 0], r1 = (float)op.R[3 * r + 1], r2 = (float)op.R[3 * r + 2];
            const float cc = r0 * cxm + r1 * cym + r2 * zz + (float)op.t[r];
            const float e = fabsf(r0) * hx + fabsf(r1) * hy;
            mn[r] = fminf(mn[r], cc - e);
            mx[r] = fmaxf(mx[r], cc + e);
        }
    }
    bool ok = true;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float pad = 2e-3f + 2e-5f * fmaxf(fabsf(mn[r]), fabsf(mx[r]));
        const float flo = ceilf((mn[r] - pad) * is);
        const float fhi = floorf((mx[r] + pad) * is);
        ok = ok && (flo > -8.0e6f) && (fhi < 8.0e6f) && (fhi - flo < 128.0f);
        lo[r] = ok ? ((int)flo >> 3) : 0;  // arithmetic shift: floor division by 8
        hi[r] = ok ? ((int)fhi >> 3) : -1;
    }
    return ok;
}

// Sets operation bit `op_bit` of a candidate's mask: a non-returning atomic,
// so the wavefront does not wait for it.
__device__ inline void cand_mark(const CandDev& cd, int gb, int op_bit)
{
    uint64_t* mw = cd.mask + (size_t)gb * cd.words + (op_bit >> 6);
    atomicOr((unsigned long long*)mw, (unsigned long long)(1ull << (op_bit & 63)));
}

// Finds or inserts a candidate block in the deduplicating candidate table;
// returns its bucket, or -1 if the table is full (sticky error set).  `fresh`
// is set when this call inserted the key (the caller then appends the bucket
// to the candidate list).  Keys only go from empty to a block within a
// kernel, so a plain read that finds the key is reliable, and the CAS is
// issued only at an empty-looking bucket.
__device__ inline int cand_claim(const CandDev& cd, const VolDev& v, uint64_t key, int bx, int by, int bz, bool& fresh)
{
    fresh = false;
    uint32_t h = hash_block(bx, by, bz) & cd.mask_bits;
    for (uint32_t probe = 0; probe <= cd.mask_bits; ++probe) {
        const uint64_t seen = cd.keys[h];
        if (seen == key) return (int)h;
        if (seen == kKeyEmpty) {
            const uint64_t old = atomicCAS((unsigned long long*)(cd.keys + h), (unsigned long long)kKeyEmpty,
                                           (unsigned long long)key);
            if (old == key) return (int)h;
            if (old == kKeyEmpty) {
                fresh = true;
                return (int)h;
            }
        }
        h = (h + 1) & cd.mask_bits;
    }
    set_error(v.err, SC_EHASHFULL);
    return -1;
}

__device__ inline void cand_append(const CandDev& cd, const VolDev& v, uint32_t idx, int gb)
{
    if (idx < cd.cap)
        cd.list[idx] = (uint32_t)gb;
    else
        set_error(v.err, SC_EHASHFULL);
}

// Per-lane insertion with its own list append (the rare LDS-overflow path;
// no list when count is null).
__device__ inline int cand_insert(const CandDev& cd, const VolDev& v, uint64_t key, int bx, int by, int bz,
                                  uint32_t* count)
{
    bool fresh;
    const int gb = cand_claim(cd, v, key, bx, by, bz, fresh);
    if (fresh && count) cand_append(cd, v, atomicAdd(count, 1u), gb);
    return gb;
}

// LDS slot of a block: low coordinate bits, no multiplies (a tile's blocks
// form a small box, so the low bits spread them).
__device__ inline uint32_t lds_slot(int bx, int by, int bz)
{
    return ((uint32_t)bx & 15u) | (((uint32_t)by & 15u) << 4) | (((uint32_t)bz & 7u) << 8);
}

template <int SET>
__device__ inline void lds_insert(uint64_t* lds, const CandDev& cd, const VolDev& v, uint32_t* count, int op_bit,
                                  int bx, int by, int bz)
{
    const uint64_t key = pack_key(bx, by, bz);
    uint32_t h = lds_slot(bx, by, bz) & (SET - 1);
    for (int probe = 0; probe < 32; ++probe) {
        // most inserts repeat a key already present: a plain read settles
        // them without a serialising atomic (entries only go from empty to a
        // key while the set is filled)
        const uint64_t seen = lds[h];
        if (seen == key) return;
        if (seen == kKeyEmpty) {
            const uint64_t old =
                atomicCAS((unsigned long long*)(lds + h), (unsigned long long)kKeyEmpty, (unsigned long long)key);
            if (old == kKeyEmpty || old == key) return;
        }
        h = (h + 1) & (SET - 1);
    }
    const int gb = cand_insert(cd, v, key, bx, by, bz, count);
    if (gb >= 0 && op_bit >= 0) cand_mark(cd, gb, op_bit);
}

// Inserts the blocks that can meet the frustum cell of pixels [u0, u1] x
// [v0, v1] with valid depths in [zlo, zhi]; false if the cell's range is out
// of bounds (nothing inserted).
template <int SET>
__device__ inline bool insert_cell(uint64_t* lds, const CandDev& cd, const VolDev& v, uint32_t* count, int op_bit,
                                   const OpDesc& op, float ifx, float ify, float is, int u0,
                                   int u1, int v0, int v1, float zlo, float zhi)
{
    const CellGeom c = cell_geom(op, ifx, ify, v.mu, u0, u1, v0, v1, zlo, zhi);
    int lo[3], hi[3];
    if (!cell_block_range(op, is, c, lo, hi)) return false;
    for (int bx = lo[0]; bx <= hi[0]; ++bx)
        for (int by = lo[1]; by <= hi[1]; ++by)
            for (int bz = lo[2]; bz <= hi[2]; ++bz) lds_insert<SET>(lds, cd, v, count, op_bit, bx, by, bz);
    return true;
}

// Per-pixel fallback of a cell spanning a depth discontinuity.
template <int SET>
__device__ inline void insert_pixels(uint64_t* lds, const CandDev& cd, const VolDev& v, uint32_t* count, int op_bit,
                                     const OpDesc& op, float ifx, float ify, float is, int u,
                                     int vv, float z)
{
    if (!insert_cell<SET>(lds, cd, v, count, op_bit, op, ifx, ify, is, u, u, vv, vv, z, z))
        set_error(v.err, SC_ERANGE);
}

// The per-thread part of cand_tile (4 x 4 cells) for a packed keyframe: the
// cell's depth range comes from the packed cell ranges, and a cell that is
// not one frustum cell reads its 2 x 2 quads' depths from the packed records
// (depth' is -inf where the quantised weight is zero, so 0 < depth' < 1e30
// is the validity test of the pixel path).  The same decisions and boxes as
// the pixel path, without the cell's 16 depths in registers.  `ins.cell`
// inserts the blocks of one frustum cell's box (false: the box is out of
// range, nothing inserted).
template <class Ins>
__device__ inline void cell_inserts_packed(const OpDesc& op, const VolDev& v, Ins& ins, int u0, int v0)
{
    const int cw = (op.width + 3) >> 2, ch = (op.height + 3) >> 2;
    const int cx = u0 >> 2, cy = v0 >> 2;
    if (cx >= cw || cy >= ch) return;
    const float2 r = op.cells[cy * cw + cx];
    if (!(r.x <= r.y)) return;  // no valid pixel
    if (r.y - r.x <= kCellSpread * v.mu && ins.cell(u0, u0 + 3, v0, v0 + 3, r.x, r.y)) return;
    const uint32_t* rec = reinterpret_cast<const uint32_t*>(op.packed);
    for (int qd = 0; qd < 4; ++qd) {
        const int qu = u0 + 2 * (qd & 1), qv = v0 + 2 * (qd >> 1);
        float z[4];
        uint32_t qvalid = 0u;
        float qmin = 3.0e38f, qmax = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int u = qu + (k & 1), vv = qv + (k >> 1);
            z[k] = 0.0f;
            if (u < op.width && vv < op.height) {
                const float zz = __uint_as_float(rec[4 * ((size_t)vv * op.width + u)]);
                if (zz > 0.0f && zz < 1.0e30f) {
                    qvalid |= 1u << k;
                    z[k] = zz;
                    qmin = fminf(qmin, zz);
                    qmax = fmaxf(qmax, zz);
                }
            }
        }
        if (!qvalid) continue;
        if (qmax - qmin <= kQuadSpread * v.mu && ins.cell(qu, qu + 1, qv, qv + 1, qmin, qmax)) continue;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if ((qvalid >> k) & 1u) {
                const int u = qu + (k & 1), vv = qv + (k >> 1);
                if (!ins.cell(u, u, vv, vv, z[k], z[k])) set_error(v.err, SC_ERANGE);
            }
    }
}

// Box inserter of the LDS hash set (insert_cell).
template <int SET>
struct HashIns {
    uint64_t* lds;
    const CandDev& cd;
    const VolDev& v;
    uint32_t* count;
    int op_bit;
    const OpDesc& op;
    float ifx, ify, is;
    __device__ bool cell(int u0, int u1, int v0, int v1, float zlo, float zhi)
    {
        return insert_cell<SET>(lds, cd, v, count, op_bit, op, ifx, ify, is, u0, u1, v0, v1, zlo, zhi);
    }
};

// Candidate tiles of packed keyframes on an LDS bit map over the tile's block
// box: the box of the whole tile's frustum (its pixels between the smallest
// depth less mu and the largest plus mu) contains every frustum cell's box,
// so a cell's blocks are bits of a bit map over it, set a z-run at a time
// (one or two LDS ORs instead of one probed insert per block); the set bits
// are then claimed in the global candidate table.  A tile whose box exceeds
// kTileBits blocks takes the LDS hash set.
constexpr int kTileBits = 65536;  // 8 KB

// The tile's block box: as cell_block_range without its size limit, widened
// by one block on every side (so that the cells' own FP32 boxes, padded the
// same way, lie inside it); false if it leaves the key range or exceeds
// kTileBits blocks.
__device__ inline bool tile_block_box(const OpDesc& op, float is, const CellGeom& c, int lo[3], int n[3])
{
    float mn[3], mx[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        mn[r] = 3.0e38f;
        mx[r] = -3.0e38f;
    }
#pragma unroll
    for (int iz = 0; iz < 2; ++iz) {
        const float zz = iz ? c.zh : c.zl;
        const float cxm = c.xm * zz, hx = c.hx * zz;
        const float cym = c.ym * zz, hy = c.hy * zz;
#pragma unroll
        for (int r = 0; r < 3; ++r) {
            const float r0 = (float)op.R[3 * r + 0], r1 = (float)op.R[3 * r + 1], r2 = (float)op.R[3 * r + 2];
            const float cc = r0 * cxm + r1 * cym + r2 * zz + (float)op.t[r];
            const float e = fabsf(r0) * hx + fabsf(r1) * hy;
            mn[r] = fminf(mn[r], cc - e);
            mx[r] = fmaxf(mx[r], cc + e);
        }
    }
    bool ok = true;
    int vol = 1;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        const float pad = 2e-3f + 2e-5f * fmaxf(fabsf(mn[r]), fabsf(mx[r]));
        const float flo = ceilf((mn[r] - pad) * is);
        const float fhi = floorf((mx[r] + pad) * is);
        ok = ok && (flo > -8.0e6f) && (fhi < 8.0e6f) && (fhi - flo < 8.0f * 1024.0f);
        lo[r] = ok ? ((int)flo >> 3) - 1 : 0;
        n[r] = ok ? ((int)fhi >> 3) + 1 - lo[r] + 1 : 1;
        vol *= n[r];
    }
    return ok && vol <= kTileBits;
}

// Box inserter of the bit map: a cell box inside the tile box sets its
// z-runs; one outside it (not expected: the tile box is a block wider) goes
// block by block to the global table.
struct BitIns {
    uint32_t* bits;
    const CandDev& cd;
    const VolDev& v;
    int op_bit;
    const OpDesc& op;
    float ifx, ify, is;
    int tlo[3], tn[3];
    __device__ bool cell(int u0, int u1, int v0, int v1, float zlo, float zhi)
    {
        const CellGeom c = cell_geom(op, ifx, ify, v.mu, u0, u1, v0, v1, zlo, zhi);
        int lo[3], hi[3];
        if (!cell_block_range(op, is, c, lo, hi)) return false;
        bool inside = true;
#pragma unroll
        for (int r = 0; r < 3; ++r) inside = inside && lo[r] >= tlo[r] && hi[r] < tlo[r] + tn[r];
        if (!inside) {
            for (int bx = lo[0]; bx <= hi[0]; ++bx)
                for (int by = lo[1]; by <= hi[1]; ++by)
                    for (int bz = lo[2]; bz <= hi[2]; ++bz) {
                        const int gb = cand_insert(cd, v, pack_key(bx, by, bz), bx, by, bz, nullptr);
                        if (gb >= 0) cand_mark(cd, gb, op_bit);
                    }
            return true;
        }
        const int run = hi[2] - lo[2] + 1;  // at most 16 blocks
        const uint32_t m = (run >= 32) ? ~0u : ((1u << run) - 1u);
        for (int bx = lo[0]; bx <= hi[0]; ++bx)
            for (int by = lo[1]; by <= hi[1]; ++by) {
                const int first = ((bx - tlo[0]) * tn[1] + (by - tlo[1])) * tn[2] + (lo[2] - tlo[2]);
                const int w = first >> 5, b = first & 31;
                atomicOr(bits + w, m << b);
                if (b + run > 32) atomicOr(bits + w + 1, m >> (32 - b));
            }
        return true;
    }
};

// Bit-map candidate generation for one TILE x TILE tile of a packed keyframe
// (4 x 4 cells); returns false when the tile's box is too large (nothing
// done: the caller takes the hash set).  `red` holds 8 floats of LDS.
template <int TILE>
__device__ inline bool cand_tile_bits(const OpDesc& op, const VolDev& v, const CandDev& cd, int tx, int ty, int op_bit,
                                      uint32_t* bits, uint16_t* idx, float* red)
{
    constexpr int kCells = TILE / 4;
    constexpr int kThreads = kCells * kCells;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int u0 = tx * TILE + 4 * (tid % kCells);
    const int v0 = ty * TILE + 4 * (tid / kCells);
    const float ifx = 1.0f / op.fx, ify = 1.0f / op.fy, is = 1.0f / v.s;
    // the tile's depth range from its cells' ranges
    const int cw = (op.width + 3) >> 2, ch = (op.height + 3) >> 2;
    const int cx = u0 >> 2, cy = v0 >> 2;
    const float2 r = (cx < cw && cy < ch) ? op.cells[cy * cw + cx] : make_float2(1.0f, 0.0f);
    const bool any = r.x <= r.y;
    float zlo = any ? r.x : 3.0e38f, zhi = any ? r.y : 0.0f;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        zlo = fminf(zlo, __shfl_xor(zlo, o));
        zhi = fmaxf(zhi, __shfl_xor(zhi, o));
    }
    if (lane == 0) {
        red[2 * wave] = zlo;
        red[2 * wave + 1] = zhi;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        zlo = fminf(zlo, red[2 * w]);
        zhi = fmaxf(zhi, red[2 * w + 1]);
    }
    if (!(zlo <= zhi)) return true;  // no valid pixel in the tile
    // the whole tile's pixel rectangle (cells at a ragged border reach past
    // the image just as far)
    const CellGeom tg =
        cell_geom(op, ifx, ify, v.mu, tx * TILE, tx * TILE + TILE - 1, ty * TILE, ty * TILE + TILE - 1, zlo, zhi);
    BitIns ins{bits, cd, v, op_bit, op, ifx, ify, is, {0, 0, 0}, {1, 1, 1}};
    if (!tile_block_box(op, is, tg, ins.tlo, ins.tn)) return false;
    const int nw = (ins.tn[0] * ins.tn[1] * ins.tn[2] + 31) >> 5;
    for (int w = tid; w < nw; w += kThreads) bits[w] = 0u;
    __syncthreads();
    cell_inserts_packed(op, v, ins, u0, v0);
    __syncthreads();
    // claims: each wavefront compacts the set bits of 16 words at a time into
    // its index list (at most 512 entries) and claims the list 64 at a time
    uint16_t* wl = idx + wave * 512;
    const int nyz = ins.tn[1] * ins.tn[2];
    int n = 0;
    auto claim = [&](int cnt) {
        for (int r0 = 0; r0 < cnt; r0 += 64) {
            const int q = r0 + lane;
            if (q < cnt) {
                const int e = wl[q];
                const int bx = ins.tlo[0] + e / nyz;
                const int rem = e - (e / nyz) * nyz;
                const int by = ins.tlo[1] + rem / ins.tn[2];
                const int bz = ins.tlo[2] + rem - (rem / ins.tn[2]) * ins.tn[2];
                bool fresh;
                const int gb = cand_claim(cd, v, pack_key(bx, by, bz), bx, by, bz, fresh);
                if (gb >= 0) cand_mark(cd, gb, op_bit);
            }
        }
        wave_lds_sync();
    };
    for (int base = wave * 16; base < nw; base += 16 * (kThreads / 64)) {
        const int w = base + lane;
        uint32_t m = (lane < 16 && w < nw) ? bits[w] : 0u;
        const uint32_t c = (uint32_t)__popc(m);
        uint32_t pre = c;  // inclusive prefix over the lanes
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t y = __shfl_up(pre, o);
            pre += (lane >= o) ? y : 0u;
        }
        const int total = (int)__shfl(pre, 63);
        if (n + total > 512) {
            claim(n);
            n = 0;
        }
        int pos = n + (int)(pre - c);
        while (m) {
            const int b = __ffs(m) - 1;
            m &= m - 1u;
            wl[pos++] = (uint16_t)(w * 32 + b);
        }
        n += total;
        wave_lds_sync();
    }
    claim(n);
    return true;
}

// Candidate generation for one TILE x TILE tile of one keyframe operation,
// one CELL x CELL pixel cell per thread (CELL 2 or 4).  A cell whose valid
// depths lie within kCellSpread mu of each other is treated as one frustum
// cell; otherwise (CELL 4) each of its 2 x 2 quads is (within kQuadSpread mu),
// and what still spans a depth difference falls back to single pixels.  The
// blocks of the frustum cells' boxes are deduplicated in an LDS hash set, then
// inserted once per
// tile into the global candidate table; with op_bit >= 0 the operation's bit
// is set in the block's mask.  With count non-null, new candidates are also
// appended to the candidate list (the plain path); the batched path finds
// them by scanning the table instead.
template <int TILE, int CELL, bool kFromCells = false>
__device__ inline void cand_tile(const OpDesc& op, const VolDev& v, const CandDev& cd, uint32_t* count, int tx,
                                 int ty, int op_bit, uint64_t* lds, uint16_t* idx)
{
    constexpr int kCells = TILE / CELL;
    constexpr int kThreads = CandCfg<TILE, CELL>::threads;
    constexpr int kSet = CandCfg<TILE, CELL>::lds_set;
    constexpr int kPix = CELL * CELL;
    const int tid = threadIdx.x;
    for (int i = tid; i < kSet; i += kThreads) lds[i] = kKeyEmpty;
    __syncthreads();
    const int u0 = tx * TILE + CELL * (tid % kCells);
    const int v0 = ty * TILE + CELL * (tid / kCells);
    const float ifx = 1.0f / op.fx, ify = 1.0f / op.fy, is = 1.0f / v.s;
    if (kFromCells) {
        HashIns<kSet> ins{lds, cd, v, count, op_bit, op, ifx, ify, is};
        cell_inserts_packed(op, v, ins, u0, v0);
    } else {
    float zc[kPix];
    uint32_t valid = 0u;
    float zmin = 3.0e38f, zmax = 0.0f;
#pragma unroll
    for (int q = 0; q < kPix; ++q) {
        const int u = u0 + (q % CELL), vv = v0 + (q / CELL);
        zc[q] = 0.0f;
        if (u < op.width && vv < op.height) {
            const int pix = vv * op.width + u;
            const float w = qweight(op.weight[pix]);
            const float z = op.depth[pix];
            if (w > 0.0f && z > 0.0f && z < 1.0e30f) {
                valid |= 1u << q;
                zc[q] = z;
                zmin = fminf(zmin, z);
                zmax = fmaxf(zmax, z);
            }
        }
    }
    if (valid) {
        bool done = false;
        if (zmax - zmin <= (CELL == 4 ? kCellSpread : kQuadSpread) * v.mu)
            done = insert_cell<kSet>(lds, cd, v, count, op_bit, op, ifx, ify, is, u0, u0 + CELL - 1, v0,
                                     v0 + CELL - 1, zmin, zmax);
        if (!done && CELL == 4) {
            for (int qd = 0; qd < 4; ++qd) {
                const int qu = u0 + 2 * (qd & 1), qv = v0 + 2 * (qd >> 1);
                const int q0 = 2 * (qd & 1) + 2 * CELL * (qd >> 1);  // first pixel of the quad in zc
                const int idx[4] = {q0, q0 + 1, q0 + CELL, q0 + CELL + 1};
                float qmin = 3.0e38f, qmax = 0.0f;
                uint32_t qvalid = 0u;
                for (int k = 0; k < 4; ++k)
                    if ((valid >> idx[k]) & 1u) {
                        qvalid |= 1u << k;
                        qmin = fminf(qmin, zc[idx[k]]);
                        qmax = fmaxf(qmax, zc[idx[k]]);
                    }
                if (!qvalid) continue;
                if (qmax - qmin <= kQuadSpread * v.mu &&
                    insert_cell<kSet>(lds, cd, v, count, op_bit, op, ifx, ify, is, qu, qu + 1, qv, qv + 1, qmin,
                                      qmax))
                    continue;
                for (int k = 0; k < 4; ++k)
                    if ((qvalid >> k) & 1u)
                        insert_pixels<kSet>(lds, cd, v, count, op_bit, op, ifx, ify, is, qu + (k & 1),
                                            qv + (k >> 1), zc[idx[k]]);
            }
        } else if (!done) {
            for (int q = 0; q < kPix; ++q)
                if ((valid >> q) & 1u)
                    insert_pixels<kSet>(lds, cd, v, count, op_bit, op, ifx, ify, is, u0 + (q % CELL),
                                        v0 + (q / CELL), zc[q]);
        }
    }
    }
    __syncthreads();
    // insert the tile's blocks: each wavefront first compacts the occupied
    // entries of its part of the set into its index list (about one in twenty
    // is occupied), then claims them 64 at a time, so it waits for about one
    // claim latency rather than one per round holding an occupied entry; new
    // candidates are appended with one atomic per wavefront (the claim loop's
    // trip count is the same for every lane)
    const int lane = tid & 63;
    constexpr int kRounds = kSet / kThreads;
    uint16_t* wl = idx + (tid >> 6) * (kRounds * 64);
    int n = 0;
#pragma unroll
    for (int it = 0; it < kRounds; ++it) {
        const int e = tid + it * kThreads;
        const bool occ = lds[e] != kKeyEmpty;
        const uint64_t bal = __ballot(occ);
        if (occ) wl[n + (int)lanes_below(bal)] = (uint16_t)e;
        n += __popcll(bal);
    }
    wave_lds_sync();
    for (int r0 = 0; r0 < n; r0 += 64) {
        const int r = r0 + lane;
        bool fresh = false;
        int gb = -1;
        if (r < n) {
            const uint64_t key = lds[wl[r]];
            int bx, by, bz;
            unpack_key(key, bx, by, bz);
            gb = cand_claim(cd, v, key, bx, by, bz, fresh);
            if (gb >= 0 && op_bit >= 0) cand_mark(cd, gb, op_bit);
        }
        if (count) {
            const uint64_t bal = __ballot(fresh);
            if (bal) {
                const uint32_t base = wave_fetch_add(count, (uint32_t)__popcll(bal), lane);
                if (fresh) cand_append(cd, v, base + lanes_below(bal), gb);
            }
        }
    }
}

}  // namespace sc
