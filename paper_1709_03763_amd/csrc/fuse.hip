// Keyframe fusion (Sec. 3, "Keyframe Fusion"; Eq. 1).
//
//   depth_weight   w_z = cos(theta) Z^-2 per pixel, quantised to 2^-10, with
//                  rejection near depth discontinuities
//   warp_kernel    forward warp of every surviving pixel into the keyframe,
//                  p* = g(T*^-1, g(T_i, pi^-1(x, Z_i(x)))), accumulated at the
//                  nearest pixel of pi(p*) in exact int64 fixed point (w on the
//                  2^-10 grid, z on the 2^-20 m grid), so that colliding
//                  atomics cannot change a bit; Eq. 1's running weighted mean
//                  equals sum(w z) / sum(w)
//   color_prep     unsharp mask C + (C - G * C), G the binomial [1 4 6 4 1]/16
//                  kernel, exact in units of 1/256, and the re-blur measure's
//                  integer luminance sums (exact int64 per-tile partials)
//   blur_final     per-frame sums of the partials and w_b (inside the
//                  depth-weight launch when fusing)
//   color_kernel   the keyframe depth and weight from the accumulators, then
//                  the back-warp of each keyframe pixel into every frame,
//                  bilinear sample of the sharpened colour, weight w_b * w_z,
//                  per-channel lower weighted median
//
// A fusion is four launches: colour prep, depth weight (which also forms
// w_b from the colour-prep partials, clears the accumulators and stores the
// relative poses, passed to it as arguments), warp and colour.
//
// Decisions are FP32 with the written operation order (-ffp-contract=off).
#include <string.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace sc {

constexpr int kMaxFrames = 64;

struct FuseFrames {
    float Rf[kMaxFrames][12];  // forward: T*^-1 T_i, rows of R then t
    float Rb[kMaxFrames][12];  // backward: T_i^-1 T*
};

// Relative poses passed by value, kStageFrames frames per launch, so that no
// host staging buffer or copy is needed.
constexpr int kStageFrames = 32;
struct PoseChunk {
    float Rf[kStageFrames][12];
    float Rb[kStageFrames][12];
};

// Work of one fusion done by the depth-weight launch, which follows the
// colour prep and precedes the warp and colour kernels on its stream: frame
// 0's workgroups clear the fixed-point accumulators of their tile's pixels,
// workgroup (0, 0) stores the first `count` relative poses, and the first
// workgroup of each frame adds up that frame's colour-prep partials into w_b.
// Null pointers and count 0 skip it (the standalone depth weight).
struct FuseInit {
    unsigned long long* acc;  // KW then KZ, 2 x H W
    const long long* parts;   // colour-prep partials, 4 per tile and frame
    double* wb;               // w_b per frame
    int32_t prep_tiles;       // colour-prep tiles per frame
    FuseFrames* fr;
    int32_t count;
    PoseChunk poses;
};

__device__ inline bool zvalid(float z, float zmin, float zmax) { return z >= zmin && z <= zmax; }

__device__ inline void backproject(float u, float v, float z, const sc_intrinsics& in, float P[3])
{
    P[0] = ((u - in.cx) * z) / in.fx;
    P[1] = ((v - in.cy) * z) / in.fy;
    P[2] = z;
}

__device__ inline void xform(const float* T, const float P[3], float q[3])
{
#pragma unroll
    for (int r = 0; r < 3; ++r) q[r] = ((T[3 * r + 0] * P[0] + T[3 * r + 1] * P[1]) + T[3 * r + 2] * P[2]) + T[9 + r];
}

__device__ inline bool project(const sc_intrinsics& in, const float q[3], float& uf, float& vf, int& iu, int& iv)
{
    if (!(q[2] > 0.0f)) return false;
    uf = (in.fx * q[0]) / q[2] + in.cx;
    vf = (in.fy * q[1]) / q[2] + in.cy;
    const float fu = floorf(uf + 0.5f), fv = floorf(vf + 0.5f);
    if (!(fu >= 0.0f && fu <= (float)(in.width - 1) && fv >= 0.0f && fv <= (float)(in.height - 1))) return false;
    iu = (int)fu;
    iv = (int)fv;
    return true;
}

// One frame's tile partials (4 exact int64 sums per tile) added up by a
// 256-thread workgroup, then w_b = 1 - max(blur_h, blur_v) in FP64 (the
// integer sums are exact, so the order of the additions does not matter).
__device__ inline void blur_reduce(const long long* p, int tiles, long long (*red)[4], double* wb)
{
    long long acc[4] = {0, 0, 0, 0};
    for (int t = threadIdx.x; t < tiles; t += blockDim.x)
#pragma unroll
        for (int k = 0; k < 4; ++k) acc[k] += p[(size_t)t * 4 + k];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        for (int o = 32; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();  // `red` may still be read from the caller's own reduction
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) red[wave][k] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
        long long s[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) s[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
        const double bh = s[0] > 0 ? (double)(s[0] - s[1]) / (double)s[0] : 0.0;
        const double bv = s[2] > 0 ? (double)(s[2] - s[3]) / (double)s[2] : 0.0;
        *wb = 1.0 - (bh > bv ? bh : bv);
    }
}

// ---------------------------------------------------------------------------
// depth weight
// ---------------------------------------------------------------------------

// One 64 x 16 tile per workgroup: the back-projection of every pixel of the
// tile and a one-pixel halo is computed once into LDS (two divisions per
// pixel), and each pixel reads its four neighbours' points from there; the
// operations are those of the per-pixel definition, so the result is the
// same bit for bit.
constexpr int kDwTW = 64, kDwTH = 16;
constexpr int kDwLW = kDwTW + 2, kDwLH = kDwTH + 2;
constexpr int kDwStage = (kDwLW * kDwLH + 255) / 256;  // staged pixels per thread (256 threads)

__global__ __launch_bounds__(256) void depth_weight_kernel(const float* __restrict__ Z, int n, sc_intrinsics in,
                                                           sc_fuse_params p, int tiles_x, int tiles,
                                                           float* __restrict__ wz, const FuseInit init)
{
    __shared__ float sx[kDwLH][kDwLW], sy[kDwLH][kDwLW], sz[kDwLH][kDwLW];
    const int W = in.width, H = in.height;
    const int64_t np = (int64_t)W * H;
    const int f = blockIdx.y, tile = blockIdx.x;
    if (f >= n || tile >= tiles) return;
    const int u0 = (tile % tiles_x) * kDwTW, v0 = (tile / tiles_x) * kDwTH;
    if (f == 0 && tile == 0) {
        for (int i = threadIdx.x; i < init.count * 12; i += blockDim.x) {
            init.fr->Rf[i / 12][i % 12] = init.poses.Rf[i / 12][i % 12];
            init.fr->Rb[i / 12][i % 12] = init.poses.Rb[i / 12][i % 12];
        }
    }
    const float* Zf = Z + (size_t)f * np;
    // staging: every depth load of a thread issues before the divisions
    float zs[kDwStage];
#pragma unroll
    for (int k = 0; k < kDwStage; ++k) {
        const int q = (int)threadIdx.x + 256 * k;
        const int uu = u0 - 1 + q % kDwLW, vv = v0 - 1 + q / kDwLW;
        zs[k] = (q < kDwLW * kDwLH && uu >= 0 && uu < W && vv >= 0 && vv < H) ? Zf[(size_t)vv * W + uu] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kDwStage; ++k) {
        const int q = (int)threadIdx.x + 256 * k;
        if (q < kDwLW * kDwLH) {
            const int i = q % kDwLW, j = q / kDwLW;
            const int uu = u0 - 1 + i, vv = v0 - 1 + j;
            float P[3] = {0.0f, 0.0f, 0.0f};
            if (uu >= 0 && uu < W && vv >= 0 && vv < H) backproject((float)uu, (float)vv, zs[k], in, P);
            sx[j][i] = P[0];
            sy[j][i] = P[1];
            sz[j][i] = P[2];
        }
    }
    __syncthreads();
    const int tx = threadIdx.x & (kDwTW - 1), ty = threadIdx.x / kDwTW;
    const int u = u0 + tx, i = tx + 1;
#pragma unroll 1
    for (int r = 0; r < kDwTH / 4; ++r) {
        const int v = v0 + ty + 4 * r, j = ty + 4 * r + 1;
        if (u >= W || v >= H) continue;
        float out = 0.0f;
        const float z = sz[j][i];
        if (zvalid(z, p.z_min, p.z_max) && u >= 1 && u <= W - 2 && v >= 1 && v <= H - 2) {
            const float zl = sz[j][i - 1], zr = sz[j][i + 1], zu = sz[j - 1][i], zd = sz[j + 1][i];
            const bool ok = zvalid(zl, p.z_min, p.z_max) && zvalid(zr, p.z_min, p.z_max) &&
                            zvalid(zu, p.z_min, p.z_max) && zvalid(zd, p.z_min, p.z_max);
            const float th = p.disc_rel * z;
            if (ok && !(fabsf(zl - z) > th) && !(fabsf(zr - z) > th) && !(fabsf(zu - z) > th) &&
                !(fabsf(zd - z) > th)) {
                // neighbours (u - 1, v), (u + 1, v), (u, v - 1), (u, v + 1)
                const float a0 = sx[j][i + 1] - sx[j][i - 1], a1 = sy[j][i + 1] - sy[j][i - 1], a2 = zr - zl;
                const float b0 = sx[j + 1][i] - sx[j - 1][i], b1 = sy[j + 1][i] - sy[j - 1][i], b2 = zd - zu;
                const float nx = a1 * b2 - a2 * b1;
                const float ny = a2 * b0 - a0 * b2;
                const float nz = a0 * b1 - a1 * b0;
                const float nn = (nx * nx + ny * ny) + nz * nz;
                if (nn > 0.0f) {
                    const float c = fabsf(nz) / sqrtf(nn);
                    const float w = c / (z * z);
                    out = rintf(w * kWeightScale) / kWeightScale;
                }
            }
        }
        wz[(size_t)f * np + (size_t)v * W + u] = out;
        if (init.acc && f == 0) {
            init.acc[(size_t)v * W + u] = 0ull;
            init.acc[np + (size_t)v * W + u] = 0ull;
        }
    }
    if (init.parts && tile == 0) {
        __shared__ long long red[4][4];
        blur_reduce(init.parts + (size_t)f * init.prep_tiles * 4, init.prep_tiles, red, init.wb + f);
    }
}

// ---------------------------------------------------------------------------
// depth fusion
// ---------------------------------------------------------------------------

// The warp by target tiles.  Workgroup k owns the 16 x 16 tile k of
// keyframe pixels (on a grid extended by kWpE tiles on each side) and, for
// each frame f, the source tile k shifted back by that frame's displacement
// d_f: the image centre back-projected at depth z_nom, moved into the
// keyframe and projected, rounded to whole pixels and clamped to +-kWpD.
// Every workgroup computes the same d_f, and a whole-pixel shift of the tile
// grid still covers each frame's pixels exactly once, so every sample is
// warped once whatever d_f is; d_f only decides how many land near the
// tile.  The samples are first added into an LDS window of keyframe pixels
// (the tile and kWpM pixels on each side); each window pixel that received
// any then goes to the device-wide accumulators with one pair of atomics,
// and samples that land outside the window go there directly.  The sums are
// exact integers, so the grouping does not change them.
constexpr int kWpT = 16, kWpM = 8, kWpL = kWpT + 2 * kWpM;
constexpr int kWpE = 4, kWpD = kWpE * kWpT;

__global__ __launch_bounds__(256) void warp_kernel(const float* __restrict__ Z, const float* __restrict__ wz, int n,
                                                   sc_intrinsics in, float z_nom, int tiles_x,
                                                   const FuseFrames* __restrict__ fr, unsigned long long* KW,
                                                   unsigned long long* KZ)
{
    __shared__ unsigned long long lw[kWpL * kWpL], lz[kWpL * kWpL];
    __shared__ int2 shift[kMaxFrames];
    const int W = in.width, H = in.height;
    const int64_t np = (int64_t)W * H;
    for (int e = threadIdx.x; e < kWpL * kWpL; e += blockDim.x) {
        lw[e] = 0ull;
        lz[e] = 0ull;
    }
    if ((int)threadIdx.x < n) {
        const float cu = (float)(W / 2), cv = (float)(H / 2);
        float P[3], q[3];
        backproject(cu, cv, z_nom, in, P);
        xform(fr->Rf[threadIdx.x], P, q);
        int2 d = make_int2(0, 0);
        if (q[2] > 0.0f) {
            const float du = rintf((in.fx * q[0]) / q[2] + in.cx - cu);
            const float dv = rintf((in.fy * q[1]) / q[2] + in.cy - cv);
            // (a NaN compares false and leaves 0)
            if (fabsf(du) <= (float)kWpD) d.x = (int)du;
            else if (du > 0.0f) d.x = kWpD;
            else if (du < 0.0f) d.x = -kWpD;
            if (fabsf(dv) <= (float)kWpD) d.y = (int)dv;
            else if (dv > 0.0f) d.y = kWpD;
            else if (dv < 0.0f) d.y = -kWpD;
        }
        shift[threadIdx.x] = d;
    }
    __syncthreads();
    const int ku = ((int)blockIdx.x % tiles_x - kWpE) * kWpT, kv = ((int)blockIdx.x / tiles_x - kWpE) * kWpT;
    const int wx0 = ku - kWpM, wy0 = kv - kWpM;
    const int tx = (int)threadIdx.x & (kWpT - 1), ty = (int)threadIdx.x / kWpT;
    // frames in groups of kWpF: every load of a group issues before its samples are warped
    constexpr int kWpF = 4;
    for (int f0 = 0; f0 < n; f0 += kWpF) {
        float wg[kWpF], zg[kWpF];
#pragma unroll
        for (int j = 0; j < kWpF; ++j) {
            wg[j] = 0.0f;
            zg[j] = 0.0f;
            const int f = f0 + j;
            if (f < n) {
                const int2 d = shift[f];
                const int u = ku + tx - d.x, v = kv + ty - d.y;
                if (u >= 0 && u < W && v >= 0 && v < H) {
                    const size_t pix = (size_t)f * np + (size_t)v * W + u;
                    wg[j] = wz[pix];
                    zg[j] = Z[pix];
                }
            }
        }
#pragma unroll
        for (int j = 0; j < kWpF; ++j) {
            const int f = f0 + j;
            const float w = wg[j];
            if (!(w > 0.0f)) continue;  // also frames past n and pixels outside the image
            const int2 d = shift[f];
            const int u = ku + tx - d.x, v = kv + ty - d.y;
            float P[3], q[3];
            backproject((float)u, (float)v, zg[j], in, P);
            xform(fr->Rf[f], P, q);
            float uf, vf;
            int iu, iv;
            if (!project(in, q, uf, vf, iu, iv)) continue;
            const long long wk = (long long)rintf(w * kWeightScale);
            const long long zk = (long long)rintf(q[2] * 1048576.0f);
            const int lx = iu - wx0, ly = iv - wy0;
            if ((unsigned)lx < (unsigned)kWpL && (unsigned)ly < (unsigned)kWpL) {
                atomicAdd(&lw[ly * kWpL + lx], (unsigned long long)wk);
                atomicAdd(&lz[ly * kWpL + lx], (unsigned long long)(wk * zk));
            } else {
                const int64_t t = (int64_t)iv * W + iu;
                atomicAdd(KW + t, (unsigned long long)wk);
                atomicAdd(KZ + t, (unsigned long long)(wk * zk));
            }
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kWpL * kWpL; e += blockDim.x) {
        const unsigned long long a = lw[e];
        if (a != 0ull) {
            // only samples inside the image were added, so the pixel is too
            const int64_t t = (int64_t)(wy0 + e / kWpL) * W + (wx0 + e % kWpL);
            atomicAdd(KW + t, a);
            atomicAdd(KZ + t, lz[e]);
        }
    }
}

// ---------------------------------------------------------------------------
// colour pre-processing
// ---------------------------------------------------------------------------

__device__ inline int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

__device__ inline int luma(uint32_t px) { return (77 * (int)(px & 255u) + 150 * (int)((px >> 8) & 255u) + 29 * (int)(px >> 16) + 128) >> 8; }

// Colour pre-processing of one 64 x 16 tile of one frame.  The tile and a
// halo (2 pixels for the 5-tap binomial, 5 before and 4 after for the 9-tap
// re-blur box) are staged in LDS with coordinates clamped to the image, which
// is the edge rule of both filters.  The binomial runs separably on pixels
// packed as R | G << 16 | B << 32: every channel's weighted sum stays below
// 16 * 16 * 255 < 2^16, so the 16-bit lanes never carry into each other and
// the sums are the per-channel integers.  Each thread then produces four
// pixels of the unsharp mask and adds their re-blur terms to four int64
// sums, reduced over the workgroup and stored as the tile's partial sums (no
// atomics).
//   sums k = 0..3: sF_h, sV_h, sF_v, sV_v, the 9x-scaled horizontal and
//   vertical variation of the frame and of its re-blurred copy (the box
//   difference telescopes to two samples).
constexpr int kPrepTW = 64, kPrepTH = 16;
constexpr int kPrepLW = kPrepTW + 9, kPrepLH = kPrepTH + 9;
constexpr int kPrepHalo = 5;
constexpr int kPrepStage = (kPrepLW * kPrepLH + 255) / 256;  // staged pixels per thread (256 threads)

// kOutCh: 3 (packed RGB, the standalone output) or 4 (RGB and a zero, one
// 8-byte store per pixel; the layout the colour kernel gathers from).
template <int kOutCh>
__global__ __launch_bounds__(256) void color_prep_kernel(const uint8_t* __restrict__ rgb, int n, int W, int H,
                                                         int tiles_x, int tiles, uint16_t* __restrict__ out,
                                                         long long* __restrict__ parts)
{
    __shared__ uint64_t pix[kPrepLH][kPrepLW];
    __shared__ uint64_t hsum[kPrepTH + 4][kPrepTW];  // horizontal binomial of staged rows 3 .. 22
    __shared__ uint8_t lum[kPrepLH][kPrepLW];  // luma <= 255; bytes keep the workgroup under 26.7 KB of LDS (six per CU)
    __shared__ long long red[4][4];
    const int f = blockIdx.y, tile = blockIdx.x;
    if (f >= n || tile >= tiles) return;
    const int u0 = (tile % tiles_x) * kPrepTW, v0 = (tile / tiles_x) * kPrepTH;
    const int64_t np = (int64_t)W * H;
    const uint8_t* C = rgb + (size_t)f * np * 3;
    // staging: every load of a thread issues before its first LDS store
    uint32_t st[kPrepStage];
#pragma unroll
    for (int k = 0; k < kPrepStage; ++k) {
        const int p = (int)threadIdx.x + 256 * k;
        st[k] = 0u;
        if (p < kPrepLW * kPrepLH) {
            const int i = p % kPrepLW, j = p / kPrepLW;
            const int uu = clampi(u0 - kPrepHalo + i, 0, W - 1), vv = clampi(v0 - kPrepHalo + j, 0, H - 1);
            const uint8_t* q = C + 3 * ((size_t)vv * W + uu);
            st[k] = (uint32_t)q[0] | ((uint32_t)q[1] << 8) | ((uint32_t)q[2] << 16);
        }
    }
#pragma unroll
    for (int k = 0; k < kPrepStage; ++k) {
        const int p = (int)threadIdx.x + 256 * k;
        if (p < kPrepLW * kPrepLH) {
            const int i = p % kPrepLW, j = p / kPrepLW;
            const uint32_t px = st[k];
            pix[j][i] = (uint64_t)(px & 255u) | ((uint64_t)((px >> 8) & 255u) << 16) | ((uint64_t)(px >> 16) << 32);
            lum[j][i] = (uint8_t)luma(px);
        }
    }
    __syncthreads();
    for (int p = threadIdx.x; p < (kPrepTH + 4) * kPrepTW; p += blockDim.x) {
        const int c = p % kPrepTW, jr = p / kPrepTW;
        const uint64_t* row = &pix[jr + kPrepHalo - 2][c + kPrepHalo - 2];
        hsum[jr][c] = (row[0] + 4 * row[1]) + ((6 * row[2] + 4 * row[3]) + row[4]);
    }
    __syncthreads();
    const int tx = threadIdx.x & (kPrepTW - 1), ty = threadIdx.x / kPrepTW;
    long long acc[4] = {0, 0, 0, 0};
    const int u = u0 + tx, i = tx + kPrepHalo;
#pragma unroll 1
    for (int r = 0; r < kPrepTH / 4; ++r) {
        const int y = ty + 4 * r, v = v0 + y, j = y + kPrepHalo;
        if (u >= W || v >= H) continue;
        // staged row j + b is hsum row y + 2 + b
        const uint64_t S = (hsum[y][tx] + 4 * hsum[y + 1][tx]) +
                           ((6 * hsum[y + 2][tx] + 4 * hsum[y + 3][tx]) + hsum[y + 4][tx]);
        const uint64_t c0 = pix[j][i];
        uint32_t sh[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int val = 512 * (int)((c0 >> (16 * k)) & 0xFFFFu) - (int)((S >> (16 * k)) & 0xFFFFu);
            sh[k] = (uint32_t)clampi(val, 0, 65280);
        }
        const size_t px = (size_t)f * np + (size_t)v * W + u;
        if (kOutCh == 4) {
            *reinterpret_cast<uint2*>(out + 4 * px) = make_uint2(sh[0] | (sh[1] << 16), sh[2]);
        } else {
            uint16_t* o = out + 3 * px;
            o[0] = (uint16_t)sh[0];
            o[1] = (uint16_t)sh[1];
            o[2] = (uint16_t)sh[2];
        }
        const int y0 = lum[j][i];
        if (u >= 1) {
            const long long dF = 9LL * abs(y0 - lum[j][i - 1]);
            const long long dB = abs(lum[j][i + 4] - lum[j][i - 5]);
            acc[0] += dF;
            acc[1] += dF > dB ? dF - dB : 0;
        }
        if (v >= 1) {
            const long long dF = 9LL * abs(y0 - lum[j - 1][i]);
            const long long dB = abs(lum[j + 4][i] - lum[j - 5][i]);
            acc[2] += dF;
            acc[3] += dF > dB ? dF - dB : 0;
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
        for (int o = 32; o > 0; o >>= 1) acc[k] += __shfl_xor(acc[k], o);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) red[wave][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < 4) {
        const int k = threadIdx.x;
        parts[((size_t)f * tiles + tile) * 4 + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

// One workgroup per frame (standalone colour pre-processing).
__global__ __launch_bounds__(256) void blur_final_kernel(const long long* __restrict__ parts, int n, int tiles,
                                                         double* wb)
{
    __shared__ long long red[4][4];
    const int f = blockIdx.x;
    if (f >= n) return;
    blur_reduce(parts + (size_t)f * tiles * 4, tiles, red, wb + f);
}

// ---------------------------------------------------------------------------
// colour fusion
// ---------------------------------------------------------------------------

struct Obs {
    float c[3];
    uint32_t w;  // weight on the 2^-20 grid; 0: no observation from this frame
};

// One thread per (keyframe pixel, frame): a workgroup of 256 threads takes
// ppw = 256 / n pixels, thread t the pixel t / n and the frame t % n.  The
// first ppw threads form each pixel's depth from the fixed-point
// accumulators (W* = sum(w), Z* = sum(w z) / sum(w), rounded once to FP32)
// and its back-projection, once per pixel, in LDS; then every thread
// back-warps its pixel into its frame and stores its observation (or none)
// in LDS.  Then each thread decides for its own observation j and each
// channel whether it is the lower weighted median: with the observations
// ordered by (value, frame), j is the first whose cumulative weight reaches
// half the total exactly when the weight ordered strictly before it is below
// half and that weight plus its own reaches half; one observation per
// channel passes, and it writes the channel.
__global__ __launch_bounds__(256) void color_kernel(const float* __restrict__ Z, const float* __restrict__ wz,
                                                    const uint16_t* __restrict__ cs, const double* __restrict__ wb,
                                                    int n, int ppw, sc_intrinsics in, float occ_rel,
                                                    const FuseFrames* __restrict__ fr,
                                                    const unsigned long long* __restrict__ KW,
                                                    const unsigned long long* __restrict__ KZ, float* Zs, float* Ws,
                                                    uint8_t* rgba)
{
    __shared__ Obs obs[256];
    __shared__ float4 pt[256];  // per pixel: camera point (x, y, Z*) and W* (0: no depth)
    const int W = in.width, H = in.height;
    // np <= 16384^2 < 2^31: pixel indices and their division in 32 bits
    const int np = W * H;
    {
        const int p = (int)blockIdx.x * ppw + (int)threadIdx.x;
        if ((int)threadIdx.x < ppw && p < np) {
            float4 e = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            const long long kw = (long long)KW[p];
            if (kw > 0) {
                const float zk = (float)(((double)(long long)KZ[p] / (double)kw) * 0x1p-20);
                const int v = p / W, u = p - v * W;
                float P[3];
                backproject((float)u, (float)v, zk, in, P);
                e = make_float4(P[0], P[1], P[2], (float)((double)kw / 1024.0));
            }
            pt[threadIdx.x] = e;
        }
    }
    __syncthreads();
    const int lp = (int)threadIdx.x / n, i = (int)threadIdx.x - lp * n;
    const int idx = (int)blockIdx.x * ppw + lp;
    const bool mine = lp < ppw && idx < np;
    Obs o;
    o.c[0] = o.c[1] = o.c[2] = 0.0f;
    o.w = 0u;
    const float4 e = mine ? pt[lp] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (e.w > 0.0f) {
        const float P[3] = {e.x, e.y, e.z};
        float q[3], uf, vf;
        int iu, iv;
        xform(fr->Rb[i], P, q);
        if (project(in, q, uf, vf, iu, iv)) {
            const size_t base = (size_t)i * np;
            const float wzi = wz[base + (size_t)iv * W + iu];
            const float zi = Z[base + (size_t)iv * W + iu];
            const float x0 = floorf(uf), y0 = floorf(vf);
            if (wzi > 0.0f && fabsf(zi - q[2]) <= occ_rel * q[2] && x0 >= 0.0f && x0 + 1.0f <= (float)(W - 1) &&
                y0 >= 0.0f && y0 + 1.0f <= (float)(H - 1)) {
                const float ax = uf - x0, ay = vf - y0;
                const int ix = (int)x0, iy = (int)y0;
                const float wcs = rintf(((float)wb[i] * wzi) * 1048576.0f);
                if (wcs > 0.0f) {
                    // four channels of 16 bits per pixel, 8-byte aligned
                    const uint2* C0 = reinterpret_cast<const uint2*>(cs) + base + (size_t)iy * W + ix;
                    const uint2* C1 = C0 + W;
                    const uint2 p00 = C0[0], p10 = C0[1], p01 = C1[0], p11 = C1[1];
                    auto ch = [](uint2 p, int k) {
                        return (float)(k == 0 ? (p.x & 0xFFFFu) : k == 1 ? (p.x >> 16) : (p.y & 0xFFFFu));
                    };
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const float c00 = ch(p00, k), c10 = ch(p10, k);
                        const float c01 = ch(p01, k), c11 = ch(p11, k);
                        const float top = c00 + ax * (c10 - c00);
                        const float bot = c01 + ax * (c11 - c01);
                        o.c[k] = top + ay * (bot - top);
                    }
                    o.w = (uint32_t)wcs;
                }
            }
        }
    }
    if (lp < ppw) obs[threadIdx.x] = o;
    __syncthreads();
    if (!mine) return;
    const Obs* po = obs + lp * n;
    uint64_t total = 0, below[3] = {0, 0, 0};
    for (int l = 0; l < n; ++l) {
        const Obs ol = po[l];
        total += ol.w;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (ol.c[k] < o.c[k] || (ol.c[k] == o.c[k] && l < i)) below[k] += ol.w;
    }
    uint8_t* out = rgba + 4 * (size_t)idx;
    if (total == 0) {
        // no frame observed the pixel (or it has no depth)
        if (i == 0) {
            Ws[idx] = 0.0f;
            Zs[idx] = 0.0f;
            out[0] = out[1] = out[2] = out[3] = 0;
        }
        return;
    }
    if (i == 0) {
        Ws[idx] = e.w;
        Zs[idx] = e.z;
        out[3] = 255;
    }
    if (o.w == 0u) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (2 * below[k] < total && 2 * (below[k] + o.w) >= total) {
            float val = rintf(o.c[k] / 256.0f);
            val = fminf(fmaxf(val, 0.0f), 255.0f);
            out[k] = (uint8_t)val;
        }
    }
}

// ---------------------------------------------------------------------------
// workspace
// ---------------------------------------------------------------------------

struct FuseWs {
    std::mutex mu;
    int device = -1;
    size_t cap_px = 0, cap_frames = 0;
    float* wz = nullptr;
    uint16_t* cs = nullptr;
    unsigned long long* acc = nullptr;   // KW, KZ
    long long* parts = nullptr;          // 4 per colour-prep tile and frame
    size_t cap_parts = 0;
    double* wb = nullptr;
    FuseFrames* d_fr = nullptr;
};

static FuseWs g_ws;

// Colour-prep tiles of one W x H frame.
static int prep_tiles_x(int W) { return (W + kPrepTW - 1) / kPrepTW; }
static int prep_tiles(int W, int H) { return prep_tiles_x(W) * ((H + kPrepTH - 1) / kPrepTH); }

// np pixels per frame, frames frames, parts int64 colour-prep partials.
static sc_status ws_reserve(size_t np, size_t frames, size_t parts)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return SC_EDEVICE;
    if (g_ws.device != dev) {
        // a different device: start over (old buffers belong to another device)
        g_ws.cap_px = g_ws.cap_frames = 0;
        g_ws.wz = nullptr;
        g_ws.cs = nullptr;
        g_ws.acc = nullptr;
        g_ws.parts = nullptr;
        g_ws.cap_parts = 0;
        g_ws.wb = nullptr;
        g_ws.d_fr = nullptr;
        g_ws.device = dev;
    }
    if (!g_ws.d_fr) {
        if (hipMalloc(&g_ws.d_fr, sizeof(FuseFrames)) != hipSuccess) return SC_ENOMEM;
        if (hipMalloc(&g_ws.wb, sizeof(double) * kMaxFrames) != hipSuccess) return SC_ENOMEM;
    }
    if (np * frames > g_ws.cap_px * g_ws.cap_frames || np > g_ws.cap_px) {
        if (hipDeviceSynchronize() != hipSuccess) return SC_EDEVICE;
        (void)hipFree(g_ws.wz);
        (void)hipFree(g_ws.cs);
        (void)hipFree(g_ws.acc);
        const size_t px = std::max(np, g_ws.cap_px);
        const size_t fr = std::max(frames, g_ws.cap_frames);
        g_ws.wz = nullptr;
        g_ws.cs = nullptr;
        g_ws.acc = nullptr;
        g_ws.cap_px = g_ws.cap_frames = 0;
        if (hipMalloc(&g_ws.wz, sizeof(float) * px * fr) != hipSuccess) return SC_ENOMEM;
        if (hipMalloc(&g_ws.cs, sizeof(uint16_t) * 4 * px * fr) != hipSuccess) return SC_ENOMEM;
        if (hipMalloc(&g_ws.acc, sizeof(unsigned long long) * 2 * px) != hipSuccess) return SC_ENOMEM;
        g_ws.cap_px = px;
        g_ws.cap_frames = fr;
    }
    if (parts > g_ws.cap_parts) {
        if (hipDeviceSynchronize() != hipSuccess) return SC_EDEVICE;
        (void)hipFree(g_ws.parts);
        g_ws.parts = nullptr;
        g_ws.cap_parts = 0;
        if (hipMalloc(&g_ws.parts, sizeof(long long) * parts) != hipSuccess) return SC_ENOMEM;
        g_ws.cap_parts = parts;
    }
    return SC_OK;
}

// Fusion parameters a fusion accepts: z_min at least 2^-5 m keeps every
// depth weight w_z <= 1 / z_min^2 at most 2^10, so a colour weight on the
// 2^-20 grid stays below 2^31 and fits the 32 bits it is held in.
static bool fuse_params_valid(const sc_fuse_params* p)
{
    return p && p->z_min >= 0x1p-5f && p->z_max >= p->z_min && p->z_max < 1e6f && p->disc_rel >= 0.0f &&
           p->occ_rel >= 0.0f;
}

static bool intr_valid(const sc_intrinsics* in)
{
    return in && in->width >= 3 && in->height >= 3 && in->fx > 0.0f && in->fy > 0.0f && in->width <= 16384 &&
           in->height <= 16384;
}

// Overlap counts (valid, visible) of one frame with a reference view, FP64
// in the written order; each thread counts kOverlapPix pixels, a workgroup
// reduces in LDS and adds its two totals with one atomic each.
struct OverlapArgs {
    double R[9], t[3], Rr[9], tr[3];
    double fx, fy, cx, cy;
    float z_min, z_max;
    int32_t width, height;
};

constexpr int kOverlapPix = 16;

__global__ void overlap_clear_kernel(uint32_t* counts)
{
    if (threadIdx.x < 2) counts[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(256) void overlap_kernel(const float* __restrict__ depth, OverlapArgs a,
                                                      uint32_t* counts)
{
    __shared__ uint32_t red[2][256];
    const int64_t n = (int64_t)a.width * a.height;
    const int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * kOverlapPix;
    uint32_t valid = 0u, visible = 0u;
    for (int k = 0; k < kOverlapPix; ++k) {
        const int64_t i = i0 + k;
        if (i >= n) break;
        const float zf = depth[i];
        if (!(zf >= a.z_min && zf <= a.z_max)) continue;
        ++valid;
        const int u = (int)(i % a.width), v = (int)(i / a.width);
        const double z = (double)zf;
        const double p[3] = {(((double)u - a.cx) / a.fx) * z, (((double)v - a.cy) / a.fy) * z, z};
        double w[3];
#pragma unroll
        for (int r = 0; r < 3; ++r) w[r] = ((a.R[3 * r] * p[0] + a.R[3 * r + 1] * p[1]) + a.R[3 * r + 2] * p[2]) + a.t[r];
        const double d[3] = {w[0] - a.tr[0], w[1] - a.tr[1], w[2] - a.tr[2]};
        double q[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) q[c] = (a.Rr[c] * d[0] + a.Rr[3 + c] * d[1]) + a.Rr[6 + c] * d[2];
        if (q[2] > 0.0) {
            const double fu = floor(((a.fx * q[0]) / q[2] + a.cx) + 0.5);
            const double fv = floor(((a.fy * q[1]) / q[2] + a.cy) + 0.5);
            visible += (fu >= 0.0 && fu <= (double)(a.width - 1) && fv >= 0.0 && fv <= (double)(a.height - 1)) ? 1u : 0u;
        }
    }
    red[0][threadIdx.x] = valid;
    red[1][threadIdx.x] = visible;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < (unsigned)o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (red[0][0]) atomicAdd(counts, red[0][0]);
        if (red[1][0]) atomicAdd(counts + 1, red[1][0]);
    }
}

static void rel_pose(const sc_pose& A, const sc_pose& B, float out[12])
{
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) {
            const double x = (A.R[0 * 3 + r] * B.R[0 * 3 + c] + A.R[1 * 3 + r] * B.R[1 * 3 + c]) + A.R[2 * 3 + r] * B.R[2 * 3 + c];
            out[3 * r + c] = (float)x;
        }
        const double y = (A.R[0 * 3 + r] * (B.t[0] - A.t[0]) + A.R[1 * 3 + r] * (B.t[1] - A.t[1])) +
                         A.R[2 * 3 + r] * (B.t[2] - A.t[2]);
        out[9 + r] = (float)y;
    }
}

static void launch_depth_weight(const float* depth, int n, const sc_intrinsics& in, const sc_fuse_params& p, float* out,
                                const FuseInit& init, hipStream_t s)
{
    const int tiles_x = (in.width + kDwTW - 1) / kDwTW;
    const int tiles = tiles_x * ((in.height + kDwTH - 1) / kDwTH);
    depth_weight_kernel<<<dim3((unsigned)tiles, (unsigned)n), 256, 0, s>>>(depth, n, in, p, tiles_x, tiles, out, init);
}

// wb null: the partials only, sharpened colour with four channels per pixel
// (a fusion forms w_b in its depth-weight launch); else three channels and
// w_b.
static void launch_color_prep(const uint8_t* rgb, int n, int W, int H, uint16_t* sharp, long long* parts, double* wb,
                              hipStream_t s)
{
    const int tiles = prep_tiles(W, H);
    const dim3 grid((unsigned)tiles, (unsigned)n);
    if (wb) {
        color_prep_kernel<3><<<grid, 256, 0, s>>>(rgb, n, W, H, prep_tiles_x(W), tiles, sharp, parts);
        blur_final_kernel<<<n, 256, 0, s>>>(parts, n, tiles, wb);
    } else {
        color_prep_kernel<4><<<grid, 256, 0, s>>>(rgb, n, W, H, prep_tiles_x(W), tiles, sharp, parts);
    }
}

// Relative poses of frames first .. first + count - 1 into the device table.
__global__ void stage_poses_kernel(PoseChunk c, int first, int count, FuseFrames* fr)
{
    for (int i = threadIdx.x; i < count * 12; i += blockDim.x) {
        fr->Rf[first + i / 12][i % 12] = c.Rf[i / 12][i % 12];
        fr->Rb[first + i / 12][i % 12] = c.Rb[i / 12][i % 12];
    }
}

// Device buffers of one fusion: per-frame weights, sharpened colour, the
// fixed-point accumulators, colour-prep partials, w_b and the relative poses.
struct FuseBufs {
    float* wz;
    uint16_t* cs;
    unsigned long long* acc;
    long long* parts;
    double* wb;
    FuseFrames* fr;
};

// The fusion kernels of one keyframe.  The relative poses of the first
// kStageFrames frames travel in the depth-weight launch; those of later
// frames are stored by stage_poses_kernel launches enqueued first.
static void launch_fuse(const FuseBufs& b, const float* depth, const uint8_t* rgb, const sc_pose* poses, int n_frames,
                        int ref, const sc_intrinsics& in, const sc_fuse_params& params, float* kf_depth,
                        float* kf_weight, uint8_t* kf_rgba, hipStream_t s)
{
    const int64_t np = (int64_t)in.width * in.height;
    FuseInit init;
    init.acc = b.acc;
    init.parts = b.parts;
    init.wb = b.wb;
    init.prep_tiles = prep_tiles(in.width, in.height);
    init.fr = b.fr;
    for (int i0 = kStageFrames; i0 < n_frames; i0 += kStageFrames) {
        const int cnt = std::min(kStageFrames, n_frames - i0);
        for (int j = 0; j < cnt; ++j) {
            rel_pose(poses[ref], poses[i0 + j], init.poses.Rf[j]);
            rel_pose(poses[i0 + j], poses[ref], init.poses.Rb[j]);
        }
        stage_poses_kernel<<<1, 256, 0, s>>>(init.poses, i0, cnt, b.fr);
    }
    init.count = std::min(kStageFrames, n_frames);
    for (int j = 0; j < init.count; ++j) {
        rel_pose(poses[ref], poses[j], init.poses.Rf[j]);
        rel_pose(poses[j], poses[ref], init.poses.Rb[j]);
    }
    launch_color_prep(rgb, n_frames, in.width, in.height, b.cs, b.parts, nullptr, s);
    launch_depth_weight(depth, n_frames, in, params, b.wz, init, s);
    // target tiles over the image and kWpE more on each side
    const int wtx = (in.width + kWpT - 1) / kWpT + 2 * kWpE, wty = (in.height + kWpT - 1) / kWpT + 2 * kWpE;
    const float z_nom = 0.5f * (params.z_min + params.z_max);
    warp_kernel<<<(unsigned)(wtx * wty), 256, 0, s>>>(depth, b.wz, n_frames, in, z_nom, wtx, b.fr, b.acc,
                                                       b.acc + np);
    const int ppw = 256 / n_frames;  // pixels per colour workgroup (n_frames <= kMaxFrames = 64)
    color_kernel<<<(unsigned)((np + ppw - 1) / ppw), 256, 0, s>>>(depth, b.wz, b.cs, b.wb, n_frames, ppw, in,
                                                                  params.occ_rel, b.fr, b.acc, b.acc + np, kf_depth,
                                                                  kf_weight, kf_rgba);
}

// ---------------------------------------------------------------------------
// allocation-free fusion: every buffer in one fixed device array
// ---------------------------------------------------------------------------

// Scratch of kf_fuse_noalloc.  In host code `scratch` names a host-side
// stand-in, never device memory: its device address is looked up once per
// device with hipGetSymbolAddress and only that address is passed on.  Every
// call on a device shares that device's copy, so calls that overlap on one
// device race.
constexpr size_t kScratchBytes = size_t(76) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char* g_scratch_dev[kMaxDevices];

// The current device's address of `scratch`, looked up on the first call on
// that device (with the device current).
static sc_status scratch_address(unsigned char** out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SC_EDEVICE;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SC_EDEVICE;
        g_scratch_dev[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_scratch_dev[dev];
    return SC_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Places the fusion buffers of np pixels x frames frames in one region
// starting at base (may be null to measure); returns the bytes used.
static size_t fuse_layout(unsigned char* base, size_t np, size_t frames, size_t parts, FuseBufs& b)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char* p = base ? base + off : nullptr;
        off = align256(off + bytes);
        return p;
    };
    b.fr = reinterpret_cast<FuseFrames*>(take(sizeof(FuseFrames)));
    b.wb = reinterpret_cast<double*>(take(sizeof(double) * kMaxFrames));
    b.acc = reinterpret_cast<unsigned long long*>(take(sizeof(unsigned long long) * 2 * np));
    b.parts = reinterpret_cast<long long*>(take(sizeof(long long) * parts));
    b.wz = reinterpret_cast<float*>(take(sizeof(float) * np * frames));
    b.cs = reinterpret_cast<uint16_t*>(take(sizeof(uint16_t) * 4 * np * frames));
    return off;
}

}  // namespace sc

using namespace sc;

extern "C" {

sc_status sc_depth_weight(const float* depth, int32_t n_frames, const sc_intrinsics* intr, const sc_fuse_params* params,
                          float* wz_out, void* stream)
{
    if (!depth || !wz_out || n_frames <= 0 || n_frames > 65535 || !intr_valid(intr) || !params) return SC_EINVAL;
    launch_depth_weight(depth, n_frames, *intr, *params, wz_out, FuseInit{}, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
}

sc_status sc_color_prep(const uint8_t* rgb, int32_t n_frames, int32_t width, int32_t height, uint16_t* sharp_out,
                        double* wb_out, void* stream)
{
    if (!rgb || !sharp_out || !wb_out || n_frames <= 0 || n_frames > kMaxFrames || width < 2 || height < 2 ||
        width > 16384 || height > 16384)
        return SC_EINVAL;
    std::lock_guard<std::mutex> lk(g_ws.mu);
    const sc_status st =
        ws_reserve((size_t)width * height, (size_t)n_frames, 4 * (size_t)prep_tiles(width, height) * n_frames);
    if (st != SC_OK) return st;
    launch_color_prep(rgb, n_frames, width, height, sharp_out, g_ws.parts, wb_out, (hipStream_t)stream);
    return hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
}

sc_status kf_fuse(const float* depth, const uint8_t* rgb, const sc_pose* poses, int32_t n_frames, int32_t ref,
                  const sc_intrinsics* intr, const sc_fuse_params* params, float* kf_depth, float* kf_weight,
                  uint8_t* kf_rgba, void* stream)
{
    if (!depth || !rgb || !poses || n_frames <= 0 || n_frames > kMaxFrames || ref < 0 || ref >= n_frames ||
        !intr_valid(intr) || !fuse_params_valid(params) || !kf_depth || !kf_weight || !kf_rgba)
        return SC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const sc_intrinsics in = *intr;
    const int64_t np = (int64_t)in.width * in.height;
    std::lock_guard<std::mutex> lk(g_ws.mu);
    sc_status st = ws_reserve((size_t)np, (size_t)n_frames, 4 * (size_t)prep_tiles(in.width, in.height) * n_frames);
    if (st != SC_OK) return st;
    const FuseBufs b{g_ws.wz, g_ws.cs, g_ws.acc, g_ws.parts, g_ws.wb, g_ws.d_fr};
    launch_fuse(b, depth, rgb, poses, n_frames, ref, in, *params, kf_depth, kf_weight, kf_rgba, s);
    return hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
}

sc_status kf_fuse_noalloc(const float* depth, const uint8_t* rgb, const sc_pose* poses, int32_t n_frames, int32_t ref,
                          const sc_intrinsics* intr, const sc_fuse_params* params, float* kf_depth, float* kf_weight,
                          uint8_t* kf_rgba, void* stream)
{
    if (!depth || !rgb || !poses || n_frames <= 0 || n_frames > kMaxFrames || ref < 0 || ref >= n_frames ||
        !intr_valid(intr) || !fuse_params_valid(params) || !kf_depth || !kf_weight || !kf_rgba)
        return SC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const sc_intrinsics in = *intr;
    const size_t np = (size_t)in.width * in.height;
    const size_t parts = 4 * (size_t)prep_tiles(in.width, in.height) * n_frames;
    FuseBufs b;
    if (fuse_layout(nullptr, np, (size_t)n_frames, parts, b) > kScratchBytes) return SC_ESCRATCH;
    unsigned char* base = nullptr;
    const sc_status st = scratch_address(&base);
    if (st != SC_OK) return st;
    fuse_layout(base, np, (size_t)n_frames, parts, b);
    launch_fuse(b, depth, rgb, poses, n_frames, ref, in, *params, kf_depth, kf_weight, kf_rgba, s);
    return hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
}

sc_status sc_overlap(const float* depth, const sc_intrinsics* intr, const sc_pose* T_frame, const sc_pose* T_ref,
                     float z_min, float z_max, uint32_t* counts, void* stream)
{
    if (!depth || !intr || !T_frame || !T_ref || !counts || intr->width <= 0 || intr->height <= 0 ||
        intr->width > 16384 || intr->height > 16384 || !(intr->fx > 0.0f) || !(intr->fy > 0.0f))
        return SC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    OverlapArgs a;
    memcpy(a.R, T_frame->R, sizeof(a.R));
    memcpy(a.t, T_frame->t, sizeof(a.t));
    memcpy(a.Rr, T_ref->R, sizeof(a.Rr));
    memcpy(a.tr, T_ref->t, sizeof(a.tr));
    a.fx = intr->fx;
    a.fy = intr->fy;
    a.cx = intr->cx;
    a.cy = intr->cy;
    a.z_min = z_min;
    a.z_max = z_max;
    a.width = intr->width;
    a.height = intr->height;
    overlap_clear_kernel<<<1, 64, 0, s>>>(counts);
    const int64_t n = (int64_t)intr->width * intr->height;
    const int64_t per_wg = 256 * kOverlapPix;
    overlap_kernel<<<(unsigned)((n + per_wg - 1) / per_wg), 256, 0, s>>>(depth, a, counts);
    return hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
}

}  // extern "C"
