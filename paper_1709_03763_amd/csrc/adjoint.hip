// Adjoint of integration.  After integrating keyframes k at poses T_k into a
// field (running weighted average, Sec. 3; quantities of Sec. 4.3), every
// voxel holds D = (W0 D0 + sum_k w_k d_k) / W with d_k = Z_k(u_k) - p_z and
// W = W0 + sum_k w_k (the colour likewise).  With the pixel and band
// decisions held fixed:
//   dL/dZ_k(u)  = sum_{v -> u} (w_k / W) dL/dD(v)
//   dL/dC_k(u)  = sum_{v -> u} (w_k / W) dL/dC(v)
//   dL/dxi_k    = sum_v (w_k / W) dL/dD(v) (0, 0, 1, p_y, -p_x, 0)
//   dL/dD0(v)   = (W0 / W) dL/dD(v),   dL/dC0(v) = (W0 / W) dL/dC(v)
// for a right perturbation T_k Exp(xi) (p = Exp(-xi) T_k^-1 x_v, so
// dp/drho = -I, dp/dphi = [p]_x and d d_k / d xi = -d p_z / d xi).
//
// The keyframes run in chunks through the batched candidate stage, which
// leaves every block a keyframe may touch with the mask of those keyframes;
// a persistent pass then visits each candidate block once, loads its weights
// and upstream gradients, walks its keyframes, scatters the pixel gradients
// and accumulates the pose terms per workgroup in LDS.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"
#include "kernels.hpp"

namespace sc {

template <int CM>
__global__ __launch_bounds__(256) void adjoint_kernel(const OpDesc* __restrict__ ops, VolDev v, CandDev cd,
                                                      const float* __restrict__ gD, const float* __restrict__ gC,
                                                      float* grad_depth, float* grad_color, float* grad_D0,
                                                      float* grad_C0, double* acc_xi, int n_ops)
{
    // pose terms 2, 3, 4 of each keyframe of the chunk, then one dummy slot
    // per lane for the lanes that carry no term
    __shared__ double s_acc[3 * kAdjChunk + 64];
    const int lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < 3 * n_ops + 64; i += blockDim.x) s_acc[i] = 0.0;
    __syncthreads();
    const uint32_t n = cd.counters[4];
    const uint32_t worker = blockIdx.x * (blockDim.x >> 6) + bcast(threadIdx.x >> 6);
    const uint32_t n_workers = gridDim.x * (blockDim.x >> 6);
    WorkCursor cur;
    cursor_init(cur, worker);
    for (;;) {
        const uint32_t i = cursor_pop(cur, cd.counters + 5, n_workers, lane);
        if (i >= n) break;
        const uint32_t h = bcast(cd.sorted[i]);
        const uint64_t key = bcast64(cd.skey[i]);
        const int slot = (int)bcast((uint32_t)cd.sslot[i]);
        int bx, by, bz;
        unpack_key(key, bx, by, bz);
        // a candidate block the forward never allocated holds no touched voxel
        const size_t sb = (size_t)max(slot, 0);
        const float* blk = v.pool + sb * v.stride;
        float Wv[8], g[8], gc[3][8], sw[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int x = lane + 64 * j;
            Wv[j] = (slot >= 0) ? blk[kPoolW + x] : 0.0f;
            g[j] = (slot >= 0) ? gD[sb * kBlockVox + x] : 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) gc[c][j] = (gC && slot >= 0) ? gC[(sb * 3 + c) * kBlockVox + x] : 0.0f;
            sw[j] = 0.0f;
        }
        OpWalk walk{cd.mask + (size_t)h * cd.words, cd.words, 0, bcast64(cd.mask[(size_t)h * cd.words])};
        for (int o = walk_next(walk); o >= 0; o = walk_next(walk)) {
            const OpDesc& op = ops[o];
            float q[3];
            double qz;
            block_origin(op, v.s, bx, by, bz, q, qz);
            const float kx = (float)(lane & 7), ky = (float)(lane >> 3);
            float base[3];
#pragma unroll
            for (int r = 0; r < 3; ++r) base[r] = (q[r] + kx * op.a[0][r]) + ky * op.a[1][r];
            VoxHits<CM, 8> hv;
            test_voxels<CM, 8, false>(op, v.mu, base, 0, hv);
            const size_t np = (size_t)op.width * op.height;
            float j2 = 0.0f, j3 = 0.0f, j4 = 0.0f;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (!((hv.hit >> j) & 1u) || !(Wv[j] > 0.0f)) continue;
                const float fz = (float)j;
                const float px = base[0] + fz * op.a[2][0];
                const float py = base[1] + fz * op.a[2][1];
                const float a = hv.w[j] / Wv[j];
                const float gg = g[j] * a;
                const size_t pix = (size_t)op.kf * np + (size_t)hv.pix[j];
                atomicAdd(grad_depth + pix, gg);
                if (CM == SC_COLOR_F32 && grad_color) {
                    atomicAdd(grad_color + 3 * pix + 0, gc[0][j] * a);
                    atomicAdd(grad_color + 3 * pix + 1, gc[1][j] * a);
                    atomicAdd(grad_color + 3 * pix + 2, gc[2][j] * a);
                }
                sw[j] += hv.w[j];
                j2 += gg;
                j3 += gg * py;
                j4 -= gg * px;
            }
            // every lane receives the three sums; lanes 0..2 add one each,
            // the others add zero to their own dummy slot (no lane-id branch)
            double t2 = (double)j2, t3 = (double)j3, t4 = (double)j4;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) {
                t2 += __shfl_xor(t2, off);
                t3 += __shfl_xor(t3, off);
                t4 += __shfl_xor(t4, off);
            }
            const double val = (lane == 0) ? t2 : (lane == 1) ? t3 : (lane == 2) ? t4 : 0.0;
            double* dst = (lane < 3) ? s_acc + 3 * o + lane : s_acc + 3 * n_ops + lane;
            atomicAdd(dst, val);
        }
        // dL/dD0 = dL/dD (W - sum_k w_k) / W: grad_D0 first collects
        // sum_k w_k over the chunks (exact in FP32 on the 2^-10 weight grid
        // below 2^14, one wavefront per block and launch), and the final
        // kernel forms W0 = W - sum_k w_k exactly before one division, so a
        // small W0 / W is not the difference of two nearly equal products
        if (slot >= 0 && grad_D0) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int x = lane + 64 * j;
                if (sw[j] > 0.0f) grad_D0[sb * kBlockVox + x] += sw[j];
            }
        }
        retire_candidate(cd, v, h, 0, lane);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * n_ops; i += blockDim.x)
        if (s_acc[i] != 0.0) atomicAdd(acc_xi + i, s_acc[i]);
}

// grad_D0 holds sum_k w_k per voxel while the chunks run; it starts at 0.
__global__ void adjoint_prior_init_kernel(int64_t n_blocks, float* grad_D0)
{
    const int64_t b = blockIdx.x;
    for (int x = threadIdx.x; x < kBlockVox; x += blockDim.x) grad_D0[b * kBlockVox + x] = 0.0f;
}

// dL/dD0 = dL/dD W0 / W and dL/dC0 = dL/dC W0 / W with W0 = W - sum_k w_k
// (exact), where W > 0; 0 elsewhere (an empty voxel stays empty whatever D0
// holds).
__global__ void adjoint_prior_final_kernel(VolDev v, int64_t n_blocks, const float* gD, const float* gC,
                                           float* grad_D0, float* grad_C0)
{
    const int64_t b = blockIdx.x;
    const float* blk = v.pool + (size_t)b * v.stride;
    for (int x = threadIdx.x; x < kBlockVox; x += blockDim.x) {
        const float W = blk[kPoolW + x];
        const bool live = W > 0.0f;
        const float f = live ? (W - grad_D0[b * kBlockVox + x]) / W : 0.0f;
        grad_D0[b * kBlockVox + x] = live ? gD[b * kBlockVox + x] * f : 0.0f;
        if (grad_C0)
            for (int c = 0; c < 3; ++c)
                grad_C0[(b * 3 + c) * kBlockVox + x] = (live && gC) ? gC[(b * 3 + c) * kBlockVox + x] * f : 0.0f;
    }
}

__global__ void xi_final_kernel(double* acc, int n, float* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        out[6 * (i / 3) + 2 + i % 3] += (float)acc[i];
        acc[i] = 0.0;
    }
}

}  // namespace sc

using namespace sc;

extern "C" {

sc_status tsdf_integrate_backward(sc_volume* vol, const sc_keyframe* kfs, int32_t n_kf, const sc_intrinsics* intr,
                                  const sc_pose* T, const float* grad_D, const float* grad_C, float* grad_depth,
                                  float* grad_color, float* grad_xi, float* grad_D0, float* grad_C0, void* stream)
{
    if (!vol || !kfs || n_kf <= 0 || !intr || intr->width <= 0 || intr->height <= 0 || !(intr->fx > 0.0f) ||
        !(intr->fy > 0.0f) || intr->width > 16384 || intr->height > 16384 || !T || !grad_D || !grad_depth ||
        !grad_xi)
        return SC_EINVAL;
    if ((grad_C != nullptr) != (grad_color != nullptr)) return SC_EINVAL;
    if (grad_C0 && (!grad_D0 || !grad_C)) return SC_EINVAL;
    if (grad_color && vol->p.color_mode != SC_COLOR_F32) return SC_EINVAL;
    if (stream_host_blocks(vol) > 0) return SC_EINVAL;  // the forward's blocks must all be on the device
    for (int i = 0; i < n_kf; ++i)
        if (!keyframe_ok(&kfs[i])) return SC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int64_t nb = 0;
    int32_t sticky = 0;
    sc_status st = sc_volume_query(vol, s, &nb, &sticky);
    if (st != SC_OK) return st;
    if (sticky != SC_OK) return sticky;
    if (grad_D0 && nb > 0) adjoint_prior_init_kernel<<<(unsigned)nb, 256, 0, s>>>(nb, grad_D0);
    const int chunk = std::min(vol->p.max_batch_ops, kAdjChunk);
    const bool f32 = vol->p.color_mode == SC_COLOR_F32;
    for (int k0 = 0; k0 < n_kf; k0 += chunk) {
        const int cnt = std::min(chunk, n_kf - k0);
        OpDesc* ops = stage_begin(vol);
        if (!ops) return SC_EDEVICE;
        // op.kf is the keyframe's index in the call: it addresses the pixel gradients
        for (int j = 0; j < cnt; ++j) make_op(vol, &kfs[k0 + j], intr, &T[k0 + j], +1, k0 + j, &ops[j]);
        st = run_candidates(vol, ops, cnt, intr, s);
        if (st != SC_OK) return st;
        const int grid = vol->n_cu * 4;
        if (f32)
            adjoint_kernel<SC_COLOR_F32><<<grid, 256, 0, s>>>(vol->d_ops, vol->dev, vol->cand, grad_D, grad_C,
                                                              grad_depth, grad_color, grad_D0, grad_C0,
                                                              vol->adj_acc, cnt);
        else
            adjoint_kernel<SC_COLOR_RGBA8><<<grid, 256, 0, s>>>(vol->d_ops, vol->dev, vol->cand, grad_D, nullptr,
                                                                grad_depth, nullptr, grad_D0, nullptr, vol->adj_acc,
                                                                cnt);
        xi_final_kernel<<<(3 * cnt + 255) / 256, 256, 0, s>>>(vol->adj_acc, 3 * cnt, grad_xi + 6 * (size_t)k0);
    }
    if (grad_D0 && nb > 0)
        adjoint_prior_final_kernel<<<(unsigned)nb, 256, 0, s>>>(vol->dev, nb, grad_D, grad_C, grad_D0, grad_C0);
    return hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
}

}  // extern "C"
