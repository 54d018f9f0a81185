// Adjoint of integration.  After integrating keyframes k at poses T_k into a
// field (running weighted average, Sec. 3; quantities of Sec. 4.3), every
// voxel holds D = (W0 D0 + sum_k w_k d_k) / W with d_k = Z_k(u_k) - p_z and
// W = W0 + sum_k w_k.  With the pixel and band decisions held fixed:
//   dL/dZ_k(u)  = sum_{v -> u} (w_k / W) dL/dD(v)
//   dL/dC_k(u)  = sum_{v -> u} (w_k / W) dL/dC(v)
//   dL/dxi_k    = sum_v (w_k / W) dL/dD(v) (0, 0, 1, p_y, -p_x, 0)
// for a right perturbation T_k Exp(xi) (p = Exp(-xi) T_k^-1 x_v, so
// dp/drho = -I, dp/dphi = [p]_x and d d_k / d xi = -d p_z / d xi).
#include "common.hpp"
#include "internal.hpp"
#include "kernels.hpp"

namespace sc {

// One one-wavefront workgroup per (block, keyframe) pair, eight voxels per
// lane; the pose terms are reduced in LDS.
template <int CM>
__global__ __launch_bounds__(64) void backward_kernel(const OpDesc* __restrict__ ops, VolDev v,
                                                      const float* __restrict__ gD, const float* __restrict__ gC,
                                                      float* grad_depth, float* grad_color, double* acc_xi)
{
    __shared__ float red[3][64];
    const int lane = threadIdx.x;
    const int64_t b = blockIdx.x;
    const int k = blockIdx.y;
    const OpDesc& op = ops[k];
    const uint64_t key = v.slot_keys[b];
    int bx, by, bz;
    unpack_key(key, bx, by, bz);
    float q[3];
    double qz;
    block_origin(op, v.s, bx, by, bz, q, qz);
    const float kx = (float)(lane & 7), ky = (float)(lane >> 3);
    float base[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) base[r] = (q[r] + kx * op.a[0][r]) + ky * op.a[1][r];
    const float* blk = v.pool + (size_t)b * v.stride;
    const size_t np = (size_t)op.width * op.height;
    float j2 = 0.0f, j3 = 0.0f, j4 = 0.0f;
#pragma unroll
    for (int kz = 0; kz < 8; ++kz) {
        const float fz = (float)kz;
        const float px = base[0] + fz * op.a[2][0];
        const float py = base[1] + fz * op.a[2][1];
        const float pz = base[2] + fz * op.a[2][2];
        int pix;
        float w, z;
        if (!touch(op, v.mu, px, py, pz, pix, w, z)) continue;
        const int i = lane + 64 * kz;
        const float Wv = blk[kPoolW + i];
        if (!(Wv > 0.0f)) continue;
        const float a = w / Wv;
        const float g = gD[b * kBlockVox + i] * a;
        atomicAdd(grad_depth + (size_t)k * np + pix, g);
        if (CM == SC_COLOR_F32 && gC && grad_color) {
            float* gc = grad_color + ((size_t)k * np + pix) * 3;
            atomicAdd(gc + 0, gC[(b * 3 + 0) * kBlockVox + i] * a);
            atomicAdd(gc + 1, gC[(b * 3 + 1) * kBlockVox + i] * a);
            atomicAdd(gc + 2, gC[(b * 3 + 2) * kBlockVox + i] * a);
        }
        j2 += g;
        j3 += g * py;
        j4 -= g * px;
    }
    red[0][lane] = j2;
    red[1][lane] = j3;
    red[2][lane] = j4;
    __syncthreads();
    for (int off = 32; off > 0; off >>= 1) {
        if (lane < off) {
            red[0][lane] += red[0][lane + off];
            red[1][lane] += red[1][lane + off];
            red[2][lane] += red[2][lane + off];
        }
        __syncthreads();
    }
    if (lane < 3 && red[lane][0] != 0.0f) atomicAdd(acc_xi + 6 * k + 2 + lane, (double)red[lane][0]);
}

__global__ void xi_final_kernel(const double* acc, int n, float* out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 6 * n) out[i] += (float)acc[i];
}

__global__ void zero_f64_kernel(double* p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

}  // namespace sc

using namespace sc;

extern "C" {

sc_status tsdf_integrate_backward(sc_volume* vol, const sc_keyframe* kfs, int32_t n_kf, const sc_intrinsics* intr,
                                  const sc_pose* T, const float* grad_D, const float* grad_C, float* grad_depth,
                                  float* grad_color, float* grad_xi, void* stream)
{
    if (!vol || !kfs || n_kf <= 0 || n_kf > vol->p.max_batch_ops || n_kf > 65535 || !intr || intr->width <= 0 || intr->height <= 0 ||
        !T || !grad_D || !grad_depth || !grad_xi)
        return SC_EINVAL;
    if ((grad_C != nullptr) != (grad_color != nullptr)) return SC_EINVAL;
    for (int i = 0; i < n_kf; ++i)
        if (!keyframe_ok(&kfs[i])) return SC_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int64_t nb = 0;
    sc_status st = sc_volume_query(vol, s, &nb, nullptr);
    if (st != SC_OK) return st;
    OpDesc* ops = stage_begin(vol);
    if (!ops) return SC_EDEVICE;
    for (int k = 0; k < n_kf; ++k) make_op(vol, &kfs[k], intr, &T[k], +1, k, &ops[k]);
    if (hipMemcpyAsync(vol->d_ops, ops, sizeof(OpDesc) * n_kf, hipMemcpyHostToDevice, s) != hipSuccess)
        return SC_EDEVICE;
    st = stage_end(vol, s);
    if (st != SC_OK) return st;
    // FP64 pose accumulators live in the batch histogram scratch (>= 6 doubles per keyframe)
    double* acc = reinterpret_cast<double*>(vol->cand.sorted);
    zero_f64_kernel<<<(6 * n_kf + 255) / 256, 256, 0, s>>>(acc, 6 * n_kf);
    if (nb > 0) {
        const dim3 grid((unsigned)nb, (unsigned)n_kf);
        if (vol->p.color_mode == SC_COLOR_F32)
            backward_kernel<SC_COLOR_F32><<<grid, 64, 0, s>>>(vol->d_ops, vol->dev, grad_D, grad_C, grad_depth,
                                                              grad_color, acc);
        else
            backward_kernel<SC_COLOR_RGBA8><<<grid, 64, 0, s>>>(vol->d_ops, vol->dev, grad_D, nullptr, grad_depth,
                                                                nullptr, acc);
    }
    xi_final_kernel<<<(6 * n_kf + 255) / 256, 256, 0, s>>>(acc, n_kf, grad_xi);
    return hipGetLastError() == hipSuccess ? SC_OK : SC_EDEVICE;
}

}  // extern "C"
