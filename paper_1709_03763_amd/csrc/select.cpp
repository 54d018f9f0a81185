// Keyframe selection for re-integration (Sec. 4.3, Eq. 3 and Fig. 4), host
// code in FP64.  The pose change of keyframe i is ||s o t_i - s o t_i'||
// with t the Euler angles and the translation of the pose and
// s = (2, 2, 2, 1, 1, 1).  Euler angles are read as Z-Y-X (yaw, pitch,
// roll), R = Rz(yaw) Ry(pitch) Rx(roll), and differences are wrapped to
// (-pi, pi].  Window sums are summed in index order.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <numeric>
#include <vector>

#include "scsurf.h"

namespace {

void euler_zyx(const double* R, double e[3])
{
    e[2] = atan2(R[3], R[0]);                     // yaw   = atan2(R10, R00)
    e[1] = atan2(-R[6], hypot(R[0], R[3]));       // pitch = atan2(-R20, |(R00, R10)|)
    e[0] = atan2(R[7], R[8]);                     // roll  = atan2(R21, R22)
}

double wrap_angle(double d)
{
    if (d > M_PI)
        d -= 2 * M_PI;
    else if (d <= -M_PI)
        d += 2 * M_PI;
    return d;
}

double pose_change(const sc_pose& a, const sc_pose& b)
{
    double ea[3], eb[3];
    euler_zyx(a.R, ea);
    euler_zyx(b.R, eb);
    const double s[6] = {2.0, 2.0, 2.0, 1.0, 1.0, 1.0};
    double diff[6];
    for (int k = 0; k < 3; ++k) diff[k] = wrap_angle(ea[k] - eb[k]);
    for (int k = 0; k < 3; ++k) diff[3 + k] = a.t[k] - b.t[k];
    double acc = 0.0;
    for (int k = 0; k < 6; ++k) {
        const double v = s[k] * diff[k];
        acc += v * v;
    }
    return sqrt(acc);
}

}  // namespace

extern "C" {

int32_t sc_select_dist(const double* dist, int32_t K, int32_t m, int32_t mode, int32_t* out)
{
    if (!dist || !out || K < 0 || m <= 0) return SC_EINVAL;
    if (K == 0) return 0;
    if (mode == SC_SEL_EQ3) {
        if (K <= m) {
            for (int i = 0; i < K; ++i) out[i] = i;
            return K;
        }
        int best = 0;
        double best_sum = -1.0;
        for (int j = 0; j + m <= K; ++j) {
            double s = 0.0;
            for (int i = j; i < j + m; ++i) s += dist[i];
            if (s > best_sum) {
                best_sum = s;
                best = j;
            }
        }
        for (int i = 0; i < m; ++i) out[i] = best + i;
        return m;
    }
    if (mode != SC_SEL_TOPM && mode != SC_SEL_ALL_ORDERED) return SC_EINVAL;
    std::vector<int32_t> idx(K);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int32_t a, int32_t b) { return dist[a] > dist[b]; });
    int n = 0;
    if (mode == SC_SEL_TOPM) {
        n = std::min(K, m);
        for (int i = 0; i < n; ++i) out[i] = idx[i];
    } else {
        for (int i = 0; i < K; ++i)
            if (dist[idx[i]] > 0.0) out[n++] = idx[i];
    }
    return n;
}

sc_status sc_relative_motion(const sc_pose* T_kf, const sc_pose* T, double* trans, double* angle)
{
    if (!T_kf || !T || !trans || !angle) return SC_EINVAL;
    // A = R_kf^T R, d = R_kf^T (t - t_kf)
    double A[9], d[3];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c)
            A[3 * r + c] = T_kf->R[r] * T->R[c] + T_kf->R[3 + r] * T->R[3 + c] + T_kf->R[6 + r] * T->R[6 + c];
        d[r] = T_kf->R[r] * (T->t[0] - T_kf->t[0]) + T_kf->R[3 + r] * (T->t[1] - T_kf->t[1]) +
               T_kf->R[6 + r] * (T->t[2] - T_kf->t[2]);
    }
    // R - R^T = 2 sin(theta) [axis]x and trace(R) = 1 + 2 cos(theta)
    const double sx = A[7] - A[5], sy = A[2] - A[6], sz = A[3] - A[1];
    const double s2 = sqrt(sx * sx + sy * sy + sz * sz) / 2.0;
    const double c2 = (A[0] + A[4] + A[8] - 1.0) / 2.0;
    *trans = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    *angle = atan2(s2, c2);
    return SC_OK;
}

int32_t sc_select(const sc_pose* T, const sc_pose* T_new, int32_t K, int32_t m, int32_t mode, int32_t* out,
                  double* dist_out)
{
    if (!T || !T_new || !out || K < 0) return SC_EINVAL;
    std::vector<double> d(K);
    for (int i = 0; i < K; ++i) d[i] = pose_change(T[i], T_new[i]);
    if (dist_out) memcpy(dist_out, d.data(), sizeof(double) * K);
    return sc_select_dist(d.data(), K, m, mode, out);
}

}  // extern "C"
