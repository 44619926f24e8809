// closure_data.hip -- training samples for the learned closure from a run at
// twice the resolution: 2x2x2 box filter of the fine velocity and of the fine
// model stress, coarse strain rate, eddy-viscosity target and features.
//
// Finite differences (both grids): central in the interior, periodic in x and
// z, one-sided in y at the first and last row (0 when ny = 1).  Lengths in
// units of each grid's cell; velocities are the same number on both grids
// (acoustic scaling), so stresses (velocity^2) need no conversion.
#include "lbm_device.h"

namespace lbmx {

namespace {

// du_a/dx_b of the velocity planes v (3 planes of n = nx*ny*nz) at (i,j,k)
template <class V>
__device__ __forceinline__ void grad_u(const V *v, long long n, int nx, int ny, int nz, int i,
                                       int j, int k, float (&g)[3][3]) {
    const int ip = i + 1 == nx ? 0 : i + 1, im = i == 0 ? nx - 1 : i - 1;
    const int kp = k + 1 == nz ? 0 : k + 1, km = k == 0 ? nz - 1 : k - 1;
    int jp = j + 1, jm = j - 1;
    float sy = 0.5f;
    if (ny == 1) {
        jp = jm = j;
        sy = 0.0f;
    } else if (j == 0) {
        jm = j;
        sy = 1.0f;
    } else if (j == ny - 1) {
        jp = j;
        sy = 1.0f;
    }
    auto at = [&](int a, int ii, int jj, int kk) -> float {
        return (float)v[a * n + ((long long)kk * ny + jj) * nx + ii];
    };
    for (int a = 0; a < 3; ++a) {
        g[a][0] = 0.5f * (at(a, ip, j, k) - at(a, im, j, k));
        g[a][1] = sy * (at(a, i, jp, k) - at(a, i, jm, k));
        g[a][2] = 0.5f * (at(a, i, j, kp) - at(a, i, j, km));
    }
}

// one thread per coarse cell: ub (3 planes) and tau (6 planes: xx yy zz xy xz yz)
template <class C>
__global__ __launch_bounds__(256) void filter_kernel(const C *__restrict__ mom, int nx, int ny,
                                                     int nz, float *__restrict__ ub,
                                                     float *__restrict__ tau) {
    const int cx = nx / 2, cy = ny / 2, cz = nz / 2;
    const long long nc = (long long)cx * cy * cz;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int I = (int)(c % cx), J = (int)((c / cx) % cy), K = (int)(c / ((long long)cx * cy));
    const long long n = (long long)nx * ny * nz;
    const C *u = mom + n;        // ux, uy, uz planes
    const C *nut = mom + 4 * n;  // nu_t plane
    float s_u[3] = {0, 0, 0}, s_t[6] = {0, 0, 0, 0, 0, 0};
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
                const long long x = ((long long)k * ny + j) * nx + i;
                s_u[0] += (float)u[x];
                s_u[1] += (float)u[n + x];
                s_u[2] += (float)u[2 * n + x];
                float g[3][3];
                grad_u(u, n, nx, ny, nz, i, j, k, g);
                const float m2 = -2.0f * (float)nut[x];
                s_t[0] += m2 * g[0][0];
                s_t[1] += m2 * g[1][1];
                s_t[2] += m2 * g[2][2];
                s_t[3] += m2 * 0.5f * (g[0][1] + g[1][0]);
                s_t[4] += m2 * 0.5f * (g[0][2] + g[2][0]);
                s_t[5] += m2 * 0.5f * (g[1][2] + g[2][1]);
            }
    const float e = 0.125f;
    const float ua = s_u[0] * e, va = s_u[1] * e, wa = s_u[2] * e;
    // box(u u) - ub ub as the block covariance about the block mean (no
    // cancellation of the two large terms in FP32)
    float cv[6] = {0, 0, 0, 0, 0, 0};
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                const long long x = ((long long)(2 * K + dk) * ny + 2 * J + dj) * nx + 2 * I + di;
                const float a = (float)u[x] - ua, b = (float)u[n + x] - va, w = (float)u[2 * n + x] - wa;
                cv[0] += a * a;
                cv[1] += b * b;
                cv[2] += w * w;
                cv[3] += a * b;
                cv[4] += a * w;
                cv[5] += b * w;
            }
    ub[c] = ua;
    ub[nc + c] = va;
    ub[2 * nc + c] = wa;
    for (int q = 0; q < 6; ++q) tau[q * nc + c] = (cv[q] + s_t[q]) * e;
}

// one thread per coarse cell: target and features
__global__ __launch_bounds__(256) void features_kernel(const float *__restrict__ ub,
                                                       const float *__restrict__ tau, int cx,
                                                       int cy, int cz, float tau0, float inv_h,
                                                       const double *__restrict__ lad,
                                                       float *__restrict__ X,
                                                       float *__restrict__ Y) {
    const long long nc = (long long)cx * cy * cz;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const int I = (int)(c % cx), J = (int)((c / cx) % cy), K = (int)(c / ((long long)cx * cy));
    float g[3][3];
    grad_u(ub, nc, cx, cy, cz, I, J, K, g);
    const float Sxx = g[0][0], Syy = g[1][1], Szz = g[2][2];
    const float Sxy = 0.5f * (g[0][1] + g[1][0]), Sxz = 0.5f * (g[0][2] + g[2][0]),
                Syz = 0.5f * (g[1][2] + g[2][1]);
    const float t[6] = {tau[c], tau[nc + c], tau[2 * nc + c], tau[3 * nc + c], tau[4 * nc + c],
                        tau[5 * nc + c]};
    const float tr3 = (t[0] + t[1] + t[2]) / 3.0f;
    const float dd = (t[0] - tr3) * Sxx + (t[1] - tr3) * Syy + (t[2] - tr3) * Szz +
                     2.0f * (t[3] * Sxy + t[4] * Sxz + t[5] * Syz);
    const float ss = Sxx * Sxx + Syy * Syy + Szz * Szz + 2.0f * (Sxy * Sxy + Sxz * Sxz + Syz * Syz);
    const float nus = ss > 1e-30f ? fmaxf(0.0f, -dd / (2.0f * ss)) : 0.0f;
    const float k = -2.0f * (tau0 + 3.0f * nus);
    const float a = k * Sxx, b = k * Syy, cc = k * Szz, d = k * Sxy, e = k * Sxz, f = k * Syz;
    const float q_xx = a * a + d * d + e * e, q_yy = d * d + b * b + f * f, q_zz = e * e + f * f + cc * cc;
    const float q_xy = a * d + d * b + e * f, q_xz = a * e + d * f + e * cc, q_yz = d * e + b * f + f * cc;
    const float tr2 = q_xx + q_yy + q_zz;
    float *x = X + c * 9;
    x[0] = a + b + cc;
    x[1] = tr2;
    x[2] = q_xx * a + q_yy * b + q_zz * cc + 2.0f * (q_xy * d + q_xz * e + q_yz * f);
    x[3] = b;
    x[4] = q_yy;
    x[5] = sqrtf(tr2);
    x[6] = ((float)J + 0.5f) * inv_h;
    x[7] = (float)lad[J];
    x[8] = 1.0f;
    Y[c] = nus;
}

}  // namespace

hipError_t launch_closure_samples(int storage, const void *mom, int nx, int ny, int nz,
                                  float *work, double tau0_coarse, double inv_h,
                                  const double *lad_coarse, float *X, float *Y, hipStream_t s) {
    const long long nc = (long long)(nx / 2) * (ny / 2) * (nz / 2);
    float *ub = work, *tau = work + 3 * nc;
    const unsigned grid = (unsigned)((nc + 255) / 256);
    if (storage == ST_F64)
        hipLaunchKernelGGL(filter_kernel<double>, dim3(grid), dim3(256), 0, s,
                           static_cast<const double *>(mom), nx, ny, nz, ub, tau);
    else
        hipLaunchKernelGGL(filter_kernel<float>, dim3(grid), dim3(256), 0, s,
                           static_cast<const float *>(mom), nx, ny, nz, ub, tau);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(features_kernel, dim3(grid), dim3(256), 0, s, ub, tau, nx / 2, ny / 2,
                       nz / 2, (float)tau0_coarse, (float)inv_h, lad_coarse, X, Y);
    return hipGetLastError();
}

}  // namespace lbmx
