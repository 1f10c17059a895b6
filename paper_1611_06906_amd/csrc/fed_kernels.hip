// Fused FED substep (Sec. 3.4, Sec. 3.5 Eq. (21)):
//   u_out = u_in - tau * L^T D L u_in
// with the per-pixel fourth-order tensor D of Eqs. (7), (8) rebuilt in
// registers from the normalised, integrated Hessian H_rho = [[a, b], [b, d]].
//
// Rows of L exist only at interior pixels (natural boundary condition), so
// T = D L u is zero outside 1 <= x <= W-2, 1 <= y <= H-2, and L^T reaches
// the border pixels through the transposed stencils.
//
// Tensor in compact form. With mu_1, mu_2 the diffusivities of the two
// eigenvalues nu_1 >= nu_2 of H_rho, mu_3 = (mu_1 + mu_2) / 2 and mu_4 = 0,
// D acts on a symmetric Hessian h as
//   T_xx = (m + al) h_xx + be h_xy
//   T_xy = T_yx = m h_xy + be (h_xx + h_yy) / 2
//   T_yy = (m - al) h_yy + be h_xy
// where m = (mu_1 + mu_2) / 2 and (al, be) = (mu_1 - mu_2) / 2 * (cos 2t, sin 2t)
// for the angle t of the first eigenvector: expanding D = E M E^T for the
// rotation E gives exactly these entries. (mu_1 - mu_2) is formed without
// cancellation: 1 - mu = q mu with q = nu^2 / lambda^2, and for two unmasked
// eigenvalues mu_1 - mu_2 = -4 m' r mu_1 mu_2 / lambda^2 (m' the mean and r the
// half-difference of the eigenvalues), which also removes the division by r.
#include "mf4d_internal.h"

namespace mf4d {

namespace {

constexpr int kTW = 64, kTH = 16;   // output tile

template <int MODE>
__device__ __forceinline__ void tensor_coeffs(float a, float b, float d, float inv_lam2,
                                              float &mbar, float &al, float &be)
{
    const float mm = 0.5f * (a + d);
    const float hd = 0.5f * (a - d);
    const float r = sqrtf(hd * hd + b * b);
    const float nu1 = mm + r, nu2 = mm - r;
    const float q1 = nu1 * nu1 * inv_lam2, q2 = nu2 * nu2 * inv_lam2;
    float mu1 = 1.f / (1.f + q1), mu2 = 1.f / (1.f + q2);
    bool k1 = false, k2 = false;   // masked eigenvalue: mu = 1
    if (MODE == MF4D_RIDGE) { k1 = nu1 >= 0.f; k2 = nu2 >= 0.f; }
    if (MODE == MF4D_VALLEY) { k1 = nu1 <= 0.f; k2 = nu2 <= 0.f; }
    if (!k1 && !k2) {
        const float k = -2.f * mm * mu1 * mu2 * inv_lam2;
        mbar = 0.5f * (mu1 + mu2);
        al = k * hd;
        be = k * b;
    } else if (k1 && k2) {
        mbar = 1.f;
        al = 0.f;
        be = 0.f;
    } else {
        float half_diff;   // (mu_1 - mu_2) / 2
        if (k1) { half_diff = 0.5f * q2 * mu2; mu1 = 1.f; }
        else { half_diff = -0.5f * q1 * mu1; mu2 = 1.f; }
        mbar = 0.5f * (mu1 + mu2);
        const float ir = r > 0.f ? 1.f / r : 0.f;
        al = half_diff * hd * ir;
        be = half_diff * b * ir;
    }
}

template <int MODE>
__global__ __launch_bounds__(256) void fed_substep_kernel(const float *__restrict__ u,
                                                          float *__restrict__ uo,
                                                          const float *__restrict__ hrho,
                                                          int H, int W, float tau, float inv_lam2,
                                                          int tiles_x, int ntiles, int per_xcd)
{
    __shared__ float su[kTH + 4][kTW + 4 + 1];
    __shared__ float sT[3][kTH + 2][kTW + 2 + 1];
    // XCD-aware order: consecutive blocks land on different XCDs, so give each
    // XCD a contiguous band of tiles to keep halo re-reads in its own L2.
    const int tile = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (tile >= ntiles) return;
    const int x0 = (tile % tiles_x) * kTW, y0 = (tile / tiles_x) * kTH;
    const size_t plane = (size_t)H * W;

    for (int i = threadIdx.x; i < (kTH + 4) * (kTW + 4); i += 256) {
        const int ly = i / (kTW + 4), lx = i % (kTW + 4);
        const int gy = y0 - 2 + ly, gx = x0 - 2 + lx;
        su[ly][lx] = (gy >= 0 && gy < H && gx >= 0 && gx < W) ? u[(size_t)gy * W + gx] : 0.f;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < (kTH + 2) * (kTW + 2); i += 256) {
        const int ly = i / (kTW + 2), lx = i % (kTW + 2);
        const int gy = y0 - 1 + ly, gx = x0 - 1 + lx;
        float txx = 0.f, txy = 0.f, tyy = 0.f;
        if (gx >= 1 && gx <= W - 2 && gy >= 1 && gy <= H - 2) {
            const float c = su[ly + 1][lx + 1];
            const float hxx = su[ly + 1][lx] - 2.f * c + su[ly + 1][lx + 2];
            const float hyy = su[ly][lx + 1] - 2.f * c + su[ly + 2][lx + 1];
            const float hxy = 0.25f * ((su[ly][lx] + su[ly + 2][lx + 2]) - (su[ly + 2][lx] + su[ly][lx + 2]));
            const size_t o = (size_t)gy * W + gx;
            float mbar, al, be;
            tensor_coeffs<MODE>(hrho[o], hrho[plane + o], hrho[2 * plane + o], inv_lam2, mbar, al, be);
            txx = (mbar + al) * hxx + be * hxy;
            txy = mbar * hxy + be * 0.5f * (hxx + hyy);
            tyy = (mbar - al) * hyy + be * hxy;
        }
        sT[0][ly][lx] = txx;
        sT[1][ly][lx] = txy;
        sT[2][ly][lx] = tyy;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kTH * kTW; i += 256) {
        const int ly = i / kTW, lx = i % kTW;
        const int gy = y0 + ly, gx = x0 + lx;
        if (gy >= H || gx >= W) continue;
        const float rxx = sT[0][ly + 1][lx] - 2.f * sT[0][ly + 1][lx + 1] + sT[0][ly + 1][lx + 2];
        const float ryy = sT[2][ly][lx + 1] - 2.f * sT[2][ly + 1][lx + 1] + sT[2][ly + 2][lx + 1];
        const float rxy = 0.5f * ((sT[1][ly][lx] + sT[1][ly + 2][lx + 2]) - (sT[1][ly + 2][lx] + sT[1][ly][lx + 2]));
        const float r = rxx + rxy + ryy;
        uo[(size_t)gy * W + gx] = su[ly + 2][lx + 2] - tau * r;
    }
}

template <int MODE>
__global__ void dparams_kernel(const float *__restrict__ hrho, float *__restrict__ dp, size_t plane,
                               float inv_lam2)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= plane) return;
    float mbar, al, be;
    tensor_coeffs<MODE>(hrho[i], hrho[plane + i], hrho[2 * plane + i], inv_lam2, mbar, al, be);
    dp[i] = mbar;
    dp[plane + i] = al;
    dp[2 * plane + i] = be;
}

}  // namespace

hipError_t launch_fed_substep(const float *u_in, float *u_out, const float *hrho, int H, int W,
                              float tau, int mode, float inv_lam2, hipStream_t s)
{
    const int tiles_x = (W + kTW - 1) / kTW, tiles_y = (H + kTH - 1) / kTH;
    const int ntiles = tiles_x * tiles_y;
    const int per = (ntiles + 7) / 8;
    dim3 grid(8 * per), block(256);
    switch (mode) {
    case MF4D_RIDGE:
        hipLaunchKernelGGL(fed_substep_kernel<MF4D_RIDGE>, grid, block, 0, s, u_in, u_out, hrho, H, W,
                           tau, inv_lam2, tiles_x, ntiles, per);
        break;
    case MF4D_VALLEY:
        hipLaunchKernelGGL(fed_substep_kernel<MF4D_VALLEY>, grid, block, 0, s, u_in, u_out, hrho, H, W,
                           tau, inv_lam2, tiles_x, ntiles, per);
        break;
    default:
        hipLaunchKernelGGL(fed_substep_kernel<MF4D_BOTH>, grid, block, 0, s, u_in, u_out, hrho, H, W,
                           tau, inv_lam2, tiles_x, ntiles, per);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_dparams(const float *hrho, float *dp, int H, int W, int mode, float inv_lam2,
                          hipStream_t s)
{
    const size_t plane = (size_t)H * W;
    dim3 grid((unsigned)((plane + 255) / 256)), block(256);
    switch (mode) {
    case MF4D_RIDGE:
        hipLaunchKernelGGL(dparams_kernel<MF4D_RIDGE>, grid, block, 0, s, hrho, dp, plane, inv_lam2);
        break;
    case MF4D_VALLEY:
        hipLaunchKernelGGL(dparams_kernel<MF4D_VALLEY>, grid, block, 0, s, hrho, dp, plane, inv_lam2);
        break;
    default:
        hipLaunchKernelGGL(dparams_kernel<MF4D_BOTH>, grid, block, 0, s, hrho, dp, plane, inv_lam2);
        break;
    }
    return hipGetLastError();
}

}  // namespace mf4d
