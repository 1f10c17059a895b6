// Fourth-order diffusion tensor of Sec. 3.2 (Eqs. (7), (8)) in compact form,
// shared by the kernels that build it.
//
// With nu_1 >= nu_2 the eigenvalues of H_rho = [[a, b], [b, d]], mu_i the
// Perona-Malik diffusivities of Eq. (7) (mu_i = 1 where the mode masks nu_i),
// mu_3 = (mu_1 + mu_2) / 2 and mu_4 = 0, the tensor D = E M E^T acts on a
// symmetric Hessian h as
//   T_xx = (m + al) h_xx + be h_xy
//   T_xy = T_yx = m h_xy + be (h_xx + h_yy) / 2
//   T_yy = (m - al) h_yy + be h_xy
// where m = (mu_1 + mu_2) / 2 and (al, be) = (mu_1 - mu_2) / 2 * (cos 2t, sin 2t)
// for the angle t of the first eigenvector: expanding E M E^T for the
// rotation E gives exactly these entries.
//
// mu_1 - mu_2 is formed without cancellation: 1 - mu = q mu with
// q = nu^2 / lambda^2, and for two unmasked eigenvalues
// mu_1 - mu_2 = -4 m' r mu_1 mu_2 / lambda^2 (m' the mean and r the half
// difference of the eigenvalues), which also removes the division by r.
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/mf4d.h"

namespace mf4d {

template <int MODE>
__device__ __forceinline__ void tensor_coeffs(float a, float b, float d, float inv_lam2,
                                              float &mbar, float &al, float &be)
{
#pragma clang fp contract(off)   // fused multiply-adds are written out
    const float mm = 0.5f * (a + d);
    const float hd = 0.5f * (a - d);
    const float r = sqrtf(fmaf(hd, hd, b * b));
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

__device__ __forceinline__ void tensor_coeffs_mode(int mode, float a, float b, float d, float inv_lam2,
                                                   float &mbar, float &al, float &be)
{
    if (mode == MF4D_RIDGE) tensor_coeffs<MF4D_RIDGE>(a, b, d, inv_lam2, mbar, al, be);
    else if (mode == MF4D_VALLEY) tensor_coeffs<MF4D_VALLEY>(a, b, d, inv_lam2, mbar, al, be);
    else tensor_coeffs<MF4D_BOTH>(a, b, d, inv_lam2, mbar, al, be);
}

}  // namespace mf4d
