// Internal declarations shared by the HIP translation units of libmf4d.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/mf4d.h"

namespace mf4d {

constexpr int kMaxR = MF4D_MAX_RADIUS;   // Gaussian radius limit
constexpr int kMaxRhoR = 8;              // integration-scale radius limit

// Separable filter taps of one scale, correlation form out[x] = sum_i k[i] in[x+i]:
//   g[i]  Gaussian G_sigma, i = 0..r (symmetric)
//   d1[i] central difference of G: (g[i-1] - g[i+1]) / 2, i = 1..r+1 (antisymmetric)
//   d2[i] second difference of G: g[i-1] - 2 g[i] + g[i+1], i = 1..r+1 (symmetric,
//         applied around the centre value so the filter sums to zero exactly)
struct Taps {
    int r;
    float g[kMaxR + 2];
    float d1[kMaxR + 2];
    float d2[kMaxR + 2];
};

struct RhoTaps {
    int r;  // 0: identity
    float g[kMaxRhoR + 1];
};

// Per-scale planes written by the scale sweep.
struct ScalePlanes {
    float *S;   // [H][W] Frobenius norm of sigma^2 H(u_sigma)
    float *A;   // [H][W] blob factor exp(-R_B^2 / 2 beta^2), 0 if the sign test fails
    float *N;   // [3][H][W] H(u_sigma) / sqrt(1 + |grad u_sigma|), or nullptr
};

// Horizontal pass of one scale: A = G u, B = D1G u, C = D2G u along x.
hipError_t launch_hpass(const float *u, float *A, float *B, float *C, int H, int W,
                        const Taps &t, hipStream_t s);

// Vertical pass of one scale plus the per-pixel vesselness ingredients.
hipError_t launch_vpass(const float *A, const float *B, const float *C, int H, int W,
                        const Taps &t, float sigma, int mode, float beta, ScalePlanes out,
                        unsigned *smax_bits, hipStream_t s);

hipError_t launch_fill_u32(unsigned *p, unsigned v, size_t n, hipStream_t s);
hipError_t launch_copy_f32(const float *src, float *dst, size_t n, hipStream_t s);

// Argmax over scales and/or normalised Hessian integration at the chosen scale.
//   idx_in  != nullptr: use these indices (no argmax)
//   idx_out != nullptr: write indices (tile interior)
//   hrho    != nullptr: write H_rho (needs N planes)
//   dparams != nullptr: write the compact tensor of H_rho
struct SelectArgs {
    const float *S;      // [ns][H][W]
    const float *A;      // [ns][H][W]
    const float *N;      // [ns][3][H][W]
    int ns;
    const unsigned *smax_bits;
    float c_param;
    const uint8_t *idx_in;
    uint8_t *idx_out;
    float *vmax_out;
    float *c_out;
    float *hrho;
    float *dparams;
    int mode;
    float inv_lam2;
    RhoTaps rho;
};
hipError_t launch_select(const SelectArgs &a, int H, int W, hipStream_t s);

// One FED substep u_out = u_in - tau L^T D L u_in with D from H_rho.
hipError_t launch_fed_substep(const float *u_in, float *u_out, const float *hrho, int H, int W,
                              float tau, int mode, float inv_lam2, hipStream_t s);

// Compact tensor planes (m, al, be) of H_rho.
hipError_t launch_dparams(const float *hrho, float *dp, int H, int W, int mode, float inv_lam2,
                          hipStream_t s);

}  // namespace mf4d
