// Tile-level device code of the scale sweep and of the normalised, integrated
// Hessian (Sec. 3.3 Eq. (9), Eq. (6)), shared by the single-image kernels and
// the batched kernels so that both compute identical values.
//
// Per scale sigma the five derivatives of u_sigma = u * G_sigma are formed by
// two separable passes with combined taps (Gaussian, its central difference
// and its second difference), which equals blurring first and differencing
// afterwards under the half-sample symmetric extension.
//
// Both passes are register-window convolutions: a thread produces kWin = 16
// consecutive outputs of one line and streams the line's inputs through a
// 16-entry register window, so every input value loaded is used by up to 16
// outputs and the taps are wave-uniform kernel arguments. Inputs are shifted
// by a per-line reference value before the difference filters, which makes
// the derivatives of locally constant lines exactly zero.
//
// The vertical pass also evaluates the per-pixel ingredients of the
// vesselness that do not depend on the image-wide c (S and the blob factor)
// and the normalised Hessian N. Once c is known, a per-pixel step takes the
// argmax over scales and gathers N at the chosen scale, and a tiled step
// integrates it with G_rho and builds the compact tensor planes.
#pragma once

#include "mf4d_internal.h"
#include "tensor_math.h"

namespace mf4d {
namespace tiles {

constexpr int K = kWin;
constexpr int kBTW = 64, kBTH = 16;   // rho-blur output tile

// vector types for the nontemporal accesses of the per-scale planes
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef float nt_f3 __attribute__((ext_vector_type(3)));

// half-sample symmetric extension (period 2n), cheap for small excursions
__device__ __forceinline__ int reflect(int i, int n)
{
    while (i < 0 || i >= n) i = (i < 0) ? -i - 1 : 2 * n - 1 - i;
    return i;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// ------------------------------------------------------------------ horizontal
// Tile: 64 rows x 64 output columns at (x0, y0); lane = row, wave w owns
// columns 16w .. 16w+15. The rows' inputs are staged in `tile` (LDS, 64 x
// (ntaps + 65) floats) with an odd pitch.
__device__ __forceinline__ void hpass_tile(const float *__restrict__ u, float *__restrict__ A,
                                          float *__restrict__ B, float *__restrict__ C, int H, int W,
                                          const WinTaps &t, int x0, int y0, float *tile)
{
#pragma clang fp contract(off)   // fused multiply-adds are written out
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int R = t.R, nt = t.ntaps;
    const int cols = nt + 64;     // columns x0-R .. x0-R+cols-1
    const int P = cols + 1;       // odd pitch: row-per-lane reads are conflict free
    const bool interior = (x0 - R >= 0) && (x0 - R + cols <= W);
    for (int ry = wv * 16; ry < wv * 16 + 16; ++ry) {
        const int gy = min(y0 + ry, H - 1);
        const float *urow = u + (size_t)gy * W;
        for (int c = lane; c < cols; c += 64) {
            const int gx = x0 - R + c;
            tile[ry * P + c] = urow[interior ? gx : reflect(gx, W)];
        }
    }
    __syncthreads();
    const float *row = tile + lane * P + wv * K;   // row[j] = input at x0 + 16 wv - R + j
    const float ref = row[R];                      // centre of this thread's first output
    float win[K], ag[K], ad1[K], ad2[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        win[k] = row[k] - ref;
        ag[k] = ad1[k] = ad2[k] = 0.f;
    }
    for (int t0 = 0; t0 < nt; t0 += K) {
#pragma unroll
        for (int t1 = 0; t1 < K; ++t1) {
            const float g = t.g[t0 + t1], d1 = t.d1[t0 + t1], d2 = t.d2[t0 + t1];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const float v = win[(k + t1) & (K - 1)];
                ag[k] = fmaf(g, v, ag[k]);
                ad1[k] = fmaf(d1, v, ad1[k]);
                ad2[k] = fmaf(d2, v, ad2[k]);
            }
            win[t1] = row[t0 + t1 + K] - ref;
        }
    }
    // transpose the 64 x 64 outputs through LDS so that stores are row-contiguous
    const float gref = ref * t.gsum;
    float *ot = tile;   // reused: [64][65]
#pragma unroll
    for (int f = 0; f < 3; ++f) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k)
            ot[lane * 65 + wv * K + k] = (f == 0) ? ag[k] + gref : (f == 1 ? ad1[k] : ad2[k]);
        __syncthreads();
        float *dst = (f == 0) ? A : (f == 1 ? B : C);
        for (int i = threadIdx.x; i < 64 * 64; i += 256) {
            const int ry = i >> 6, cx = i & 63;
            const int y = y0 + ry, x = x0 + cx;
            if (y < H && x < W) dst[(size_t)y * W + x] = ot[ry * 65 + cx];
        }
    }
}

// ------------------------------------------------------------------ per pixel
// Vesselness ingredients that do not depend on the image-wide c (Eq. (9)):
// S = |sigma^2 H|_F and the blob factor (0 where the mode's sign test fails),
// and the normalised Hessian N = H / sqrt(1 + |grad u_sigma|) (Eq. (6)),
// stored at pixel o. Returns S.
template <int MODE>
__device__ __forceinline__ float vessel_store(float uxx, float uxy, float uyy, float gx, float gy, float sigma2,
                                              float inv2beta2, float *__restrict__ SA, float *__restrict__ No,
                                              size_t o, size_t plane)
{
#pragma clang fp contract(off)   // fused multiply-adds are written out
    // The hardware square root, reciprocal, reciprocal square root and 2^x
    // (about 1 ulp each) replace the correctly rounded library sequences.
    constexpr float kLog2e = 1.4426950408889634f;
    // scale-normalised Hessian sigma^2 H; eigenvalues m +- r
    const float hxx = sigma2 * uxx, hxy = sigma2 * uxy, hyy = sigma2 * uyy;
    const float m = 0.5f * (hxx + hyy);
    const float hd = 0.5f * (hxx - hyy);
    const float r = __builtin_amdgcn_sqrtf(fmaf(hd, hd, hxy * hxy));
    const float Sv = __builtin_amdgcn_sqrtf(fmaf(2.f * hxy, hxy, fmaf(hxx, hxx, hyy * hyy)));   // sqrt(nu~1^2 + nu~2^2)
    // |nu~2| = |m| + r carries the sign of m (a zero trace passes the test)
    const float am = fabsf(m);
    const float big = am + r;
    bool pass = big > 0.f;
    if (MODE == MF4D_RIDGE) pass = pass && !(m > 0.f);
    if (MODE == MF4D_VALLEY) pass = pass && !(m < 0.f);
    const float rb = (am - r) * __builtin_amdgcn_rcpf(big);   // |R_B| = |nu~1| / |nu~2|
    const float e = __builtin_amdgcn_exp2f(-(rb * rb) * inv2beta2 * kLog2e);
    const float blob = pass ? e : 0.f;
    // S and the blob factor per pixel ([H][W][2]), written once and read once
    __builtin_nontemporal_store(nt_f2{Sv, blob}, (nt_f2 *)(SA + 2 * o));
    if (No) {
        const float f = __builtin_amdgcn_rsqf(1.f + __builtin_amdgcn_sqrtf(fmaf(gx, gx, gy * gy)));
        __builtin_nontemporal_store(nt_f3{uxx * f, uxy * f, uyy * f}, (nt_f3 *)(No + 3 * o));   // [H][W][3]
    }
    return Sv;
}

// The same per-pixel values for a runtime mode, without branches: the mode's
// sign test is a select, so one copy of the code serves every mode.
struct VesselPx {
    float S, blob, n0, n1, n2;
};

__device__ __forceinline__ VesselPx vessel_px(int mode, float uxx, float uxy, float uyy, float gx, float gy,
                                              float sigma2, float inv2beta2)
{
#pragma clang fp contract(off)   // fused multiply-adds are written out
    constexpr float kLog2e = 1.4426950408889634f;
    const float hxx = sigma2 * uxx, hxy = sigma2 * uxy, hyy = sigma2 * uyy;
    const float m = 0.5f * (hxx + hyy);
    const float hd = 0.5f * (hxx - hyy);
    const float r = __builtin_amdgcn_sqrtf(fmaf(hd, hd, hxy * hxy));
    const float Sv = __builtin_amdgcn_sqrtf(fmaf(2.f * hxy, hxy, fmaf(hxx, hxx, hyy * hyy)));
    const float am = fabsf(m);
    const float big = am + r;
    const bool sign_ok = mode == MF4D_RIDGE ? !(m > 0.f) : (mode == MF4D_VALLEY ? !(m < 0.f) : true);
    const bool pass = big > 0.f && sign_ok;
    const float rb = (am - r) * __builtin_amdgcn_rcpf(big);
    const float e = __builtin_amdgcn_exp2f(-(rb * rb) * inv2beta2 * kLog2e);
    const float f = __builtin_amdgcn_rsqf(1.f + __builtin_amdgcn_sqrtf(fmaf(gx, gx, gy * gy)));
    return VesselPx{Sv, pass ? e : 0.f, uxx * f, uxy * f, uyy * f};
}

__device__ __forceinline__ float vessel_store_mode(int mode, float uxx, float uxy, float uyy, float gx, float gy,
                                                   float sigma2, float inv2beta2, float *__restrict__ SA,
                                                   float *__restrict__ No, size_t o, size_t plane)
{
    const VesselPx v = vessel_px(mode, uxx, uxy, uyy, gx, gy, sigma2, inv2beta2);
    // every scale's planes are written once and read once, after all scales:
    // nontemporal stores keep them from evicting the sweep's working set
    __builtin_nontemporal_store(nt_f2{v.S, v.blob}, (nt_f2 *)(SA + 2 * o));
    if (No) __builtin_nontemporal_store(nt_f3{v.n0, v.n1, v.n2}, (nt_f3 *)(No + 3 * o));   // N per pixel: [H][W][3]
    return v.S;
}

// ------------------------------------------------------------------ vertical
// Tile: 64 output columns x 64 rows at (x0, ty0); lane = column, wave w owns
// rows 16w .. 16w+15, streamed from global memory through the register
// window. Returns the largest S this thread wrote (0 if none).
template <int MODE>
__device__ __forceinline__ float vpass_tile(const float *__restrict__ A, const float *__restrict__ B,
                                            const float *__restrict__ C, int H, int W, const WinTaps &t,
                                            float sigma2, float inv2beta2, float *__restrict__ SA,
                                            float *__restrict__ No, int x0, int ty0)
{
#pragma clang fp contract(off)   // fused multiply-adds are written out
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int x = x0 + lane;
    const int xc = min(x, W - 1);
    const int y0 = ty0 + wv * K;
    const int R = t.R, nt = t.ntaps;
    const int base = y0 - R;
    const bool interior = (base >= 0) && (base + nt + K <= H);
    const size_t ro = (size_t)reflect(min(y0, H - 1), H) * W + xc;
    const float aref = A[ro], bref = B[ro];
    float wa[K], wb[K], wc[K];
    float ux[K], uxx[K], uy[K], uyy[K], uxy[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int gy = interior ? base + k : reflect(base + k, H);
        const size_t o = (size_t)gy * W + xc;
        wa[k] = A[o] - aref;
        wb[k] = B[o] - bref;
        wc[k] = C[o];
        ux[k] = uxx[k] = uy[k] = uyy[k] = uxy[k] = 0.f;
    }
    for (int t0 = 0; t0 < nt; t0 += K) {
#pragma unroll
        for (int t1 = 0; t1 < K; ++t1) {
            const float g = t.g[t0 + t1], d1 = t.d1[t0 + t1], d2 = t.d2[t0 + t1];
#pragma unroll
            for (int k = 0; k < K; ++k) {
                const int s = (k + t1) & (K - 1);
                ux[k] = fmaf(g, wb[s], ux[k]);
                uxx[k] = fmaf(g, wc[s], uxx[k]);
                uy[k] = fmaf(d1, wa[s], uy[k]);
                uxy[k] = fmaf(d1, wb[s], uxy[k]);
                uyy[k] = fmaf(d2, wa[s], uyy[k]);
            }
            const int j = base + t0 + t1 + K;
            const int gy = interior ? j : reflect(j, H);
            const size_t o = (size_t)gy * W + xc;
            wa[t1] = A[o] - aref;
            wb[t1] = B[o] - bref;
            wc[t1] = C[o];
        }
    }
    const float bsum = bref * t.gsum;
    const size_t plane = (size_t)H * W;
    float smax = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int y = y0 + k;
        if (x < W && y < H) {
            const float Sv = vessel_store<MODE>(uxx[k], uxy[k], uyy[k], ux[k] + bsum, uy[k], sigma2, inv2beta2,
                                                SA, No, (size_t)y * W + x, plane);
            smax = fmaxf(smax, Sv);
        }
    }
    return smax;
}

// folds one value per thread into *smax_bits (S >= 0: the float order equals
// the unsigned order of its bits)
__device__ __forceinline__ void block_max_to(float v, unsigned *smax_bits)
{
    __shared__ float red[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    float mx = wave_max(v);
    if (lane == 0) red[wv] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        atomicMax(smax_bits, __float_as_uint(mx));
    }
}

// ---------------------------------------------------------------- select
__device__ __forceinline__ float frangi_v(float S, float blob, float inv2c2)
{
#pragma clang fp contract(off)
    // V = blob * (1 - exp(-S^2 / (2 c^2)))
    return blob * -expm1f(-(S * S) * inv2c2);
}

// argmax over scales at pixel o (smallest index among equal maxima); writes
// the maximum to *vbest. c = 0 makes every V zero (index 0). Every scale's
// loads are issued before the comparisons.
__device__ __forceinline__ int argmax_px(const float *__restrict__ SA, int ns, size_t plane, size_t o, float c,
                                         float *vbest)
{
    int best = 0;
    float bv = 0.f;
    if (c > 0.f) {
        // (S, blob) of every scale, loaded before the comparisons; each pair is
        // read once, so the loads are nontemporal
        nt_f2 sa[MF4D_MAX_SCALES];
#pragma unroll
        for (int s = 0; s < MF4D_MAX_SCALES; ++s)
            if (s < ns) sa[s] = __builtin_nontemporal_load((const nt_f2 *)(SA + 2 * (s * plane + o)));
        const float inv2c2 = 1.f / (2.f * c * c);
        bv = frangi_v(sa[0].x, sa[0].y, inv2c2);
#pragma unroll
        for (int s = 1; s < MF4D_MAX_SCALES; ++s)
            if (s < ns) {
                const float v = frangi_v(sa[s].x, sa[s].y, inv2c2);
                if (v > bv) { bv = v; best = s; }
            }
    }
    *vbest = bv;
    return best;
}

// H_rho = G_rho * N (separable, symmetric extension) on the kBTW x kBTH tile
// at (x0, y0); writes H_rho and/or the compact tensor planes of H_rho. The
// tile's inputs (with a halo of HR) are staged in LDS; thread (x, g) blurs
// rows RG g - HR .. RG g + RG - 1 + HR (RG = kBTH / 4) of column x
// horizontally into registers and then vertically, so only one LDS buffer
// is needed.
// N holds all ns scales, per pixel ([ns][H][W][3]); each staged pixel takes
// the three values of its scale idx (clamped to ns - 1).
template <int HR>
__device__ __forceinline__ void rho_blur_tile(const float *__restrict__ N, const uint8_t *__restrict__ idx, int ns,
                                              float *__restrict__ Hr, float *__restrict__ coef, int mode,
                                              float inv_lam2, int H, int W, const RhoTaps &t, int x0, int y0)
{
#pragma clang fp contract(off)   // fused multiply-adds are written out
    constexpr int PW = kBTW + 2 * HR, PH = kBTH + 2 * HR;
    constexpr int RG = kBTH / 4;       // output rows per thread
    constexpr int RH = RG + 2 * HR;    // rows blurred horizontally per thread
    __shared__ float sN[3][PH][PW + 1];
    const size_t plane = (size_t)H * W;
    const bool interior = x0 - HR >= 0 && y0 - HR >= 0 && x0 + kBTW + HR <= W && y0 + kBTH + HR <= H;
    // all loads of the staged tile are issued before any LDS store (the
    // scale indices first)
    constexpr int NI = (PW * PH + 255) / 256;
    float v0[NI], v1[NI], v2[NI];
    size_t off[NI];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int i = min((int)threadIdx.x + 256 * it, PW * PH - 1);
        const int ly = i / PW, lx = i - ly * PW;
        const int gy = interior ? y0 - HR + ly : reflect(y0 - HR + ly, H);
        const int gx = interior ? x0 - HR + lx : reflect(x0 - HR + lx, W);
        off[it] = (size_t)gy * W + gx;
    }
    int sc[NI];
#pragma unroll
    for (int it = 0; it < NI; ++it) sc[it] = min((int)idx[off[it]], ns - 1);
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const float *Np = N + 3 * ((size_t)sc[it] * plane + off[it]);
        v0[it] = Np[0];
        v1[it] = Np[1];
        v2[it] = Np[2];
    }
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int i = (int)threadIdx.x + 256 * it;
        if (i < PW * PH) {
            const int ly = i / PW, lx = i - ly * PW;
            sN[0][ly][lx] = v0[it];
            sN[1][ly][lx] = v1[it];
            sN[2][ly][lx] = v2[it];
        }
    }
    __syncthreads();
    const int lx = threadIdx.x & 63, g = threadIdx.x >> 6;
    float h[3][RG];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        float sT[RH];   // horizontal blur of staged rows RG g .. RG g + RH - 1
#pragma unroll
        for (int r = 0; r < RH; ++r) {
            const float *row = &sN[k][RG * g + r][lx + HR];
            float s = t.g[0] * row[0];
#pragma unroll
            for (int j = 1; j <= HR; ++j) s = fmaf(t.g[j], row[-j] + row[j], s);
            sT[r] = s;
        }
#pragma unroll
        for (int r = 0; r < RG; ++r) {
            float s = t.g[0] * sT[r + HR];
#pragma unroll
            for (int j = 1; j <= HR; ++j) s = fmaf(t.g[j], sT[r + HR - j] + sT[r + HR + j], s);
            h[k][r] = s;
        }
    }
    const int gx = x0 + lx;
#pragma unroll
    for (int r = 0; r < RG; ++r) {
        const int gy = y0 + RG * g + r;
        if (gx >= W || gy >= H) continue;
        const size_t o = (size_t)gy * W + gx;
        if (Hr) {
            Hr[o] = h[0][r];
            Hr[plane + o] = h[1][r];
            Hr[2 * plane + o] = h[2][r];
        }
        if (coef) {
            float mb, al, be;
            tensor_coeffs_mode(mode, h[0][r], h[1][r], h[2][r], inv_lam2, mb, al, be);
            coef[o] = mb;
            coef[plane + o] = al;
            coef[2 * plane + o] = be;
        }
    }
}

}  // namespace tiles
}  // namespace mf4d
