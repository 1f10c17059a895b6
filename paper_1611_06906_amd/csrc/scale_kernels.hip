// Scale sweep (Sec. 3.3 Eq. (9)) and normalised, integrated Hessian (Eq. (6)).
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
// vesselness that do not depend on the image-wide c (S and the blob factor),
// the normalised Hessian N, and a block maximum of S folded into one
// device-wide maximum. Once c is known, a per-pixel kernel takes the argmax
// over scales and gathers N at the chosen scale, and a tiled kernel
// integrates it with G_rho.
#include "mf4d_internal.h"
#include "tensor_math.h"

namespace mf4d {

namespace {

constexpr int K = kWin;

// half-sample symmetric extension (period 2n), cheap for small excursions
__device__ __forceinline__ int reflect(int i, int n)
{
    while (i < 0 || i >= n) i = (i < 0) ? -i - 1 : 2 * n - 1 - i;
    return i;
}

// ------------------------------------------------------------------ horizontal
// Block: 64 rows x 64 output columns; lane = row, wave w owns columns
// 16w .. 16w+15. The rows' inputs are staged in LDS with an odd pitch.
__global__ __launch_bounds__(256) void hpass_kernel(const float *__restrict__ u,
                                                    float *__restrict__ A,
                                                    float *__restrict__ B,
                                                    float *__restrict__ C, int H, int W,
                                                    WinTaps t)
{
    extern __shared__ float tile[];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int x0 = blockIdx.x * 64, y0 = blockIdx.y * 64;
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
                ag[k] += g * v;
                ad1[k] += d1 * v;
                ad2[k] += d2 * v;
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

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

// ------------------------------------------------------------------ vertical
// Block: 64 output columns x 64 rows; lane = column, wave w owns rows
// 16w .. 16w+15, streamed from global memory through the register window.
template <int MODE>
__global__ __launch_bounds__(256) void vpass_kernel(const float *__restrict__ A,
                                                    const float *__restrict__ B,
                                                    const float *__restrict__ C, int H, int W,
                                                    WinTaps t, float sigma2, float inv2beta2,
                                                    float *__restrict__ So,
                                                    float *__restrict__ Ao,
                                                    float *__restrict__ No,
                                                    unsigned *__restrict__ smax_bits)
{
    __shared__ float red[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int x = blockIdx.x * 64 + lane;
    const int xc = min(x, W - 1);
    const int y0 = blockIdx.y * 64 + wv * K;
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
                ux[k] += g * wb[s];
                uxx[k] += g * wc[s];
                uy[k] += d1 * wa[s];
                uxy[k] += d1 * wb[s];
                uyy[k] += d2 * wa[s];
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
            // scale-normalised Hessian sigma^2 H; eigenvalues m +- r
            const float hxx = sigma2 * uxx[k], hxy = sigma2 * uxy[k], hyy = sigma2 * uyy[k];
            const float m = 0.5f * (hxx + hyy);
            const float hd = 0.5f * (hxx - hyy);
            const float r = sqrtf(hd * hd + hxy * hxy);
            const float Sv = sqrtf(hxx * hxx + hyy * hyy + 2.f * hxy * hxy);   // sqrt(nu~1^2 + nu~2^2)
            // |nu~2| = |m| + r carries the sign of m (a zero trace passes the test)
            const float am = fabsf(m);
            const float big = am + r;
            bool pass = big > 0.f;
            if (MODE == MF4D_RIDGE) pass = pass && !(m > 0.f);
            if (MODE == MF4D_VALLEY) pass = pass && !(m < 0.f);
            float blob = 0.f;
            if (pass) {
                const float rb = (am - r) / big;   // |R_B| = |nu~1| / |nu~2|
                blob = expf(-(rb * rb) * inv2beta2);
            }
            const size_t o = (size_t)y * W + x;
            So[o] = Sv;
            Ao[o] = blob;
            if (No) {
                const float gx = ux[k] + bsum, gy = uy[k];
                const float f = 1.f / sqrtf(1.f + sqrtf(gx * gx + gy * gy));
                No[o] = uxx[k] * f;
                No[plane + o] = uxy[k] * f;
                No[2 * plane + o] = uyy[k] * f;
            }
            smax = fmaxf(smax, Sv);
        }
    }
    float mx = wave_max(smax);
    if (lane == 0) red[wv] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        mx = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
        // S >= 0, so the float order equals the unsigned order of its bits
        atomicMax(smax_bits, __float_as_uint(mx));
    }
}

__global__ void fill_u32_kernel(unsigned *p, unsigned v, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void copy_f32_kernel(const float *__restrict__ s, float *__restrict__ d, size_t n)
{
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

// ---------------------------------------------------------------- select
__device__ __forceinline__ float frangi_v(float S, float blob, float inv2c2)
{
    // V = blob * (1 - exp(-S^2 / (2 c^2)))
    return blob * -expm1f(-(S * S) * inv2c2);
}

__device__ __forceinline__ float c_of(const SelectArgs &a)
{
    return a.c_param > 0.f ? a.c_param : 0.5f * __uint_as_float(*a.smax_bits);
}

// Per pixel: argmax over scales (or the given index) and N at that scale.
__global__ __launch_bounds__(256) void argmax_kernel(SelectArgs a, size_t plane)
{
    const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const float c = c_of(a);
    if (o == 0 && a.c_out) *a.c_out = c;
    if (o >= plane) return;
    int best = 0;
    if (a.idx_in) {
        best = a.idx_in[o];
        if (best >= a.ns) best = a.ns - 1;   // out-of-range caller indices are clamped
    } else {
        float bv = 0.f;
        if (c > 0.f) {
            const float inv2c2 = 1.f / (2.f * c * c);
            bv = frangi_v(a.S[o], a.A[o], inv2c2);
            for (int s = 1; s < a.ns; ++s) {
                const float v = frangi_v(a.S[s * plane + o], a.A[s * plane + o], inv2c2);
                if (v > bv) { bv = v; best = s; }
            }
        }
        if (a.idx_out) a.idx_out[o] = (uint8_t)best;
        if (a.vmax_out) a.vmax_out[o] = bv;
    }
    if (a.nsel) {
        const float *Nb = a.N + (size_t)best * 3 * plane;
        a.nsel[o] = Nb[o];
        a.nsel[plane + o] = Nb[plane + o];
        a.nsel[2 * plane + o] = Nb[2 * plane + o];
    }
}

// H_rho = G_rho * N (separable, symmetric extension), 64 x 32 output tiles;
// writes H_rho and/or the compact tensor planes of H_rho.
constexpr int kBTW = 64, kBTH = 32;

template <int HR>
__global__ __launch_bounds__(256) void rho_blur_kernel(const float *__restrict__ N, float *__restrict__ Hr,
                                                       float *__restrict__ coef, int mode, float inv_lam2,
                                                       int H, int W, RhoTaps t, int tiles_x)
{
    constexpr int PW = kBTW + 2 * HR, PH = kBTH + 2 * HR;
    __shared__ float sN[3][PH][PW + 1];
    __shared__ float sT[3][PH][kBTW + 1];
    const int x0 = (blockIdx.x % tiles_x) * kBTW, y0 = (blockIdx.x / tiles_x) * kBTH;
    const size_t plane = (size_t)H * W;
    const bool interior = x0 - HR >= 0 && y0 - HR >= 0 && x0 + kBTW + HR <= W && y0 + kBTH + HR <= H;
    for (int i = threadIdx.x; i < PW * PH; i += 256) {
        const int ly = i / PW, lx = i - ly * PW;
        const int gy = interior ? y0 - HR + ly : reflect(y0 - HR + ly, H);
        const int gx = interior ? x0 - HR + lx : reflect(x0 - HR + lx, W);
        const size_t o = (size_t)gy * W + gx;
        sN[0][ly][lx] = N[o];
        sN[1][ly][lx] = N[plane + o];
        sN[2][ly][lx] = N[2 * plane + o];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < PH * kBTW; i += 256) {
        const int ly = i >> 6, lx = i & 63;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float s = t.g[0] * sN[k][ly][lx + HR];
#pragma unroll
            for (int j = 1; j <= HR; ++j) s += t.g[j] * (sN[k][ly][lx + HR - j] + sN[k][ly][lx + HR + j]);
            sT[k][ly][lx] = s;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kBTH * kBTW; i += 256) {
        const int ly = i >> 6, lx = i & 63;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= W || gy >= H) continue;
        const size_t o = (size_t)gy * W + gx;
        float h[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float s = t.g[0] * sT[k][ly + HR][lx];
#pragma unroll
            for (int j = 1; j <= HR; ++j) s += t.g[j] * (sT[k][ly + HR - j][lx] + sT[k][ly + HR + j][lx]);
            h[k] = s;
        }
        if (Hr) {
            Hr[o] = h[0];
            Hr[plane + o] = h[1];
            Hr[2 * plane + o] = h[2];
        }
        if (coef) {
            float mb, al, be;
            tensor_coeffs_mode(mode, h[0], h[1], h[2], inv_lam2, mb, al, be);
            coef[o] = mb;
            coef[plane + o] = al;
            coef[2 * plane + o] = be;
        }
    }
}

}  // namespace

hipError_t launch_hpass(const float *u, float *A, float *B, float *C, int H, int W,
                        const WinTaps &t, hipStream_t s)
{
    dim3 grid((W + 63) / 64, (H + 63) / 64);
    const size_t lds = (size_t)64 * (t.ntaps + 65) * sizeof(float);
    hipLaunchKernelGGL(hpass_kernel, grid, dim3(256), lds, s, u, A, B, C, H, W, t);
    return hipGetLastError();
}

hipError_t launch_vpass(const float *A, const float *B, const float *C, int H, int W,
                        const WinTaps &t, float sigma, int mode, float beta, ScalePlanes out,
                        unsigned *smax_bits, hipStream_t s)
{
    dim3 grid((W + 63) / 64, (H + 63) / 64);
    const float sigma2 = sigma * sigma;
    const float inv2beta2 = 1.f / (2.f * beta * beta);
    switch (mode) {
    case MF4D_RIDGE:
        hipLaunchKernelGGL(vpass_kernel<MF4D_RIDGE>, grid, dim3(256), 0, s, A, B, C, H, W, t, sigma2,
                           inv2beta2, out.S, out.A, out.N, smax_bits);
        break;
    case MF4D_VALLEY:
        hipLaunchKernelGGL(vpass_kernel<MF4D_VALLEY>, grid, dim3(256), 0, s, A, B, C, H, W, t, sigma2,
                           inv2beta2, out.S, out.A, out.N, smax_bits);
        break;
    default:
        hipLaunchKernelGGL(vpass_kernel<MF4D_BOTH>, grid, dim3(256), 0, s, A, B, C, H, W, t, sigma2,
                           inv2beta2, out.S, out.A, out.N, smax_bits);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned *p, unsigned v, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_copy_f32(const float *src, float *dst, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(copy_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_select(const SelectArgs &a, int H, int W, hipStream_t s)
{
    const size_t plane = (size_t)H * W;
    SelectArgs b = a;
    const bool tensor = a.hrho || a.coef;
    if (!tensor) b.nsel = nullptr;
    hipLaunchKernelGGL(argmax_kernel, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, s, b, plane);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !tensor) return e;
    const int tiles_x = (W + kBTW - 1) / kBTW, tiles_y = (H + kBTH - 1) / kBTH;
    dim3 grid(tiles_x * tiles_y), block(256);
    switch (a.rho.r) {
#define MF4D_RHO_CASE(R)                                                                               \
    case R:                                                                                            \
        hipLaunchKernelGGL(rho_blur_kernel<R>, grid, block, 0, s, a.nsel, a.hrho, a.coef, a.mode,          \
                           a.inv_lam2, H, W, a.rho, tiles_x);                                          \
        break;
        MF4D_RHO_CASE(0) MF4D_RHO_CASE(1) MF4D_RHO_CASE(2) MF4D_RHO_CASE(3) MF4D_RHO_CASE(4)
        MF4D_RHO_CASE(5) MF4D_RHO_CASE(6) MF4D_RHO_CASE(7) MF4D_RHO_CASE(8)
#undef MF4D_RHO_CASE
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace mf4d
