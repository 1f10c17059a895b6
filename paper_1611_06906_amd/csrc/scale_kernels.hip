// Scale sweep (Sec. 3.3 Eq. (9)) and normalised, integrated Hessian (Eq. (6)).
//
// Per scale sigma the five derivatives of u_sigma = u * G_sigma are formed by
// two separable passes with combined taps (Gaussian, its central difference
// and its second difference), which equals blurring first and differencing
// afterwards under the half-sample symmetric extension. The vertical pass
// also evaluates, per pixel, the ingredients of the vesselness that do not
// depend on the image-wide c (S and the blob factor), the normalised Hessian
// N, and a block maximum of S that is folded into one device-wide maximum.
// A second kernel takes the per-pixel argmax once c is known, gathers N at
// the chosen scale and integrates it with G_rho.
#include "mf4d_internal.h"

namespace mf4d {

namespace {

constexpr int kHBlock = 256;   // outputs per horizontal block (one row)

__device__ __forceinline__ int reflect(int i, int n)
{
    // half-sample symmetric extension, periodic with period 2n
    const int p = 2 * n;
    i %= p;
    if (i < 0) i += p;
    return i < n ? i : p - 1 - i;
}

__global__ __launch_bounds__(kHBlock) void hpass_kernel(const float *__restrict__ u,
                                                        float *__restrict__ A,
                                                        float *__restrict__ B,
                                                        float *__restrict__ C, int H, int W,
                                                        Taps t)
{
    __shared__ float row[kHBlock + 2 * (kMaxR + 1)];
    const int y = blockIdx.y;
    const int x0 = blockIdx.x * kHBlock;
    const int R = t.r + 1;
    const float *urow = u + (size_t)y * W;
    const bool interior = (x0 - R >= 0) && (x0 + kHBlock + R <= W);
    for (int i = threadIdx.x; i < kHBlock + 2 * R; i += kHBlock) {
        const int gx = x0 - R + i;
        row[i] = urow[interior ? gx : reflect(gx, W)];
    }
    __syncthreads();
    const int x = x0 + threadIdx.x;
    if (x >= W) return;
    const float *p = row + R + threadIdx.x;
    const float c = p[0];
    float a = t.g[0] * c, b = 0.f, d = 0.f;
    for (int i = 1; i <= t.r; ++i) {
        const float l = p[-i], r = p[i];
        a += t.g[i] * (l + r);
        b += t.d1[i] * (r - l);
        d += t.d2[i] * ((l - c) + (r - c));
    }
    {
        const float l = p[-R], r = p[R];
        b += t.d1[R] * (r - l);
        d += t.d2[R] * ((l - c) + (r - c));
    }
    const size_t o = (size_t)y * W + x;
    A[o] = a;
    B[o] = b;
    C[o] = d;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
    return v;
}

template <int MODE>
__global__ __launch_bounds__(256) void vpass_kernel(const float *__restrict__ A,
                                                    const float *__restrict__ B,
                                                    const float *__restrict__ C, int H, int W,
                                                    Taps t, float sigma2, float inv2beta2,
                                                    float *__restrict__ So,
                                                    float *__restrict__ Ao,
                                                    float *__restrict__ No,
                                                    unsigned *__restrict__ smax_bits)
{
    __shared__ float red[4];
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int x = blockIdx.x * 64 + lane;
    const int y = blockIdx.y * 4 + wv;   // one row per wave: reflection branch is uniform
    float Sv = 0.f;
    if (x < W && y < H) {
        const int R = t.r + 1;
        const size_t o = (size_t)y * W + x;
        const float a0 = A[o], b0 = B[o], c0 = C[o];
        float ux = t.g[0] * b0, uxx = t.g[0] * c0, uy = 0.f, uyy = 0.f, uxy = 0.f;
        const bool interior = (y - R >= 0) && (y + R < H);
        for (int i = 1; i <= t.r; ++i) {
            const int ym = interior ? y - i : reflect(y - i, H);
            const int yp = interior ? y + i : reflect(y + i, H);
            const size_t om = (size_t)ym * W + x, op = (size_t)yp * W + x;
            const float am = A[om], ap = A[op], bm = B[om], bp = B[op], cm = C[om], cp = C[op];
            ux += t.g[i] * (bm + bp);
            uxx += t.g[i] * (cm + cp);
            uy += t.d1[i] * (ap - am);
            uxy += t.d1[i] * (bp - bm);
            uyy += t.d2[i] * ((am - a0) + (ap - a0));
        }
        {
            const int ym = interior ? y - R : reflect(y - R, H);
            const int yp = interior ? y + R : reflect(y + R, H);
            const size_t om = (size_t)ym * W + x, op = (size_t)yp * W + x;
            const float am = A[om], ap = A[op], bm = B[om], bp = B[op];
            uy += t.d1[R] * (ap - am);
            uxy += t.d1[R] * (bp - bm);
            uyy += t.d2[R] * ((am - a0) + (ap - a0));
        }
        // scale-normalised Hessian sigma^2 H; eigenvalues m +- r
        const float hxx = sigma2 * uxx, hxy = sigma2 * uxy, hyy = sigma2 * uyy;
        const float m = 0.5f * (hxx + hyy);
        const float hd = 0.5f * (hxx - hyy);
        const float r = sqrtf(hd * hd + hxy * hxy);
        Sv = sqrtf(hxx * hxx + hyy * hyy + 2.f * hxy * hxy);   // sqrt(nu~1^2 + nu~2^2)
        // |nu~2| = |m| + r carries the sign of m (ties m == 0 pass the test)
        const float am_ = fabsf(m);
        const float big = am_ + r;
        bool pass = big > 0.f;
        if (MODE == MF4D_RIDGE) pass = pass && !(m > 0.f);
        if (MODE == MF4D_VALLEY) pass = pass && !(m < 0.f);
        float blob = 0.f;
        if (pass) {
            const float rb = (am_ - r) / big;   // |R_B| = |nu~1| / |nu~2|
            blob = expf(-(rb * rb) * inv2beta2);
        }
        So[o] = Sv;
        Ao[o] = blob;
        if (No) {
            const float f = 1.f / sqrtf(1.f + sqrtf(ux * ux + uy * uy));
            const size_t plane = (size_t)H * W;
            No[o] = uxx * f;
            No[plane + o] = uxy * f;
            No[2 * plane + o] = uyy * f;
        }
    }
    float mx = wave_max(Sv);
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
constexpr int kSTW = 64, kSTH = 16;             // output tile
constexpr int kSPW = kSTW + 2 * kMaxRhoR;       // padded tile
constexpr int kSPH = kSTH + 2 * kMaxRhoR;

__device__ __forceinline__ float frangi_v(float S, float blob, float inv2c2)
{
    // V = blob * (1 - exp(-S^2 / (2 c^2)))
    return blob * -expm1f(-(S * S) * inv2c2);
}

__global__ __launch_bounds__(256) void select_kernel(SelectArgs a, int H, int W, int tiles_x)
{
    __shared__ float sN[3][kSPH][kSPW + 1];
    __shared__ float sT[3][kSPH][kSTW + 1];
    const int tx = blockIdx.x % tiles_x, ty = blockIdx.x / tiles_x;
    const int x0 = tx * kSTW, y0 = ty * kSTH;
    const int hr = a.rho.r;
    const int PW = kSTW + 2 * hr, PH = kSTH + 2 * hr;
    const size_t plane = (size_t)H * W;

    float c;
    if (a.c_param > 0.f) c = a.c_param;
    else c = 0.5f * __uint_as_float(*a.smax_bits);
    const float inv2c2 = c > 0.f ? 1.f / (2.f * c * c) : 0.f;
    const bool need_n = a.hrho != nullptr;

    if (blockIdx.x == 0 && threadIdx.x == 0 && a.c_out) *a.c_out = c;

    // argmax (or given index) at every position of the padded tile
    for (int i = threadIdx.x; i < PW * PH; i += blockDim.x) {
        const int ly = i / PW, lx = i % PW;
        const int gy = reflect(y0 - hr + ly, H), gx = reflect(x0 - hr + lx, W);
        const size_t o = (size_t)gy * W + gx;
        const bool inside_tile = lx >= hr && lx < hr + kSTW && ly >= hr && ly < hr + kSTH &&
                                 (x0 - hr + lx) < W && (y0 - hr + ly) < H;
        int best = 0;
        if (a.idx_in) {
            best = a.idx_in[o];
            if (best >= a.ns) best = a.ns - 1;   // out-of-range caller indices are clamped
        } else {
            float bv = c > 0.f ? frangi_v(a.S[o], a.A[o], inv2c2) : 0.f;
            for (int s = 1; s < a.ns; ++s) {
                const float v = c > 0.f ? frangi_v(a.S[s * plane + o], a.A[s * plane + o], inv2c2) : 0.f;
                if (v > bv) { bv = v; best = s; }
            }
            if (inside_tile) {
                if (a.idx_out) a.idx_out[o] = (uint8_t)best;
                if (a.vmax_out) a.vmax_out[o] = bv;
            }
        }
        if (need_n) {
            const float *Nb = a.N + (size_t)best * 3 * plane;
            sN[0][ly][lx] = Nb[o];
            sN[1][ly][lx] = Nb[plane + o];
            sN[2][ly][lx] = Nb[2 * plane + o];
        }
    }
    if (!need_n) return;
    __syncthreads();
    // horizontal G_rho over PH rows x TW columns
    for (int i = threadIdx.x; i < PH * kSTW; i += blockDim.x) {
        const int ly = i / kSTW, lx = i % kSTW;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float s = a.rho.g[0] * sN[k][ly][lx + hr];
            for (int j = 1; j <= hr; ++j) s += a.rho.g[j] * (sN[k][ly][lx + hr - j] + sN[k][ly][lx + hr + j]);
            sT[k][ly][lx] = s;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSTH * kSTW; i += blockDim.x) {
        const int ly = i / kSTW, lx = i % kSTW;
        const int gx = x0 + lx, gy = y0 + ly;
        if (gx >= W || gy >= H) continue;
        float h[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            float s = a.rho.g[0] * sT[k][ly + hr][lx];
            for (int j = 1; j <= hr; ++j) s += a.rho.g[j] * (sT[k][ly + hr - j][lx] + sT[k][ly + hr + j][lx]);
            h[k] = s;
        }
        const size_t o = (size_t)gy * W + gx;
        a.hrho[o] = h[0];
        a.hrho[plane + o] = h[1];
        a.hrho[2 * plane + o] = h[2];
    }
}

}  // namespace

hipError_t launch_hpass(const float *u, float *A, float *B, float *C, int H, int W,
                        const Taps &t, hipStream_t s)
{
    dim3 grid((W + kHBlock - 1) / kHBlock, H);
    hipLaunchKernelGGL(hpass_kernel, grid, dim3(kHBlock), 0, s, u, A, B, C, H, W, t);
    return hipGetLastError();
}

hipError_t launch_vpass(const float *A, const float *B, const float *C, int H, int W,
                        const Taps &t, float sigma, int mode, float beta, ScalePlanes out,
                        unsigned *smax_bits, hipStream_t s)
{
    dim3 grid((W + 63) / 64, (H + 3) / 4);
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
    const int tiles_x = (W + kSTW - 1) / kSTW, tiles_y = (H + kSTH - 1) / kSTH;
    hipLaunchKernelGGL(select_kernel, dim3(tiles_x * tiles_y), dim3(256), 0, s, a, H, W, tiles_x);
    return hipGetLastError();
}

}  // namespace mf4d
