// Single-image kernels of the scale sweep and of the normalised, integrated
// Hessian; the tile-level code lives in scale_tiles.h.
#include <algorithm>
#include <cstdlib>
#include <cstring>

#include "scale_mfma.h"

namespace mf4d {

namespace {

using namespace tiles;

__global__ __launch_bounds__(256) void hpass_kernel(const float *__restrict__ u, float *__restrict__ A,
                                                    float *__restrict__ B, float *__restrict__ C, int H, int W,
                                                    WinTaps t)
{
    extern __shared__ float tile[];
    hpass_tile(u, A, B, C, H, W, t, blockIdx.x * 64, blockIdx.y * 64, tile);
}

template <int MODE>
__global__ __launch_bounds__(256) void vpass_kernel(const float *__restrict__ A, const float *__restrict__ B,
                                                    const float *__restrict__ C, int H, int W, WinTaps t,
                                                    float sigma2, float inv2beta2, float *__restrict__ SA,
                                                    float *__restrict__ No,
                                                    unsigned *__restrict__ smax_bits)
{
    const float v = vpass_tile<MODE>(A, B, C, H, W, t, sigma2, inv2beta2, SA, No, blockIdx.x * 64,
                                     blockIdx.y * 64);
    block_max_to(v, smax_bits);
}

// Matrix-core passes; blocks are remapped so that each XCD takes a
// contiguous run of neighbouring tiles (their halos share its L2).
template <int NC>
__global__ __launch_bounds__(256) void hpass_mfma_kernel(const float *__restrict__ u, float *__restrict__ A,
                                                         float *__restrict__ B, float *__restrict__ C, int H, int W,
                                                         WinTaps t, int tiles_x, int ntiles, int per_xcd)
{
    extern __shared__ f4 lds4[];
    const int b = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (b >= ntiles) return;
    hpass_mfma_tile<NC>(u, A, B, C, H, W, t, (b % tiles_x) * kHMW, (b / tiles_x) * kHMH, (float *)lds4);
}

template <int NC>
__global__ __launch_bounds__(256) void vpass_mfma_kernel(const float *__restrict__ A, const float *__restrict__ B,
                                                         const float *__restrict__ C, int H, int W, WinTaps t,
                                                         float sigma2, float inv2beta2, int mode,
                                                         float *__restrict__ SA, float *__restrict__ No,
                                                         unsigned *__restrict__ smax_bits,
                                                         int segs, int seg_rows, int nblk, int per_xcd)
{
    extern __shared__ f4 lds4[];
    const int b = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (b >= nblk) return;
    const int strip = b / segs, seg = b - strip * segs;
    const int ys = seg * seg_rows, ye = min(H, ys + seg_rows);
    const float v = vpass_mfma_tile<NC>(A, B, C, H, W, t, sigma2, inv2beta2, mode, SA, No, strip * kVMW, ys, ye,
                                        (float *)lds4);
    block_max_to(v, smax_bits);
}

template <int NC, int LV = fused_level_default(NC)>
__global__ __launch_bounds__(256, 2) void sweep_fused_kernel(const float *__restrict__ u, int H, int W, WinTaps t,
                                                          float sigma2, float inv2beta2, int mode,
                                                          float *__restrict__ SA, float *__restrict__ No,
                                                          unsigned *__restrict__ smax_bits,
                                                          int segs, int seg_rows, int nblk, int per_xcd,
                                                          ScaleNeed need)
{
    extern __shared__ f4 lds4[];
    const int b = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (b >= nblk) return;
    const int strip = b / segs, seg = b - strip * segs;
    const int ys = seg * seg_rows, ye = min(H, ys + seg_rows);
    if (need.bits) {
        // a workgroup none of whose 32 x 32 blocks needs this scale has nothing
        // to compute (the same decision for every thread)
        bool any = false;
        for (int by = ys / kVMStep; by * kVMStep < ye; ++by)
            any = any || ((need.bits[by * need.bx + strip] >> need.scale) & 1);
        if (!any) return;
    }
    const float v = sweep_fused_tile<NC, LV>(u, H, W, t, sigma2, inv2beta2, mode, SA, No, strip * kVMW, ys, ye,
                                             (float *)lds4);
    block_max_to(v, smax_bits);
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
        float bv;
        best = argmax_px(a.SA, a.ns, plane, o, c, &bv);
        if (a.idx_out) a.idx_out[o] = (uint8_t)best;
        if (a.vmax_out) a.vmax_out[o] = bv;
    }
    (void)best;
}

template <int HR>
__global__ __launch_bounds__(256) void rho_blur_kernel(const float *__restrict__ N, const uint8_t *__restrict__ idx,
                                                       int ns, float *__restrict__ Hr, float *__restrict__ coef,
                                                       int mode, float inv_lam2, int H, int W, RhoTaps t, int tiles_x,
                                                       unsigned *smax_reset)
{
    // the image-wide max of S starts the next cycle at 0 (the argmax before
    // this kernel on the stream has read it)
    if (smax_reset && blockIdx.x == 0 && threadIdx.x == 0) *smax_reset = 0u;
    rho_blur_tile<HR>(N, idx, ns, Hr, coef, mode, inv_lam2, H, W, t, (blockIdx.x % tiles_x) * kBTW,
                      (blockIdx.x / tiles_x) * kBTH);
}

}  // namespace

int sweep_chunks(const WinTaps &t)
{
    const int nc = mfma_chunks_for(t.R);
    if (nc > kMfmaMaxChunks) return 0;
    const char *e = std::getenv("MF4D_SWEEP");
    if (e && std::strcmp(e, "valu") == 0) return 0;
    return nc;
}

int sweep_engine(const WinTaps &t)
{
    const int nc = sweep_chunks(t);
    if (!nc) return kSweepValu;
    const char *e = std::getenv("MF4D_SWEEP");
    if (e && std::strcmp(e, "split") == 0) return kSweepSplit;
    return nc <= kFusedMaxChunks ? kSweepFused : kSweepSplit;
}

// Split level of the fused kernel (which ring planes are split once per row):
// the default per chunk count, and level 2 at 8 chunks when the scales run
// concurrently, where that kernel takes one workgroup per CU anyway (below).
static int fused_level(int nc, bool shared) { return (nc == 8 && shared) ? 2 : fused_level_default(nc); }

int fused_seg_rows(int H, int W, int nc, bool shared)
{
    if (const char *e = std::getenv("MF4D_VSEG_ROWS")) {   // any multiple of the step gives the same values
        const int r = std::atoi(e);
        if (r > 0) return kVMStep * ((r + kVMStep - 1) / kVMStep);
    }
    // one round of workgroups at the kernel's occupancy (workgroups per CU
    // by its registers and LDS); longer strips amortise each one's first
    // window. When the scales of a cycle run concurrently, the kernels bound
    // by the matrix cores (6 chunks or more) take one workgroup per CU, which
    // leaves registers and LDS on every CU to the memory-bound small scales.
    int per_cu = (shared && nc >= 6) ? 1 : nc <= 3 ? 4 : (nc == 4 ? 3 : 2);
    per_cu = std::max(1, std::min(per_cu, (int)(kLdsPerCu / fused_lds(nc, fused_level(nc, shared)))));   // what the LDS holds
    const int strips = (W + kVMW - 1) / kVMW, steps = (H + kVMStep - 1) / kVMStep;
    const int segs = std::max(1, std::min(steps, (256 * per_cu + strips - 1) / strips));
    return kVMStep * ((steps + segs - 1) / segs);
}

hipError_t launch_sweep_scale(const float *u, float *hA, float *hB, float *hC, int H, int W, const WinTaps &t,
                              float sigma, int mode, float beta, ScalePlanes out, unsigned *smax_bits, bool shared,
                              hipStream_t s, ScaleNeed need)
{
    if (sweep_engine(t) != kSweepFused) {
        hipError_t e = launch_hpass(u, hA, hB, hC, H, W, t, s);
        if (e != hipSuccess) return e;
        return launch_vpass(hA, hB, hC, H, W, t, sigma, mode, beta, out, smax_bits, s);
    }
    const float sigma2 = sigma * sigma;
    const float inv2beta2 = 1.f / (2.f * beta * beta);
    const int seg_rows = fused_seg_rows(H, W, sweep_chunks(t), shared);
    const int segs = (H + seg_rows - 1) / seg_rows;
    const int nblk = segs * ((W + kVMW - 1) / kVMW);
    const int per = (nblk + 7) / 8;
    switch (sweep_chunks(t)) {
#define MF4D_FU(NC, LV)                                                                                       \
        hipLaunchKernelGGL((sweep_fused_kernel<NC, LV>), dim3(8 * per), dim3(256), fused_lds(NC, LV), s, u, H, W, t, \
                           sigma2, inv2beta2, mode, out.SA, out.N, smax_bits, segs, seg_rows, nblk, per, need); \
        break;
    case 2: MF4D_FU(2, fused_level_default(2))
    case 3: MF4D_FU(3, 0)
    case 4: MF4D_FU(4, fused_level_default(4))
    case 5: MF4D_FU(5, 0)
    case 6: MF4D_FU(6, fused_level_default(6))
    case 7: MF4D_FU(7, 0)
    case 8:
        if (fused_level(8, shared) == 2) {
            MF4D_FU(8, 2)
        } else {
            MF4D_FU(8, fused_level_default(8))
        }
#undef MF4D_FU
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int vpass_seg_rows(int H, int W)
{
    if (const char *e = std::getenv("MF4D_VSEG_ROWS")) {   // any multiple of the step gives the same values
        const int r = std::atoi(e);
        if (r > 0) return kVMStep * ((r + kVMStep - 1) / kVMStep);
    }
    const int strips = (W + kVMW - 1) / kVMW, steps = (H + kVMStep - 1) / kVMStep;
    const int segs = std::max(1, std::min(steps, (1024 + strips - 1) / strips));
    return kVMStep * ((steps + segs - 1) / segs);
}

hipError_t launch_hpass(const float *u, float *A, float *B, float *C, int H, int W,
                        const WinTaps &t, hipStream_t s)
{
    if (const int nc = sweep_chunks(t)) {
        const int tiles_x = (W + kHMW - 1) / kHMW;
        const int ntiles = tiles_x * ((H + kHMH - 1) / kHMH);
        const int per = (ntiles + 7) / 8;
        switch (nc) {
#define MF4D_HM(NC)                                                                                           \
    case NC:                                                                                                  \
        hipLaunchKernelGGL(hpass_mfma_kernel<NC>, dim3(8 * per), dim3(256), hpass_mfma_lds(NC), s, u, A, B, C, H, \
                           W, t, tiles_x, ntiles, per);                                                      \
        break;
            MF4D_HM(2) MF4D_HM(3) MF4D_HM(4) MF4D_HM(5) MF4D_HM(6) MF4D_HM(7) MF4D_HM(8) MF4D_HM(9)
#undef MF4D_HM
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    dim3 grid((W + 63) / 64, (H + 63) / 64);
    const size_t lds = (size_t)64 * (t.ntaps + 65) * sizeof(float);
    hipLaunchKernelGGL(hpass_kernel, grid, dim3(256), lds, s, u, A, B, C, H, W, t);
    return hipGetLastError();
}

hipError_t launch_vpass(const float *A, const float *B, const float *C, int H, int W,
                        const WinTaps &t, float sigma, int mode, float beta, ScalePlanes out,
                        unsigned *smax_bits, hipStream_t s)
{
    const float sigma2 = sigma * sigma;
    const float inv2beta2 = 1.f / (2.f * beta * beta);
    if (const int nc = sweep_chunks(t)) {
        const int seg_rows = vpass_seg_rows(H, W);
        const int segs = (H + seg_rows - 1) / seg_rows;
        const int nblk = segs * ((W + kVMW - 1) / kVMW);
        const int per = (nblk + 7) / 8;
        switch (nc) {
#define MF4D_VM(NC)                                                                                            \
    case NC:                                                                                                   \
        hipLaunchKernelGGL(vpass_mfma_kernel<NC>, dim3(8 * per), dim3(256), vpass_mfma_lds(NC), s, A, B, C, H, W, \
                           t, sigma2, inv2beta2, mode, out.SA, out.N, smax_bits, segs, seg_rows, nblk, per); \
        break;
            MF4D_VM(2) MF4D_VM(3) MF4D_VM(4) MF4D_VM(5) MF4D_VM(6) MF4D_VM(7) MF4D_VM(8) MF4D_VM(9)
#undef MF4D_VM
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    dim3 grid((W + 63) / 64, (H + 63) / 64);
    switch (mode) {
    case MF4D_RIDGE:
        hipLaunchKernelGGL(vpass_kernel<MF4D_RIDGE>, grid, dim3(256), 0, s, A, B, C, H, W, t, sigma2,
                           inv2beta2, out.SA, out.N, smax_bits);
        break;
    case MF4D_VALLEY:
        hipLaunchKernelGGL(vpass_kernel<MF4D_VALLEY>, grid, dim3(256), 0, s, A, B, C, H, W, t, sigma2,
                           inv2beta2, out.SA, out.N, smax_bits);
        break;
    default:
        hipLaunchKernelGGL(vpass_kernel<MF4D_BOTH>, grid, dim3(256), 0, s, A, B, C, H, W, t, sigma2,
                           inv2beta2, out.SA, out.N, smax_bits);
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

hipError_t launch_rho(const SelectArgs &a, int H, int W, hipStream_t s)
{
    const int tiles_x = (W + kBTW - 1) / kBTW, tiles_y = (H + kBTH - 1) / kBTH;
    dim3 grid(tiles_x * tiles_y), block(256);
    // N at the chosen scale is gathered through the indices
    const uint8_t *gidx = a.idx_in ? a.idx_in : a.idx_out;
    const float *src = a.N;
    if (!gidx) return hipErrorInvalidValue;
    switch (a.rho.r) {
#define MF4D_RHO_ONLY(R)                                                                                       \
    case R:                                                                                                    \
        hipLaunchKernelGGL(rho_blur_kernel<R>, grid, block, 0, s, src, gidx, a.ns, a.hrho, a.coef, a.mode,       \
                           a.inv_lam2, H, W, a.rho, tiles_x, a.smax_reset);                                    \
        break;
        MF4D_RHO_ONLY(0) MF4D_RHO_ONLY(1) MF4D_RHO_ONLY(2) MF4D_RHO_ONLY(3) MF4D_RHO_ONLY(4)
        MF4D_RHO_ONLY(5) MF4D_RHO_ONLY(6) MF4D_RHO_ONLY(7) MF4D_RHO_ONLY(8)
#undef MF4D_RHO_ONLY
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_select(const SelectArgs &a, int H, int W, hipStream_t s)
{
    const size_t plane = (size_t)H * W;
    const bool tensor = a.hrho || a.coef;
    // the argmax writes only indices; the integration gathers N through them
    if (!a.idx_in || a.c_out) {   // with given indices the kernel only reports c
        hipLaunchKernelGGL(argmax_kernel, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, s, a, plane);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (!tensor) return hipSuccess;
    if (!a.idx_in && !a.idx_out) return hipErrorInvalidValue;
    return launch_rho(a, H, W, s);
}

}  // namespace mf4d
