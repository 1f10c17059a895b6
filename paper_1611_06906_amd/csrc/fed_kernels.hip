// FED substeps (Sec. 3.4, Sec. 3.5 Eq. (21)):  u <- u - tau L^T D L u.
//
// Rows of L exist only at interior pixels (natural boundary condition), so
// T = D L u is zero outside 1 <= x <= W-2, 1 <= y <= H-2 and L^T reaches the
// border pixels through the transposed stencils:
//   L_xx, L_yy: [1 -2 1] along x / y;  L_xy = L_yx: (+1 at (-1,-1), (1,1);
//   -1 at (-1,1), (1,-1)) / 4, so  r = L^T T = D2x T_xx + 2 Dxy T_xy + D2y T_yy.
//
// Two kinds of kernel:
//  * fed_hrho_kernel: one substep from H_rho, rebuilding the fourth-order
//    tensor (tensor_math.h) in registers at every position it needs.
//  * fed_stream_kernel<S> / fed_stream2_kernel<S>: S consecutive substeps
//    from the compact tensor planes (m, al, be) computed once per cycle (P is
//    frozen over the cycle, so no per-substep eigen-solves), one wave per
//    column strip streaming down its rows with the intermediate images in
//    registers (fed_tiles.h); one or two columns per lane, the same values.
#include "mf4d_internal.h"
#include "tensor_math.h"
#include <atomic>
#include <cstdlib>

#include "fed_tiles.h"

namespace mf4d {

namespace {

// XCD-aware tile order: consecutive blocks go to different XCDs, so give each
// XCD a contiguous band of tiles and keep halo re-reads in its own L2.
__device__ __forceinline__ int xcd_tile(int per_xcd)
{
    return (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
}

constexpr int kTW = 64, kTH = 16;   // output tile of the H_rho kernel

template <int MODE>
__global__ __launch_bounds__(256) void fed_hrho_kernel(const float *__restrict__ u,
                                                       float *__restrict__ uo,
                                                       const float *__restrict__ hrho,
                                                       int H, int W, float tau, float inv_lam2,
                                                       int tiles_x, int ntiles, int per_xcd)
{
    __shared__ float su[kTH + 4][kTW + 4 + 1];
    __shared__ float sT[3][kTH + 2][kTW + 2 + 1];
    const int tile = xcd_tile(per_xcd);
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
        uo[(size_t)gy * W + gx] = su[ly + 2][lx + 2] - tau * (rxx + rxy + ryy);
    }
}

template <int S>
__global__ __launch_bounds__(256) void fed_stream_kernel(const float *__restrict__ u, float *__restrict__ uo,
                                                         const float *__restrict__ coef, int H, int W,
                                                         FedTaus taus, int strips, int segs, int seg_rows,
                                                         int blocks_per_xcd, int nblocks)
{
    // XCD-aware: each XCD takes a contiguous run of blocks
    const int blk = (blockIdx.x % 8) * blocks_per_xcd + blockIdx.x / 8;
    if (blk >= nblocks) return;
    const int wave = __builtin_amdgcn_readfirstlane(blk * 4 + (threadIdx.x >> 6));   // uniform per wave
    const int strip = wave % strips, seg = wave / strips;
    if (seg >= segs) return;
    tiles::fed_stream_wave<S>(u, uo, coef, H, W, taus, strip, seg, seg_rows);
}


template <int S>
__global__ __launch_bounds__(256) void fed_stream2_kernel(const float *__restrict__ u, float *__restrict__ uo,
                                                          const float *__restrict__ coef, int H, int W,
                                                          FedTaus taus, int strips, int segs, int seg_rows,
                                                          int blocks_per_xcd, int nblocks)
{
    // XCD-aware: each XCD takes a contiguous run of blocks
    const int blk = (blockIdx.x % 8) * blocks_per_xcd + blockIdx.x / 8;
    if (blk >= nblocks) return;
    const int wave = __builtin_amdgcn_readfirstlane(blk * 4 + (threadIdx.x >> 6));   // uniform per wave
    const int strip = wave % strips, seg = wave / strips;
    if (seg >= segs) return;
    tiles::fed_stream_wave2<S>(u, uo, coef, H, W, taus, strip, seg, seg_rows);
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
        hipLaunchKernelGGL(fed_hrho_kernel<MF4D_RIDGE>, grid, block, 0, s, u_in, u_out, hrho, H, W, tau,
                           inv_lam2, tiles_x, ntiles, per);
        break;
    case MF4D_VALLEY:
        hipLaunchKernelGGL(fed_hrho_kernel<MF4D_VALLEY>, grid, block, 0, s, u_in, u_out, hrho, H, W, tau,
                           inv_lam2, tiles_x, ntiles, per);
        break;
    default:
        hipLaunchKernelGGL(fed_hrho_kernel<MF4D_BOTH>, grid, block, 0, s, u_in, u_out, hrho, H, W, tau,
                           inv_lam2, tiles_x, ntiles, per);
        break;
    }
    return hipGetLastError();
}

// Blocks of the streaming kernel (for the current form and `steps`) that
// one CU holds at once, and the device's CU count (cached per device).
int stream_blocks_per_cu(int steps, int *cus)
{
    // filled on first use; threads that race here store the same values
    static std::atomic<int> cache[16][3][5];   // [device][cols][steps]: 0 = not yet asked
    static std::atomic<int> ncu[16];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 16) dev = 0;
    if (steps < 1 || steps > 4) steps = 4;
    const int cols = stream_cols_per_lane(steps);
    int n = ncu[dev].load(std::memory_order_relaxed);
    if (!n) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
        ncu[dev].store(n, std::memory_order_relaxed);
    }
    std::atomic<int> &c = cache[dev][cols][steps];
    int nb = c.load(std::memory_order_relaxed);
    if (!nb) {
        const void *fn = nullptr;
        switch (steps) {
        case 1: fn = cols == 2 ? (const void *)fed_stream2_kernel<1> : (const void *)fed_stream_kernel<1>; break;
        case 2: fn = cols == 2 ? (const void *)fed_stream2_kernel<2> : (const void *)fed_stream_kernel<2>; break;
        case 3: fn = cols == 2 ? (const void *)fed_stream2_kernel<3> : (const void *)fed_stream_kernel<3>; break;
        default: fn = cols == 2 ? (const void *)fed_stream2_kernel<4> : (const void *)fed_stream_kernel<4>; break;
        }
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, 0) != hipSuccess || nb < 1) nb = 1;
        c.store(nb, std::memory_order_relaxed);
    }
    *cus = n;
    return nb;
}

int stream_cols_per_lane(int steps)
{
    if (const char *e = std::getenv("MF4D_STREAM_COLS")) {
        const int c = std::atoi(e);
        if (c == 1 || c == 2) return c;
    }
    // measured at 4096^2: two columns per lane win only at four substeps
    return steps >= 4 ? 2 : 1;
}

hipError_t launch_fed_stream(const float *u_in, float *u_out, const float *coef, int H, int W, int steps,
                             const float *taus, int seg_rows, hipStream_t s)
{
    FedTaus t{};
    for (int k = 0; k < steps; ++k) t.t[k] = taus[k];
    const int cols = stream_cols_per_lane(steps);
    const int outw = 64 * cols - 4 * steps;
    const int strips = (W + outw - 1) / outw;
    const int segs = (H + seg_rows - 1) / seg_rows;
    const int nblocks = (strips * segs + 3) / 4;
    const int per = (nblocks + 7) / 8;
    dim3 grid(8 * per), block(256);
#define MF4D_ST(K)                                                                                            \
    case K:                                                                                                   \
        if (cols == 2)                                                                                        \
            hipLaunchKernelGGL(fed_stream2_kernel<K>, grid, block, 0, s, u_in, u_out, coef, H, W, t, strips, segs, \
                               seg_rows, per, nblocks);                                                       \
        else                                                                                                  \
            hipLaunchKernelGGL(fed_stream_kernel<K>, grid, block, 0, s, u_in, u_out, coef, H, W, t, strips, segs,  \
                               seg_rows, per, nblocks);                                                       \
        break;
    switch (steps) {
        MF4D_ST(1) MF4D_ST(2) MF4D_ST(3) MF4D_ST(4)
    default:
        return hipErrorInvalidValue;
    }
#undef MF4D_ST
    return hipGetLastError();
}

}  // namespace mf4d
