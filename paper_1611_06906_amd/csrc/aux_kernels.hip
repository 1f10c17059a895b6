// Kernels around the hot path: deterministic l2 reductions and their
// per-cycle bookkeeping (the stability monitor, l2-optimal stopping), the
// diffusivity of the isotropic model and the scale-image postprocessing.
#include <cmath>

#include "mf4d_internal.h"

namespace mf4d {

namespace {

// Partial sums of d^2 (d = u, or u - ref) in FP64. Thread t of block b takes
// elements b * 256 + t + k * (nb * 256); each block reduces its threads in a
// fixed tree, so the result depends on nb only, not on scheduling.
__global__ __launch_bounds__(256) void l2_partial_kernel(const float *__restrict__ u, const float *__restrict__ ref,
                                                         size_t m, double *__restrict__ partial,
                                                         unsigned *__restrict__ nonfinite)
{
    __shared__ double sh[256];
    double acc = 0.0;
    bool bad = false;
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < m; i += stride) {
        const float v = u[i];
        bad = bad || !std::isfinite(v);
        const double d = ref ? (double)v - (double)ref[i] : (double)v;
        acc = fma(d, d, acc);
    }
    if (bad && nonfinite) atomicOr(nonfinite, 1u);
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// One block: the total of the partial sums (fixed order), then the action
// for `what`: kMonitorInit / kMonitorCycle keep the squared norm and flag
// growth beyond growth_tol; kStopStep records e = sqrt(total) as step k of
// the stopping run and marks whether it improves on the best so far.
__global__ __launch_bounds__(256) void l2_final_kernel(const double *__restrict__ partial, int nb,
                                                       MonitorState *st, int what, float growth_tol, int k,
                                                       double *__restrict__ l2_out, int *__restrict__ best_out)
{
    __shared__ double sh[256];
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) acc += partial[i];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x != 0) return;
    const double total = sh[0];
    if (what == kMonitorInit) {
        st->prev = total;
    } else if (what == kMonitorCycle) {
        const double lim = st->prev * (1.0 + (double)growth_tol) * (1.0 + (double)growth_tol);
        if (total > lim) st->growth = 1u;
        st->prev = total;
    } else {
        const double e = sqrt(total);
        if (l2_out) l2_out[k] = e;
        if (k == 0 || e < st->best) {
            st->best = e;
            st->best_k = k;
            st->take = 1u;
            if (best_out) *best_out = k;
        } else {
            st->take = 0u;
        }
    }
}

__global__ void monitor_reset_kernel(MonitorState *st)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        st->prev = 0.0;
        st->best = 0.0;
        st->nonfinite = 0u;
        st->growth = 0u;
        st->take = 0u;
        st->best_k = 0;
    }
}

// Copies src to dst when the last stopping step improved on the best.
__global__ __launch_bounds__(256) void take_copy_kernel(const float *__restrict__ src, float *__restrict__ dst,
                                                        size_t m, const MonitorState *st)
{
    if (!st->take) return;
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < m; i += stride) dst[i] = src[i];
}

// Isotropic model, vertical pass: from the horizontal planes A = G u,
// B = D1G u, C = D2G u (along x), the Hessian of u_sigma
//   h_xx = G_y C, h_xy = D1G_y B, h_yy = D2G_y A
// (correlation over rows with the symmetric extension), then
// g = 1 / (1 + (h_xx^2 + 2 h_xy^2 + h_yy^2) / lambda^2). Writes the tensor
// planes (g, 0, 0) and, if hess is given, the Hessian planes.
__global__ __launch_bounds__(256) void ifod_coef_kernel(const float *__restrict__ A, const float *__restrict__ B,
                                                        const float *__restrict__ C, int H, int W, WinTaps t,
                                                        float inv_lam2, float *__restrict__ coef,
                                                        float *__restrict__ hess)
{
#pragma clang fp contract(off)   // fused multiply-adds are written out
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    const int n2 = 2 * H;
    float hxx = 0.f, hxy = 0.f, hyy = 0.f;
    for (int k = 0; k <= 2 * t.R; ++k) {
        int yy = (y + k - t.R) % n2;
        if (yy < 0) yy += n2;
        if (yy >= H) yy = n2 - 1 - yy;
        const size_t o = (size_t)yy * W + x;
        hxx = __builtin_fmaf(t.g[k], C[o], hxx);
        hxy = __builtin_fmaf(t.d1[k], B[o], hxy);
        hyy = __builtin_fmaf(t.d2[k], A[o], hyy);
    }
    const size_t p = (size_t)y * W + x;
    const size_t m = (size_t)H * W;
    const float F = __builtin_fmaf(hxx, hxx, __builtin_fmaf(2.f * hxy, hxy, hyy * hyy));
    coef[p] = 1.f / __builtin_fmaf(F, inv_lam2, 1.f);
    coef[m + p] = 0.f;
    coef[2 * m + p] = 0.f;
    if (hess) {
        hess[p] = hxx;
        hess[m + p] = hxy;
        hess[2 * m + p] = hyy;
    }
}

// Scale-image postprocessing. A pixel with vmax >= theta marches across the
// crease (the eigenvector of the stronger eigenvalue of its scale's Hessian;
// N is that Hessian times a positive factor) in unit steps t = 1..tmax on
// both sides, sampling the pixel at offset round(t e) (half away from zero)
// while the samples stay inside the image and on vessel pixels, and takes
// the scale nearest to the mean sigma of its samples (ties: smaller index).
// The sum of the float32 sigmas and the comparisons |sum - n sigma_s| are
// exact in double, so only the march itself depends on FP32 rounding.
__global__ __launch_bounds__(256) void postprocess_kernel(const uint8_t *__restrict__ idx,
                                                          const float *__restrict__ vmax,
                                                          const float *__restrict__ N, int ns, int H, int W,
                                                          ScaleTable sig, float theta, int tmax,
                                                          uint8_t *__restrict__ out)
{
    // the scale table in LDS: the march looks it up with a per-lane index,
    // which from the kernel arguments is a dependent memory load per step
    __shared__ double ssig[MF4D_MAX_SCALES];
    if (threadIdx.x < (unsigned)ns) ssig[threadIdx.x] = (double)sig.s[threadIdx.x];
    __syncthreads();
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    const size_t plane = (size_t)H * W;
    const size_t p = (size_t)y * W + x;
    int s0 = idx[p];
    if (s0 >= ns) s0 = ns - 1;
    if (!(vmax[p] >= theta)) {
        out[p] = (uint8_t)s0;
        return;
    }
    const float *n3 = N + 3 * ((size_t)s0 * plane + p);
    const float a = n3[0], b = n3[1], d = n3[2];
    // eigenvector of the larger eigenvalue (m + r), then the stronger one
    const float pm = 0.5f * (a - d);
    const float r = sqrtf(pm * pm + b * b);
    float vx, vy;
    if (pm >= 0.f) { vx = pm + r; vy = b; }
    else { vx = b; vy = r - pm; }
    const float len = sqrtf(vx * vx + vy * vy);
    float ex = 1.f, ey = 0.f;
    if (len > 0.f) { ex = vx / len; ey = vy / len; }
    const float mtr = 0.5f * (a + d);
    if (mtr < 0.f && r > 0.f) {   // |m - r| > |m + r|: the second eigenvalue is the stronger
        const float tx = ex;
        ex = -ey;
        ey = tx;
    }
    double sum = ssig[s0];
    double cnt = 1.0;
    // The march stops at the first step outside the image or off the vessel.
    // Its loads are issued kPPChunk steps at a time (positions past the image
    // or past tmax read the pixel itself and are never used), so the steps
    // of a chunk wait for memory once instead of once each; the tests and the
    // sums run in the same order as one step at a time.
    constexpr int kPPChunk = 8;
    for (int dir = -1; dir <= 1; dir += 2) {
        bool going = true;
        for (int t0 = 1; going && t0 <= tmax; t0 += kPPChunk) {
            float vq[kPPChunk];
            int sq[kPPChunk];
            bool inb[kPPChunk];
#pragma unroll
            for (int j = 0; j < kPPChunk; ++j) {
                const int t = t0 + j;
                const float ft = (float)(dir * t);
                const int xx = x + (int)roundf(ft * ex);
                const int yy = y + (int)roundf(ft * ey);
                inb[j] = t <= tmax && xx >= 0 && xx < W && yy >= 0 && yy < H;
                const size_t q = inb[j] ? (size_t)yy * W + xx : p;
                vq[j] = vmax[q];
                sq[j] = idx[q];
            }
#pragma unroll
            for (int j = 0; j < kPPChunk; ++j) {
                if (!going || !inb[j] || !(vq[j] >= theta)) {
                    going = false;
                    continue;
                }
                const int sj = sq[j] >= ns ? ns - 1 : sq[j];
                sum += ssig[sj];
                cnt += 1.0;
            }
        }
    }
    int best = 0;
    double bd = fabs(sum - cnt * (double)sig.s[0]);
    for (int s = 1; s < ns; ++s) {
        const double dd = fabs(sum - cnt * (double)sig.s[s]);
        if (dd < bd) { bd = dd; best = s; }
    }
    out[p] = (uint8_t)best;
}

int red_blocks(size_t m)
{
    size_t nb = (m + 2047) / 2048;
    if (nb < 1) nb = 1;
    if (nb > (size_t)kRedBlocks) nb = kRedBlocks;
    return (int)nb;
}

}  // namespace

hipError_t launch_monitor_reset(MonitorState *st, hipStream_t s)
{
    hipLaunchKernelGGL(monitor_reset_kernel, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_l2(const float *u, const float *ref, size_t m, double *partial, MonitorState *st, int what,
                     float growth_tol, int k, double *l2_out, int *best_out, hipStream_t s)
{
    const int nb = red_blocks(m);
    hipLaunchKernelGGL(l2_partial_kernel, dim3(nb), dim3(256), 0, s, u, ref, m, partial, &st->nonfinite);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(l2_final_kernel, dim3(1), dim3(256), 0, s, partial, nb, st, what, growth_tol, k, l2_out,
                       best_out);
    return hipGetLastError();
}

hipError_t launch_take_copy(const float *src, float *dst, size_t m, const MonitorState *st, hipStream_t s)
{
    size_t nb = (m + 1023) / 1024;
    if (nb > 4096) nb = 4096;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(take_copy_kernel, dim3((unsigned)nb), dim3(256), 0, s, src, dst, m, st);
    return hipGetLastError();
}

hipError_t launch_ifod_coef(const float *A, const float *B, const float *C, int H, int W, const WinTaps &t,
                            float inv_lam2, float *coef, float *hess, hipStream_t s)
{
    dim3 grid((W + 63) / 64, (H + 3) / 4);
    hipLaunchKernelGGL(ifod_coef_kernel, grid, dim3(256), 0, s, A, B, C, H, W, t, inv_lam2, coef, hess);
    return hipGetLastError();
}

hipError_t launch_postprocess(const uint8_t *idx, const float *vmax, const float *N, int ns, int H, int W,
                              const ScaleTable &sig, float theta, int tmax, uint8_t *out, hipStream_t s)
{
    dim3 grid((W + 63) / 64, (H + 3) / 4);
    hipLaunchKernelGGL(postprocess_kernel, grid, dim3(256), 0, s, idx, vmax, N, ns, H, W, sig, theta, tmax, out);
    return hipGetLastError();
}

}  // namespace mf4d
