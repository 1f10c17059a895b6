// Crease extraction from the filtered image (Sec. 3.6) and its evaluation
// against ground-truth centrelines (Sec. 4): the field d = det(g | Hg), a
// marching-squares pass that writes at most two segments per cell into fixed
// slots (no atomics on positions, so the output does not depend on
// scheduling), and a matcher per ground-truth segment.
#include <cmath>

#include "mf4d_internal.h"

namespace mf4d {

namespace {

// Vertical pass of the crease field: from A = G u, B = D1G u, C = D2G u
// (along x) the gradient and Hessian of u_sigma,
//   g_x = G_y B, g_y = D1G_y A, h_xx = G_y C, h_xy = D1G_y B, h_yy = D2G_y A,
// and d = g_x (h_xy g_x + h_yy g_y) - g_y (h_xx g_x + h_xy g_y).
// planes: [6][H][W] = g_x, g_y, h_xx, h_xy, h_yy, d.
__global__ __launch_bounds__(256) void crease_field_kernel(const float *__restrict__ A, const float *__restrict__ B,
                                                           const float *__restrict__ C, int H, int W, WinTaps t,
                                                           float *__restrict__ planes)
{
#pragma clang fp contract(off)   // fused multiply-adds are written out
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W || y >= H) return;
    const int n2 = 2 * H;
    float gx = 0.f, gy = 0.f, hxx = 0.f, hxy = 0.f, hyy = 0.f;
    for (int k = 0; k <= 2 * t.R; ++k) {
        int yy = (y + k - t.R) % n2;
        if (yy < 0) yy += n2;
        if (yy >= H) yy = n2 - 1 - yy;
        const size_t o = (size_t)yy * W + x;
        const float a = A[o], b = B[o], c = C[o];
        gx = __builtin_fmaf(t.g[k], b, gx);
        gy = __builtin_fmaf(t.d1[k], a, gy);
        hxx = __builtin_fmaf(t.g[k], c, hxx);
        hxy = __builtin_fmaf(t.d1[k], b, hxy);
        hyy = __builtin_fmaf(t.d2[k], a, hyy);
    }
    const size_t m = (size_t)H * W, p = (size_t)y * W + x;
    const float hgx = __builtin_fmaf(hxx, gx, hxy * gy);
    const float hgy = __builtin_fmaf(hxy, gx, hyy * gy);
    planes[p] = gx;
    planes[m + p] = gy;
    planes[2 * m + p] = hxx;
    planes[3 * m + p] = hxy;
    planes[4 * m + p] = hyy;
    planes[5 * m + p] = __builtin_fmaf(gx, hgy, -(gy * hgx));
}

// +1 ridge (stronger eigenvalue negative), -1 valley, 0 none.
__device__ __forceinline__ int crease_type(float a, float b, float c, float strength)
{
    const float m = 0.5f * (a + c);
    const float hd = 0.5f * (a - c);
    const float r = sqrtf(hd * hd + b * b);
    if (!(r > 0.f) || m == 0.f) return 0;
    if (fabsf(m) + r < strength) return 0;
    return m < 0.f ? 1 : -1;
}

// Does v run closer to the weaker eigenvector of (a, b, c) than to the
// stronger? q = v^T (H - m Id) v has the sign of (v.e1)^2 - (v.e2)^2.
__device__ __forceinline__ bool along_weak(float vx, float vy, float a, float b, float c)
{
    const float m = 0.5f * (a + c);
    const float q = 0.5f * (a - c) * (vx * vx - vy * vy) + 2.f * b * vx * vy;
    return m > 0.f ? q <= 0.f : q >= 0.f;
}

// Edge pairs of the segments of a cell by inside-pattern (bit k: corner k has
// d >= 0; corners (x,y), (x+1,y), (x+1,y+1), (x,y+1); edges 0 top, 1 right,
// 2 bottom, 3 left); saddles split by the sign of the mean of the corners.
__device__ __forceinline__ int cell_edges(int pat, float centre, int e[4])
{
    switch (pat) {
    case 1: case 14: e[0] = 0; e[1] = 3; return 1;
    case 2: case 13: e[0] = 0; e[1] = 1; return 1;
    case 4: case 11: e[0] = 1; e[1] = 2; return 1;
    case 8: case 7: e[0] = 2; e[1] = 3; return 1;
    case 3: case 12: e[0] = 1; e[1] = 3; return 1;
    case 6: case 9: e[0] = 0; e[1] = 2; return 1;
    case 5:
        if (centre >= 0.f) { e[0] = 0; e[1] = 1; e[2] = 2; e[3] = 3; }
        else { e[0] = 0; e[1] = 3; e[2] = 1; e[3] = 2; }
        return 2;
    case 10:
        if (centre >= 0.f) { e[0] = 0; e[1] = 3; e[2] = 1; e[3] = 2; }
        else { e[0] = 0; e[1] = 1; e[2] = 2; e[3] = 3; }
        return 2;
    default: return 0;
    }
}

// One thread per cell (x, y), 0 <= x < W - 1, 0 <= y < H - 1.
__global__ __launch_bounds__(256) void marching_kernel(const float *__restrict__ planes, int H, int W, float strength,
                                                       int mode, float *__restrict__ seg, int8_t *__restrict__ type,
                                                       unsigned *__restrict__ count)
{
    const int x = blockIdx.x * 64 + (threadIdx.x & 63);
    const int y = blockIdx.y * 4 + (threadIdx.x >> 6);
    if (x >= W - 1 || y >= H - 1) return;
    const size_t m = (size_t)H * W;
    const float *hxx = planes + 2 * m, *hxy = planes + 3 * m, *hyy = planes + 4 * m, *d = planes + 5 * m;
    const int cx[4] = {0, 1, 1, 0}, cy[4] = {0, 0, 1, 1};
    size_t pc[4];
    float dc[4];
    int pat = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        pc[k] = (size_t)(y + cy[k]) * W + (x + cx[k]);
        dc[k] = d[pc[k]];
        if (dc[k] >= 0.f) pat |= 1 << k;
    }
    const float centre = 0.25f * (dc[0] + dc[1] + dc[2] + dc[3]);
    int e[4];
    const int ns = cell_edges(pat, centre, e);
    const size_t cell = (size_t)y * (W - 1) + x;
    float out[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    int8_t ty_out[2] = {0, 0};
    int slot = 0;
    for (int q = 0; q < ns; ++q) {
        // Each end is measured from its edge's nearer corner (the fraction
        // |d_a| / (|d_a| + |d_b|) <= 1/2 needs no cancellation, so an end
        // close to either corner keeps its full relative precision), and the
        // segment's direction is the integer step between the two ends'
        // corners plus the difference of their offsets from them: exact in
        // the offsets where both ends hang off one corner (a short segment
        // cutting it off), at least ~1/2 long otherwise. Taken from the
        // image coordinates, a segment a few 1e-5 px long near x = 4000
        // would point wherever their float32 rounding puts its ends.
        float px[2], py[2], ox[2], oy[2], ha[2], hb[2], hc[2];
        int ty[2], anc[2];
        for (int j = 0; j < 2; ++j) {
            const int ed = e[2 * q + j];
            int a = ed, b = (ed + 1) & 3;
            if (fabsf(dc[b]) < fabsf(dc[a])) {
                const int t_ = a;
                a = b;
                b = t_;
            }
            const float tt = dc[a] / (dc[a] - dc[b]);
            ox[j] = tt * (float)(cx[b] - cx[a]);
            oy[j] = tt * (float)(cy[b] - cy[a]);
            anc[j] = a;
            px[j] = (float)(x + cx[a]) + ox[j];
            py[j] = (float)(y + cy[a]) + oy[j];
            const size_t pa = pc[a], pb = pc[b];
            ha[j] = hxx[pa] + tt * (hxx[pb] - hxx[pa]);
            hb[j] = hxy[pa] + tt * (hxy[pb] - hxy[pa]);
            hc[j] = hyy[pa] + tt * (hyy[pb] - hyy[pa]);
            ty[j] = crease_type(ha[j], hb[j], hc[j], strength);
        }
        if (ty[0] == 0 || ty[0] != ty[1]) continue;
        const float vx = (float)(cx[anc[1]] - cx[anc[0]]) + (ox[1] - ox[0]);
        const float vy = (float)(cy[anc[1]] - cy[anc[0]]) + (oy[1] - oy[0]);
        if (!along_weak(vx, vy, 0.5f * (ha[0] + ha[1]), 0.5f * (hb[0] + hb[1]), 0.5f * (hc[0] + hc[1])))
            continue;
        if ((mode == MF4D_RIDGE && ty[0] != 1) || (mode == MF4D_VALLEY && ty[0] != -1)) continue;
        out[4 * slot + 0] = px[0];
        out[4 * slot + 1] = py[0];
        out[4 * slot + 2] = px[1];
        out[4 * slot + 3] = py[1];
        ty_out[slot] = (int8_t)ty[0];
        ++slot;
    }
    float4 *s4 = (float4 *)(seg + 8 * cell);
    s4[0] = make_float4(out[0], out[1], out[2], out[3]);
    s4[1] = make_float4(out[4], out[5], out[6], out[7]);
    type[2 * cell] = ty_out[0];
    type[2 * cell + 1] = ty_out[1];
    if (count && slot) atomicAdd(count, (unsigned)slot);
}

__device__ __forceinline__ float point_segment(float px, float py, float ax, float ay, float bx, float by)
{
    const float vx = bx - ax, vy = by - ay;
    const float l2 = vx * vx + vy * vy;
    float t = 0.f;
    if (l2 > 0.f) t = fminf(1.f, fmaxf(0.f, ((px - ax) * vx + (py - ay) * vy) / l2));
    const float dx = px - (ax + t * vx), dy = py - (ay + t * vy);
    return sqrtf(dx * dx + dy * dy);
}

// One thread per ground-truth segment: the reconstructed segment of its type
// with the least directed Hausdorff distance from it (at most radius; ties:
// the first cell in row-major order, then slot 0), over the cells that can
// hold one (the segment's bounding box grown by radius).
__global__ __launch_bounds__(256) void crease_match_kernel(const float *__restrict__ seg,
                                                           const int8_t *__restrict__ type, int H, int W,
                                                           const float *__restrict__ gt,
                                                           const int *__restrict__ gt_type, int n, float radius,
                                                           float *__restrict__ dist, int *__restrict__ match)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float g0x = gt[4 * i], g0y = gt[4 * i + 1], g1x = gt[4 * i + 2], g1y = gt[4 * i + 3];
    const int gtt = gt_type[i];
    int x0 = (int)floorf(fminf(g0x, g1x) - radius) - 1, x1 = (int)ceilf(fmaxf(g0x, g1x) + radius) + 1;
    int y0 = (int)floorf(fminf(g0y, g1y) - radius) - 1, y1 = (int)ceilf(fmaxf(g0y, g1y) + radius) + 1;
    x0 = max(x0, 0);
    y0 = max(y0, 0);
    x1 = min(x1, W - 2);
    y1 = min(y1, H - 2);
    // Distances are taken in coordinates relative to the segment's first end:
    // every point compared lies within a few pixels of it, so the offsets are
    // exact float32 differences (of values within a factor of two of each
    // other, or small) and the distances keep float32's relative precision,
    // instead of an absolute error of the coordinates' ulp (2.4e-4 near 4096).
    const float l1x = g1x - g0x, l1y = g1y - g0y;
    float best = INFINITY;
    int bm = -1;
    for (int y = y0; y <= y1; ++y)
        for (int x = x0; x <= x1; ++x)
            for (int sl = 0; sl < 2; ++sl) {
                const size_t c = (size_t)y * (W - 1) + x;
                if (type[2 * c + sl] != gtt) continue;
                const float *R = seg + 8 * c + 4 * sl;
                const float ax = R[0] - g0x, ay = R[1] - g0y, bx = R[2] - g0x, by = R[3] - g0y;
                const float h = fmaxf(point_segment(0.f, 0.f, ax, ay, bx, by), point_segment(l1x, l1y, ax, ay, bx, by));
                if (h <= radius && h < best) {
                    best = h;
                    bm = (int)(2 * c + sl);
                }
            }
    match[i] = bm;
    if (bm < 0) {
        dist[i] = -1.f;
        return;
    }
    const float *R = seg + 4 * (size_t)bm;
    dist[i] = point_segment(0.5f * l1x, 0.5f * l1y, R[0] - g0x, R[1] - g0y, R[2] - g0x, R[3] - g0y);
}

}  // namespace

hipError_t launch_crease_field(const float *A, const float *B, const float *C, int H, int W, const WinTaps &t,
                               float *planes, hipStream_t s)
{
    dim3 grid((W + 63) / 64, (H + 3) / 4);
    hipLaunchKernelGGL(crease_field_kernel, grid, dim3(256), 0, s, A, B, C, H, W, t, planes);
    return hipGetLastError();
}

hipError_t launch_marching(const float *planes, int H, int W, float strength, int mode, float *seg, int8_t *type,
                           unsigned *count, hipStream_t s)
{
    dim3 grid((W - 1 + 63) / 64, (H - 1 + 3) / 4);
    hipLaunchKernelGGL(marching_kernel, grid, dim3(256), 0, s, planes, H, W, strength, mode, seg, type, count);
    return hipGetLastError();
}

hipError_t launch_crease_match(const float *seg, const int8_t *type, int H, int W, const float *gt, const int *gt_type,
                               int n, float radius, float *dist, int *match, hipStream_t s)
{
    hipLaunchKernelGGL(crease_match_kernel, dim3((n + 255) / 256), dim3(256), 0, s, seg, type, H, W, gt, gt_type, n,
                       radius, dist, match);
    return hipGetLastError();
}

}  // namespace mf4d
