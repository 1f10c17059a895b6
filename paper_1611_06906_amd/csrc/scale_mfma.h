// Matrix-core forms of the two separable passes of the scale sweep
// (Sec. 3.3, derivatives of u_sigma for Eq. (9) and Eq. (6)), shared by the
// single-image and the batched kernels: FP32 MFMA products, and in the fused
// kernel at even chunk counts split-BF16 products (see "split BF16" below).
//
// A 1-D correlation of 16 consecutive outputs with a (2R+1)-tap filter is the
// product of a 16 x K banded Toeplitz matrix T[m][k] = tap[k - m] with the K
// inputs starting R before the first output (K >= 16 + 2R, a multiple of 16).
// One v_mfma_f32_16x16x4f32 multiplies a 16 x 4 slice of T by a 4 x 16 block
// of inputs, so 16 columns (or rows) are filtered at once and K / 4 products
// finish 256 outputs of one filter. Each lane keeps its Toeplitz entries for
// all three filters (Gaussian, central difference, second difference) in
// registers. The order of the K terms is free, so lane group q supplies the
// four consecutive inputs 4q .. 4q+3 of each 16-input chunk over the four
// products of the chunk, which one 16-byte LDS read delivers. The last chunk
// is taken in contiguous 4-input slices instead (lane group q supplies input
// 4j + q of slice j): inputs from 16 + 2R on meet zero taps in every row, so
// the slices made only of them are skipped (last_slices).
//
// Inputs are shifted by the value at the block's first output before the
// products (as in the register-window passes), so locally constant lines
// give exactly zero derivatives; the Gaussian output adds the shift back.
// The values of a 16 x 16 block depend only on its position, not on how
// blocks are grouped into workgroups.
#pragma once

#include "scale_tiles.h"

namespace mf4d {
namespace tiles {

typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int kMfmaMaxChunks = 9;      // K <= 144: radius R <= 64
constexpr int kFusedMaxChunks = 8;     // LDS of two fused workgroups per CU
constexpr int kHMW = 256, kHMH = 16;   // horizontal tile: output columns x rows (4 waves x 4 blocks)
constexpr int kVMW = 32, kVMStep = 32; // vertical strip width and rows per step (4 waves x one block)
constexpr size_t kLdsPerCu = 160 * 1024; // LDS per compute unit (gfx950)

__host__ __device__ constexpr int mfma_chunks_for(int R) { return (16 + 2 * R + 15) / 16; }

__host__ __device__ constexpr size_t hpass_mfma_lds(int nc) { return sizeof(float) * kHMH * (kHMW - 16 + 16 * nc + 4); }
__host__ __device__ constexpr size_t vpass_mfma_lds(int nc) { return sizeof(float) * 3 * kVMW * (16 * nc + 48 + 4); }

// Half-sample symmetric extension in closed form (the same index as
// reflect() for any i): i mod 2n, mirrored in the upper half.
__device__ __forceinline__ int reflect_any(int i, int n)
{
    const int p = 2 * n;
    int j = i % p;
    j = j < 0 ? j + p : j;
    return j < n ? j : p - 1 - j;
}

__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// This lane's entries of the Toeplitz slices: a[c][j] = tap[k - m] for row
// m = lane % 16 and input k = 16c + 4(lane / 16) + j (zero outside 0..2R);
// in the last chunk k = 16c + 4j + lane / 16.
template <int NC>
__device__ __forceinline__ void toeplitz_lane(const float *tap, int R, float (&a)[NC][4])
{
    const int lane = threadIdx.x & 63, m = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int t = (c < NC - 1 ? 16 * c + 4 * kq + j : 16 * c + 4 * j + kq) - m;
            a[c][j] = (t >= 0 && t <= 2 * R) ? tap[t] : 0.f;
        }
}

// Slices of the last chunk that hold inputs inside the band (0..4): the
// chunk's inputs 16 + 2R - 16 (NC - 1) on have zero taps for every row.
template <int NC>
__host__ __device__ __forceinline__ int last_slices(int R)
{
    const int z = 16 + 2 * R - 16 * (NC - 1);
    return z <= 0 ? 0 : (z >= 16 ? 4 : (z + 3) / 4);
}

// ------------------------------------------------------------------ split BF16
// Products of FP32 values on the BF16 matrix cores: each value x is split by
// truncation into three BF16 parts, x = hi + mid + lo exactly (8 significant
// bits each), and a product a b is taken as the six part products above
// 2^-24 |a b| (hi hi, hi mid, mid hi, hi lo, lo hi, mid mid), accumulated in
// FP32 by v_mfma_f32_16x16x32_bf16 in that fixed order.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
union BF8 {
    uint32_t u[4];
    bf8 v;
};

__device__ __forceinline__ float bf_trunc(float x) { return __uint_as_float(__float_as_uint(x) & 0xffff0000u); }
__device__ __forceinline__ uint32_t bf_pack(float a, float b)   // a, b exact in BF16: a low half, b high half
{
    return (__float_as_uint(a) >> 16) | (__float_as_uint(b) & 0xffff0000u);
}

__device__ __forceinline__ void split3(const float (&x)[8], BF8 &h, BF8 &m, BF8 &l)
{
#pragma clang fp contract(off)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float x0 = x[2 * q], x1 = x[2 * q + 1];
        const float h0 = bf_trunc(x0), h1 = bf_trunc(x1);
        const float r0 = x0 - h0, r1 = x1 - h1;
        const float m0 = bf_trunc(r0), m1 = bf_trunc(r1);
        h.u[q] = bf_pack(h0, h1);
        m.u[q] = bf_pack(m0, m1);
        l.u[q] = bf_pack(r0 - m0, r1 - m1);
    }
}

struct BF3 {
    BF8 h, m, l;
};

__device__ __forceinline__ f4 mfma_bf3(const BF3 &a, const BF3 &b, f4 c)
{
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h.v, b.h.v, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h.v, b.m.v, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.m.v, b.h.v, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h.v, b.l.v, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.l.v, b.h.v, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.m.v, b.m.v, c, 0, 0, 0);
    return c;
}

// This lane's Toeplitz entries of 32-input slice sl, split: tap[k - m] for
// row m = lane % 16 and input k = 32 sl + 8 (lane / 16) + j, j = 0..7.
template <int NSL>
__device__ __forceinline__ void toeplitz_bf3(const float *tap, int R, BF3 (&a)[NSL])
{
    const int lane = threadIdx.x & 63, m = lane & 15, g = lane >> 4;
#pragma unroll
    for (int sl = 0; sl < NSL; ++sl) {
        float x[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int t = 32 * sl + 8 * g + j - m;
            x[j] = (t >= 0 && t <= 2 * R) ? tap[t] : 0.f;
        }
        split3(x, a[sl].h, a[sl].m, a[sl].l);
    }
}

__device__ __forceinline__ void split8(const f4 &x0, const f4 &x1, BF3 &b)
{
    const float x[8] = {x0[0], x0[1], x0[2], x0[3], x1[0], x1[1], x1[2], x1[3]};
    split3(x, b.h, b.m, b.l);
}

// ------------------------------------------------------------------ horizontal
// Tile: 16 rows x 256 output columns at (x0, y0); wave w owns columns
// 64w .. 64w+63 as four 16 x 16 blocks. The rows' inputs (x0 - R onwards)
// are staged in LDS, row-major with a pitch of 4 mod 8 floats.
template <int NC>
__device__ __forceinline__ void hpass_mfma_tile(const float *__restrict__ u, float *__restrict__ A,
                                               float *__restrict__ B, float *__restrict__ C, int H, int W,
                                               const WinTaps &t, int x0, int y0, float *lds)
{
#pragma clang fp contract(off)   // fused multiply-adds are written out
    constexpr int K = 16 * NC;
    constexpr int Lc = kHMW - 16 + K;   // staged columns
    constexpr int P = Lc + 4;
    const int R = t.R;
    float ag[NC][4], a1[NC][4], a2[NC][4];
    toeplitz_lane<NC>(t.g, R, ag);
    toeplitz_lane<NC>(t.d1, R, a1);
    toeplitz_lane<NC>(t.d2, R, a2);
    // 16 rows x Lc columns = (Lc / 16) values per thread, all loads issued
    // before the LDS stores
    constexpr int NI = Lc / 16;
    const bool interior = (x0 - R >= 0) && (x0 - R + Lc <= W);
    float v[NI];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int i = threadIdx.x + 256 * it;
        const int r = i / Lc, c = i - r * Lc;
        const int gy = min(y0 + r, H - 1);
        const int gx = x0 - R + c;
        v[it] = u[(size_t)gy * W + (interior ? gx : reflect_any(gx, W))];
    }
#pragma unroll
    for (int it = 0; it < NI; ++it) {
        const int i = threadIdx.x + 256 * it;
        const int r = i / Lc, c = i - r * Lc;
        lds[r * P + c] = v[it];
    }
    __builtin_amdgcn_s_waitcnt(0);   // taps and staged values have arrived
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int n = lane & 15, kq = lane >> 4;
    const int JL = last_slices<NC>(R);
    const float *row = lds + n * P;   // image row y0 + n
    const int y = y0 + n;
    const float gsum = t.gsum;
    const bool vec = ((W & 3) == 0) && ((((uintptr_t)A | (uintptr_t)B | (uintptr_t)C) & 15) == 0);
#pragma unroll 1
    for (int blk = 0; blk < 4; ++blk) {
        const int xb = 64 * wv + 16 * blk;   // staged column of the block's input x0 + xb - R
        const float ref = row[xb + R];       // input at the block's first output
        f4 cg = {0.f, 0.f, 0.f, 0.f}, c1 = cg, c2 = cg;
#pragma unroll
        for (int c = 0; c < NC - 1; ++c) {
            const f4 b = *(const f4 *)(row + xb + 16 * c + 4 * kq) - ref;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                cg = mfma_f32(ag[c][j], b[j], cg);
                c1 = mfma_f32(a1[c][j], b[j], c1);
                c2 = mfma_f32(a2[c][j], b[j], c2);
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < JL) {
                const float b = row[xb + 16 * (NC - 1) + 4 * j + kq] - ref;
                cg = mfma_f32(ag[NC - 1][j], b, cg);
                c1 = mfma_f32(a1[NC - 1][j], b, c1);
                c2 = mfma_f32(a2[NC - 1][j], b, c2);
            }
        // this lane holds outputs x0 + xb + 4 kq + i of row y
        const int xo = x0 + xb + 4 * kq;
        if (y < H && xo < W) {
            const float gref = ref * gsum;
            const size_t o = (size_t)y * W + xo;
            if (vec && xo + 3 < W) {
                *(f4 *)(A + o) = cg + gref;
                *(f4 *)(B + o) = c1;
                *(f4 *)(C + o) = c2;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (xo + i < W) {
                        A[o + i] = cg[i] + gref;
                        B[o + i] = c1[i];
                        C[o + i] = c2[i];
                    }
            }
        }
    }
}

// ------------------------------------------------------------------ vertical
// Strip: 32 columns at x0, output rows ys .. ye-1 (ys a multiple of 32,
// ye <= H). The three horizontal-pass planes stream through an LDS ring of
// K + 48 rows (column-major, so a lane's four consecutive rows are one
// 16-byte read): each step filters 32 rows (wave w: columns 16 (w & 1),
// rows 16 (w >> 1)) from the K + 16 rows of its window while the next 32
// rows are loaded into the other 32 slots, so one barrier per step
// suffices. Writes S, the blob factor and N; returns the largest S this
// thread wrote (0 if none).
template <int NC>
__device__ __forceinline__ float vpass_mfma_tile(const float *__restrict__ A, const float *__restrict__ B,
                                                 const float *__restrict__ C, int H, int W, const WinTaps &t,
                                                 float sigma2, float inv2beta2, int mode, float *__restrict__ SA,
                                                 float *__restrict__ No, int x0, int ys,
                                                 int ye, float *lds)
{
#pragma clang fp contract(off)   // fused multiply-adds are written out
    constexpr int K = 16 * NC;
    constexpr int RS = K + 48;   // ring rows; ring slot of input row y is (y - ys + R) mod RS
    constexpr int P = RS + 4;    // column pitch (4 mod 8 floats)
    constexpr int PL = kVMW * P;
    const int R = t.R;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int n = lane & 15, kq = lane >> 4;
    const int fc = tid & 31, fq = tid >> 5;   // loader: column, quad of rows
    const int JL = last_slices<NC>(R);
    const size_t fx = (size_t)min(x0 + fc, W - 1);
    float *fA = lds + fc * P;
    float ag[NC][4], a1[NC][4], a2[NC][4];
    toeplitz_lane<NC>(t.g, R, ag);
    toeplitz_lane<NC>(t.d1, R, a1);
    toeplitz_lane<NC>(t.d2, R, a2);
    // rows r0 + 4 fq + i, i < 4, of the three planes into registers
    auto load_quad = [&](int r0, f4 &va, f4 &vb, f4 &vc) {
        const bool inside = r0 >= 0 && r0 + 32 <= H;   // uniform over the block
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int y = r0 + 4 * fq + i;
            const size_t o = (size_t)(inside ? y : reflect_any(y, H)) * W + fx;
            va[i] = A[o];
            vb[i] = B[o];
            vc[i] = C[o];
        }
    };
    // prologue: the first window, rows ys - R .. ys - R + K + 15, 32 rows per pass
    constexpr int NQ = (K + 16 + 31) / 32;
#pragma unroll
    for (int q0 = 0; q0 < NQ; ++q0) {
        if (q0 * 32 + 4 * fq < K + 16) {
            f4 va, vb, vc;
            load_quad(ys - R + 32 * q0, va, vb, vc);
            *(f4 *)(fA + 32 * q0 + 4 * fq) = va;
            *(f4 *)(fA + PL + 32 * q0 + 4 * fq) = vb;
            *(f4 *)(fA + 2 * PL + 32 * q0 + 4 * fq) = vc;
        }
    }
    __builtin_amdgcn_s_waitcnt(0);   // taps and ring rows have arrived
    __syncthreads();
    const int col = 16 * (wv & 1) + n;
    const int x = x0 + col;
    const float *rA = lds + col * P, *rB = rA + PL, *rC = rA + 2 * PL;
    const size_t plane = (size_t)H * W;
    const float gsum = t.gsum;
    float smax = 0.f;
    for (int yb = ys; yb < ye; yb += kVMStep) {
        const bool more = yb + kVMStep < ye;
        f4 na, nb, nc;   // rows of the next step (loaded even after the last step: the count stays fixed)
        load_quad(yb - R + K + 16, na, nb, nc);
        const int y0 = yb + 16 * (wv >> 1);
        const int s0 = (y0 - ys) % RS;           // slot of input row y0 - R
        const int sr = (y0 - ys + R) % RS;       // slot of input row y0
        const float aref = rA[sr], bref = rB[sr];
        f4 cuy = {0.f, 0.f, 0.f, 0.f}, cuyy = cuy, cux = cuy, cuxy = cuy, cuxx = cuy;
#pragma unroll
        for (int c = 0; c < NC - 1; ++c) {
            int s = s0 + 16 * c + 4 * kq;
            s = s >= RS ? s - RS : s;
            const f4 va = *(const f4 *)(rA + s) - aref;
            const f4 vb = *(const f4 *)(rB + s) - bref;
            const f4 vc = *(const f4 *)(rC + s);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                cuy = mfma_f32(a1[c][j], va[j], cuy);
                cuyy = mfma_f32(a2[c][j], va[j], cuyy);
                cux = mfma_f32(ag[c][j], vb[j], cux);
                cuxy = mfma_f32(a1[c][j], vb[j], cuxy);
                cuxx = mfma_f32(ag[c][j], vc[j], cuxx);
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < JL) {   // last chunk, contiguous slices
                int s = s0 + 16 * (NC - 1) + 4 * j + kq;
                s = s >= RS ? s - RS : s;
                const float va = rA[s] - aref, vb = rB[s] - bref, vc = rC[s];
                cuy = mfma_f32(a1[NC - 1][j], va, cuy);
                cuyy = mfma_f32(a2[NC - 1][j], va, cuyy);
                cux = mfma_f32(ag[NC - 1][j], vb, cux);
                cuxy = mfma_f32(a1[NC - 1][j], vb, cuxy);
                cuxx = mfma_f32(ag[NC - 1][j], vc, cuxx);
            }
        if (more) {   // the next step's rows go to the slots no window of this step uses
            const int sn = (yb - ys + K + 16 + 4 * fq) % RS;
            *(f4 *)(fA + sn) = na;
            *(f4 *)(fA + PL + sn) = nb;
            *(f4 *)(fA + 2 * PL + sn) = nc;
        }
        // this lane holds rows y0 + 4 kq + i of column x
        const float bsum = bref * gsum;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int y = y0 + 4 * kq + i;
            if (x < W && y < ye) {
                const float Sv = vessel_store_mode(mode, cuxx[i], cuxy[i], cuyy[i], cux[i] + bsum, cuy[i], sigma2,
                                                   inv2beta2, SA, No, (size_t)y * W + x, plane);
                smax = fmaxf(smax, Sv);
            }
        }
        __syncthreads();
    }
    return smax;
}


// ------------------------------------------------------------------ fused
// Both passes of one scale on a strip of 32 columns at x0, output rows
// ys .. ye-1 (ys a multiple of 32, ye <= H), without the horizontal-pass
// planes in HBM. Each step stages 32 rows of u (columns x0 - R onwards) in
// LDS, runs the horizontal products on them (wave w: columns 16 (w & 1),
// rows 16 (w >> 1), the same 16 x 16 blocks and shifts as hpass_mfma_tile)
// and puts the three results into the vertical pass's ring of K + 16 rows,
// whose products and per-pixel outputs are those of vpass_mfma_tile; the
// values equal those of the two separate passes bit for bit. Rows outside
// the image are the horizontal pass of the reflected row of u.
// With an even number of chunks the products are split-BF16 instead
// (32-input slices on v_mfma_f32_16x16x32_bf16, six part products per FP32
// product): the same staging, shifts, ring and epilogue, about 1.25x the rate
// of the FP32 form at sigma = 16, but not the bits of the FP32 split passes.
// Odd chunk counts keep FP32 products: 32-input slices would read past the
// staged row.
// Split level of the fused sweep (split-BF16 products only): which ring planes
// hold their three BF16 parts, formed once as a row enters the ring, instead
// of FP32 values split by every window that reads them. Level 1: C (the second
// x-difference); level 2: C and B (the first). Both enter the vertical products
// unshifted, so every window would split a row the same way: the products are
// the same bits at every level. A part plane takes 1.5x the LDS of an FP32
// one, so the level is chosen per chunk count by what keeps the workgroups per
// CU: 2 at 2 and 6 chunks, 1 at 4 (level 2 would drop it from three to two),
// 0 at 8 (84 KB at level 1 would drop it from two to one). Concurrent scales
// run 8 chunks at one workgroup per CU anyway, so they take level 2 there.
__host__ __device__ constexpr int fused_level_default(int nc)
{
    return nc % 2 ? 0 : (nc == 4 ? 1 : (nc == 8 ? 0 : 2));
}
__host__ __device__ constexpr int fused_cpitch(int nc) { return 16 * nc + 24; }   // part plane pitch (halves)
// LDS: the FP32 ring planes (A, and B and C below their levels), the part
// planes (pitch 8 mod 16 halves: a lane's 16-byte window reads fall on distinct
// banks) and the staged rows of u (the size of an FP32 ring plane)
__host__ __device__ constexpr size_t fused_lds(int nc, int lv)
{
    return sizeof(float) * (4 - lv) * kVMW * (16 * nc + 16 + 4) + sizeof(uint16_t) * 3 * lv * kVMW * fused_cpitch(nc);
}
__host__ __device__ constexpr size_t fused_lds(int nc) { return fused_lds(nc, fused_level_default(nc)); }

template <int NC, int LV = fused_level_default(NC)>
__device__ __forceinline__ float sweep_fused_tile(const float *__restrict__ u, int H, int W, const WinTaps &t,
                                                  float sigma2, float inv2beta2, int mode, float *__restrict__ SA,
                                                  float *__restrict__ No, int x0, int ys,
                                                  int ye, float *lds)
{
#pragma clang fp contract(off)   // fused multiply-adds are written out
    constexpr int K = 16 * NC;
    constexpr int RS = K + 16;        // ring rows; ring slot of row y is (y - ys + R) mod RS
    constexpr int P = RS + 4;         // ring column pitch (4 mod 8 floats)
    constexpr int PL = kVMW * P;
    constexpr int UW = K + 16;        // staged u columns x0 - R .. x0 - R + UW - 1
    constexpr int UP = UW + 4;        // staged row pitch (4 mod 8 floats)
    constexpr int NG = UW / 16;       // 16-column groups of a staged row
    constexpr int NU = 2 * NG;        // staged values per thread: row 16 h + tid / 16, column 16 g + tid % 16
    // even chunk counts: split-BF16 products over NC / 2 slices of 32 inputs
    constexpr bool BF = (NC % 2 == 0);
    static_assert(LV >= 0 && LV <= 2 && (BF || LV == 0), "planes are split only for split-BF16 products");
    constexpr int CP = fused_cpitch(NC);   // pitch of a part plane (halves)
    constexpr int CPL = kVMW * CP;         // halves per part plane
    // FP32 planes A, then B (LV < 2) and C (LV < 1) at ring + PL, ring + 2 PL;
    // then the part planes [3][kVMW][CP] of C (LV >= 1) and B (LV >= 2)
    float *ring = lds;
    uint16_t *cpart = (uint16_t *)(lds + (3 - LV) * PL);
    uint16_t *bpart = cpart + 3 * CPL;
    float *us = (float *)(cpart + 3 * LV * CPL);
    const int R = t.R;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: the ring slots below are scalar
    const int n = lane & 15, kq = lane >> 4;
    const int tr = tid >> 4, tc = tid & 15;               // staging: row and column of value 0
    const int JL = last_slices<NC>(R);
    const int cb = 16 * (wv & 1), rb = 16 * (wv >> 1);   // this wave's block: columns cb.., rows rb..
    const bool xin = (x0 - R >= 0) && (x0 - R + UW <= W);
    constexpr int NSL = BF ? NC / 2 : 1;
    constexpr int NCF = BF ? 1 : NC;
    float ag[NCF][4], a1[NCF][4], a2[NCF][4];
    BF3 bg[NSL], b1[NSL], b2[NSL];
    if constexpr (BF) {
        toeplitz_bf3<NSL>(t.g, R, bg);
        toeplitz_bf3<NSL>(t.d1, R, b1);
        toeplitz_bf3<NSL>(t.d2, R, b2);
    } else {
        toeplitz_lane<NC>(t.g, R, ag);
        toeplitz_lane<NC>(t.d1, R, a1);
        toeplitz_lane<NC>(t.d2, R, a2);
    }
    const float gsum = t.gsum;
    // 32 rows of u from row r0 on (reflected), all loads before any LDS store;
    // value 2 g + h is row r0 + 16 h + tr, column x0 - R + 16 g + tc, so inside
    // the image every load is one base address plus a constant
    auto load_u = [&](int r0, float (&v)[NU]) {
        if (xin && r0 >= 0 && r0 + 32 <= H) {   // uniform over the block
            const float *p0 = u + (size_t)(r0 + tr) * W + (x0 - R + tc);
            const float *p1 = p0 + (size_t)16 * W;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                v[2 * g] = p0[16 * g];
                v[2 * g + 1] = p1[16 * g];
            }
        } else {
#pragma unroll
            for (int g = 0; g < NG; ++g)
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int gy = reflect_any(r0 + 16 * h + tr, H);
                    const int gx = reflect_any(x0 - R + 16 * g + tc, W);
                    v[2 * g + h] = u[(size_t)gy * W + gx];
                }
        }
    };
    auto store_u = [&](const float (&v)[NU]) {
        float *q = us + tr * UP + tc;
#pragma unroll
        for (int g = 0; g < NG; ++g)
#pragma unroll
            for (int h = 0; h < 2; ++h) q[16 * h * UP + 16 * g] = v[2 * g + h];
    };
    // horizontal products of this wave's block of the staged rows; lane holds
    // columns cb + 4 kq + i of staged row rb + n
    auto hpass_block = [&](f4 &hg, f4 &h1, f4 &h2) {
#pragma clang fp contract(off)   // as in hpass_mfma_tile: the shift is added back after rounding ref * gsum
        const float *row = us + (rb + n) * UP;
        const float ref = row[cb + R];
        hg = (f4){0.f, 0.f, 0.f, 0.f};
        h1 = hg;
        h2 = hg;
        if constexpr (BF) {
#pragma unroll
            for (int sl = 0; sl < NSL; ++sl) {
                const float *q = row + cb + 32 * sl + 8 * kq;
                BF3 b;
                split8(*(const f4 *)q - ref, *(const f4 *)(q + 4) - ref, b);
                hg = mfma_bf3(bg[sl], b, hg);
                h1 = mfma_bf3(b1[sl], b, h1);
                h2 = mfma_bf3(b2[sl], b, h2);
            }
            hg = hg + ref * gsum;
            return;
        }
#pragma unroll
        for (int c = 0; c < NCF - 1; ++c) {
            const f4 b = *(const f4 *)(row + cb + 16 * c + 4 * kq) - ref;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                hg = mfma_f32(ag[c][j], b[j], hg);
                h1 = mfma_f32(a1[c][j], b[j], h1);
                h2 = mfma_f32(a2[c][j], b[j], h2);
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < JL) {   // last chunk, contiguous slices
                const float b = row[cb + 16 * (NCF - 1) + 4 * j + kq] - ref;
                hg = mfma_f32(ag[NCF - 1][j], b, hg);
                h1 = mfma_f32(a1[NCF - 1][j], b, h1);
                h2 = mfma_f32(a2[NCF - 1][j], b, h2);
            }
        hg = hg + ref * gsum;
    };
    // the three BF16 parts of split3 of x, as their upper halves
    auto put_parts = [&](uint16_t *q, float x) {
        const float h = bf_trunc(x), r = x - h, m = bf_trunc(r);
        q[0] = (uint16_t)(__float_as_uint(h) >> 16);
        q[CPL] = (uint16_t)(__float_as_uint(m) >> 16);
        q[2 * CPL] = (uint16_t)(__float_as_uint(r - m) >> 16);
    };
    auto ring_put = [&](int slot, const f4 &hg, const f4 &h1, const f4 &h2) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int c = cb + 4 * kq + i;
            float *cp = ring + c * P + slot;
            cp[0] = hg[i];
            if constexpr (LV >= 2) put_parts(bpart + c * CP + slot, h1[i]);
            else cp[PL] = h1[i];
            if constexpr (LV >= 1) put_parts(cpart + c * CP + slot, h2[i]);
            else cp[2 * PL] = h2[i];
        }
    };
    // prologue: the first window, rows ys - R .. ys - R + RS - 1, 32 rows at a time
    constexpr int NB0 = (RS + 31) / 32;
#pragma unroll 1
    for (int bt = 0; bt < NB0; ++bt) {
        float v[NU];
        load_u(ys - R + 32 * bt, v);
        if (bt > 0) __syncthreads();   // the previous batch's staged rows have been read
        store_u(v);
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        f4 hg, h1, h2;
        hpass_block(hg, h1, h2);
        const int slot = 32 * bt + rb + n;
        if (slot < RS) ring_put(slot, hg, h1, h2);
    }
    {   // staged u for the rows that enter the window of the second step
        float v[NU];
        load_u(ys - R + RS, v);
        __syncthreads();
        store_u(v);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    const int col = cb + n;
    const int x = x0 + col;
    const float *rA = ring + col * P, *rB = rA + PL;
    // Window reads: slot s0 of a step's first window row is a multiple of 16
    // (steps of 32 rows, blocks of 16) and RS = 16 (NC + 1), so each 16-slot
    // chunk wraps around the ring as a whole and its wrap is wave-uniform;
    // the lane's offset within the chunk (4 kq, or kq in the last chunk's
    // slices) is added after the wrap.
    const float *rAq = rA + 4 * kq, *rAk = rA + kq;
    const size_t plane = (size_t)H * W;
    float smax = 0.f;
    // u rows entering the window two steps ahead: loaded at the end of the
    // previous step (loop-carried), so they are in flight during the epilogue
    // and this step's products (loaded even when unused)
    float v[NU];
    load_u(ys + kVMStep - R + RS, v);
    for (int yb = ys; yb < ye; yb += kVMStep) {
        const bool more = yb + kVMStep < ye;
        // vertical products of this step's window
        const int y0 = yb + rb;
        const int s0 = (y0 - ys) % RS;           // slot of row y0 - R
        const int sr = (y0 - ys + R) % RS;       // slot of row y0
        // split-BF16 products take B unshifted: it already vanishes exactly on
        // rows that are constant around the block (the horizontal shift)
        const float aref = rA[sr], bref = BF ? 0.f : rB[sr];
        f4 cuy = {0.f, 0.f, 0.f, 0.f}, cuyy = cuy, cux = cuy, cuxy = cuy, cuxx = cuy;
        if constexpr (BF) {
            // window rows 32 sl + 8 kq .. + 7 of this lane: an 8-slot group that
            // wraps around the ring as a whole (s0 and RS are multiples of 16)
#pragma unroll
            for (int sl = 0; sl < NSL; ++sl) {
                int sg = s0 + 32 * sl + 8 * kq;
                sg = sg >= RS ? sg - RS : sg;
                const float *q = rA + sg;
                BF3 va, vb, vc;
                split8(*(const f4 *)q - aref, *(const f4 *)(q + 4) - aref, va);
                if constexpr (LV >= 2) {
                    const uint16_t *qb = bpart + col * CP + sg;
                    vb.h.v = *(const bf8 *)qb;
                    vb.m.v = *(const bf8 *)(qb + CPL);
                    vb.l.v = *(const bf8 *)(qb + 2 * CPL);
                } else {
                    split8(*(const f4 *)(q + PL), *(const f4 *)(q + PL + 4), vb);
                }
                if constexpr (LV >= 1) {
                    const uint16_t *qc = cpart + col * CP + sg;
                    vc.h.v = *(const bf8 *)qc;
                    vc.m.v = *(const bf8 *)(qc + CPL);
                    vc.l.v = *(const bf8 *)(qc + 2 * CPL);
                } else {
                    split8(*(const f4 *)(q + 2 * PL), *(const f4 *)(q + 2 * PL + 4), vc);
                }
                cuy = mfma_bf3(b1[sl], va, cuy);
                cuyy = mfma_bf3(b2[sl], va, cuyy);
                cux = mfma_bf3(bg[sl], vb, cux);
                cuxy = mfma_bf3(b1[sl], vb, cuxy);
                cuxx = mfma_bf3(bg[sl], vc, cuxx);
            }
        } else {
#pragma unroll
        for (int c = 0; c < NCF - 1; ++c) {
            int sc = s0 + 16 * c;
            sc = sc >= RS ? sc - RS : sc;
            const float *q = rAq + sc;
            const f4 va = *(const f4 *)q - aref;
            const f4 vb = *(const f4 *)(q + PL) - bref;
            const f4 vc = *(const f4 *)(q + 2 * PL);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                cuy = mfma_f32(a1[c][j], va[j], cuy);
                cuyy = mfma_f32(a2[c][j], va[j], cuyy);
                cux = mfma_f32(ag[c][j], vb[j], cux);
                cuxy = mfma_f32(a1[c][j], vb[j], cuxy);
                cuxx = mfma_f32(ag[c][j], vc[j], cuxx);
            }
        }
        int sl = s0 + 16 * (NCF - 1);
        sl = sl >= RS ? sl - RS : sl;
        const float *ql = rAk + sl;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j < JL) {   // last chunk, contiguous slices
                const float va = ql[4 * j] - aref, vb = ql[PL + 4 * j] - bref, vc = ql[2 * PL + 4 * j];
                cuy = mfma_f32(a1[NCF - 1][j], va, cuy);
                cuyy = mfma_f32(a2[NCF - 1][j], va, cuyy);
                cux = mfma_f32(ag[NCF - 1][j], vb, cux);
                cuxy = mfma_f32(a1[NCF - 1][j], vb, cuxy);
                cuxx = mfma_f32(ag[NCF - 1][j], vc, cuxx);
            }
        }
        // horizontal products of the rows entering the next window
        f4 hg, h1, h2;
        hpass_block(hg, h1, h2);
        __syncthreads();   // the window's first 32 rows and the staged rows have been read
        if (more) {
            // slots of rows yb - R .. yb - R + 31: a wave-uniform multiple of 16 plus n
            ring_put((yb - ys + rb) % RS + n, hg, h1, h2);
            store_u(v);
        }
        load_u(yb + 2 * kVMStep - R + RS, v);
        // this lane holds rows y0 + 4 kq + i of column x
        const float bsum = bref * gsum;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int y = y0 + 4 * kq + i;
            if (x < W && y < ye) {
                const float Sv = vessel_store_mode(mode, cuxx[i], cuxy[i], cuyy[i], cux[i] + bsum, cuy[i], sigma2,
                                                   inv2beta2, SA, No, (size_t)y * W + x, plane);
                smax = fmaxf(smax, Sv);
            }
        }
        __syncthreads();
    }
    return smax;
}

}  // namespace tiles
}  // namespace mf4d
