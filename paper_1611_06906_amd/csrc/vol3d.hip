// The filter on volumes (the 3-D extension that Sec. 5 names as the next
// step): scale sweep with Frangi's tube measure, the normalised integrated
// Hessian of Eq. (6) per component, the fourth-order tensor built from the
// eigentensors of H_rho as Eqs. (7), (8) build it in 2-D, and FED cycles
// (Eq. (21)) of the operator L^T D L with the 3-D second-difference stencils
// and natural boundaries. Volumes are float32 [D][H][W], x fastest.
//
// Kernels: the sweep's z and y passes produce 8 outputs per thread along the
// pass through register windows, the x pass stages its block's rows in LDS
// and ends in the per-voxel tube factor and N planes; the argmax and the
// eigen-solves map one thread to one voxel (blocks of 64 x 4 threads over
// (x, y), one z plane per grid layer, so a wave reads and writes 64
// consecutive floats of a row); the integration and the FED substep march
// along z over tiles of (x, y) with LDS and register rings. The eigen-solves
// (or, without the mode masks, the inverse that replaces them) run in FP64;
// the tensor is stored as the six entries of P = Q diag(mu) Q^T.
#include <cmath>
#include <cstring>
#include <vector>

#include "mf4d_internal.h"

using namespace mf4d;

namespace {

constexpr double kTauLimit3 = 1.0 / 27.0;   // stencil bound 3 * 16 + 6 * 1 = 54, tau <= 2 / 54
constexpr double kAlpha3 = 0.5;             // Frangi's plate/line parameter of the tube measure
typedef float vf2 __attribute__((ext_vector_type(2)));   // 8-byte nontemporal accesses
constexpr int kBX = 64, kBY = 4;

// Half-sample symmetric extension for any i (period 2n).
__device__ __forceinline__ int sym_index(int i, int n)
{
    const int p = 2 * n;
    int j = i % p;
    j = j < 0 ? j + p : j;
    return j < n ? j : p - 1 - j;
}

// Consecutive workgroups go to the 8 XCDs in turn: renumber them so that
// each XCD takes a contiguous run of tiles (a bijection for any grid size),
// and the halo lines that neighbouring tiles share stay in its L2.
__device__ __forceinline__ int xcd_block()
{
    const int nb = gridDim.x, q8 = nb >> 3, r8 = nb & 7, xcd = blockIdx.x & 7;
    return (xcd < r8 ? xcd * (q8 + 1) : r8 * (q8 + 1) + (xcd - r8) * q8) + (blockIdx.x >> 3);
}

struct Vox {
    int x, y, z;
    size_t o;        // linear index
    bool inside;
};

__device__ __forceinline__ Vox voxel(int D, int H, int W)
{
    Vox v;
    v.x = blockIdx.x * kBX + threadIdx.x;
    v.y = blockIdx.y * kBY + threadIdx.y;
    v.z = blockIdx.z;
    v.inside = v.x < W && v.y < H && v.z < D;
    v.o = ((size_t)v.z * H + v.y) * W + v.x;
    return v;
}

// ------------------------------------------------------------------ sweep
// The three separable passes of one scale run z, y, x: the pass with one
// input reads whole planes apart, the pass with six inputs reads along rows.
// Inputs are shifted by the voxel's own value (constant lines give exact
// zeros); each Gaussian output adds it back.
//
// Pass along z: Z = (G, D1 G, D2 G) u, planes [3][m]. A thread produces kLW
// consecutive outputs of one (y, x) column and streams the column's inputs
// through a kLW-entry register window (input z0 - R + i in slot i mod kLW),
// so each input is loaded once for up to kLW outputs; every output takes its
// taps in the same order as a one-output loop would, so the values are the
// same.
constexpr int kLW = 8;   // outputs per thread along the pass (z and y passes)

__global__ __launch_bounds__(256) void sweep3_z_kernel(const float *__restrict__ u, float *__restrict__ Z, int D,
                                                       int H, int W, WinTaps t)
{
    const int x = blockIdx.x * kBX + threadIdx.x, y = blockIdx.y * kBY + threadIdx.y, z0 = blockIdx.z * kLW;
    if (x >= W || y >= H) return;
    const size_t plane = (size_t)H * W, m = plane * D;
    const size_t pos = (size_t)y * W + x;   // voxel (0, y, x)
    const int R = t.R, nt = 2 * R + 1;
    const bool inner = z0 - R >= 0 && z0 + kLW - 1 + R < D;   // the same for the whole block
    auto in = [&](int z) { return u[pos + (size_t)(inner ? z : sym_index(z, D)) * plane]; };
    float ref[kLW], w[kLW], g[kLW], d1[kLW], d2[kLW];
#pragma unroll
    for (int j = 0; j < kLW; ++j) {
        ref[j] = z0 + j < D ? u[pos + (size_t)(z0 + j) * plane] : 0.f;
        w[j] = in(z0 - R + j);
        g[j] = d1[j] = d2[j] = 0.f;
    }
    for (int t0 = 0; t0 < nt; t0 += kLW) {
#pragma unroll
        for (int t1 = 0; t1 < kLW; ++t1) {
            const int k = t0 + t1;
            if (k < nt) {
                const float tg = t.g[k], td1 = t.d1[k], td2 = t.d2[k];
#pragma unroll
                for (int j = 0; j < kLW; ++j) {
                    const float a = w[(j + t1) % kLW] - ref[j];   // input z0 + j + k - R
                    g[j] = fmaf(tg, a, g[j]);
                    d1[j] = fmaf(td1, a, d1[j]);
                    d2[j] = fmaf(td2, a, d2[j]);
                }
                // replaces input z0 - R + k, used by no later tap; the last tap's
                // replacement would be used by none (and may lie past the volume)
                if (k + 1 < nt) w[t1] = in(z0 - R + k + kLW);
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kLW; ++j)
        if (z0 + j < D) {
            const size_t o = pos + (size_t)(z0 + j) * plane;
            Z[o] = g[j] + ref[j] * t.gsum;
            Z[m + o] = d1[j];
            Z[2 * m + o] = d2[j];
        }
}

// Pass along y: from Z0 = G u the outputs (G, D1 G, D2 G), from Z1 = D1 u the
// outputs (G, D1 G), from Z2 = D2 u the output G. Y planes [6][m] in the
// order Y00, Y01, Y02, Y10, Y11, Y20 (first digit: z filter, second: y filter).
// A thread produces kLW consecutive outputs of one (z, x) row through three
// register windows, as the z pass does.
__global__ __launch_bounds__(256) void sweep3_y_kernel(const float *__restrict__ Z, float *__restrict__ Y, int D,
                                                       int H, int W, WinTaps t)
{
    const int x = blockIdx.x * kBX + threadIdx.x, y0 = (blockIdx.y * kBY + threadIdx.y) * kLW, z = blockIdx.z;
    if (x >= W || y0 >= H) return;
    const size_t m = (size_t)D * H * W;
    const size_t col = (size_t)z * H * W + x;   // voxel (z, 0, x)
    const int R = t.R, nt = 2 * R + 1;
    const bool inner = y0 - R >= 0 && y0 + kLW - 1 + R < H;
    auto at = [&](int y) { return col + (size_t)(inner ? y : sym_index(y, H)) * W; };
    float r0[kLW], r1[kLW], r2[kLW], w0[kLW], w1[kLW], w2[kLW];
    float a00[kLW], a01[kLW], a02[kLW], a10[kLW], a11[kLW], a20[kLW];
#pragma unroll
    for (int j = 0; j < kLW; ++j) {
        const size_t o = col + (size_t)(y0 + j < H ? y0 + j : H - 1) * W;
        r0[j] = Z[o];
        r1[j] = Z[m + o];
        r2[j] = Z[2 * m + o];
        const size_t q = at(y0 - R + j);
        w0[j] = Z[q];
        w1[j] = Z[m + q];
        w2[j] = Z[2 * m + q];
        a00[j] = a01[j] = a02[j] = a10[j] = a11[j] = a20[j] = 0.f;
    }
    for (int t0 = 0; t0 < nt; t0 += kLW) {
#pragma unroll
        for (int t1 = 0; t1 < kLW; ++t1) {
            const int k = t0 + t1;
            if (k < nt) {
                const float tg = t.g[k], td1 = t.d1[k], td2 = t.d2[k];
#pragma unroll
                for (int j = 0; j < kLW; ++j) {
                    const int sl = (j + t1) % kLW;   // input y0 + j + k - R
                    const float b0 = w0[sl] - r0[j], b1 = w1[sl] - r1[j], b2 = w2[sl] - r2[j];
                    a00[j] = fmaf(tg, b0, a00[j]);
                    a01[j] = fmaf(td1, b0, a01[j]);
                    a02[j] = fmaf(td2, b0, a02[j]);
                    a10[j] = fmaf(tg, b1, a10[j]);
                    a11[j] = fmaf(td1, b1, a11[j]);
                    a20[j] = fmaf(tg, b2, a20[j]);
                }
                if (k + 1 < nt) {   // as in the z pass: the last tap's replacement is never used
                    const size_t q = at(y0 - R + k + kLW);
                    w0[t1] = Z[q];
                    w1[t1] = Z[m + q];
                    w2[t1] = Z[2 * m + q];
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < kLW; ++j)
        if (y0 + j < H) {
            const size_t o = col + (size_t)(y0 + j) * W;
            Y[o] = a00[j] + r0[j] * t.gsum;
            Y[m + o] = a01[j];
            Y[2 * m + o] = a02[j];
            Y[3 * m + o] = a10[j] + r1[j] * t.gsum;
            Y[4 * m + o] = a11[j];
            Y[5 * m + o] = a20[j] + r2[j] * t.gsum;
        }
}

// Eigenvalues of the symmetric 3 x 3 matrix (a00, a11, a22, a01, a02, a12)
// in descending order, from the trigonometric solution of its characteristic
// cubic in double: with q = tr/3, B = A - q I, p^2 = |B|_F^2 / 6 and
// r = det(B) / 2p^3, the roots are q + 2p cos(acos(r)/3 + 2 pi k/3). The
// error is a few ulp of |A| (about 1e-8 |A| where two roots nearly
// coincide), far below that of the float32 Hessian.
// sin and cos of x in [0, pi/3] from their Taylor series through x^19 and
// x^18 (Horner in x^2): the truncation error there is below x^20/20! < 2e-18.
__device__ __forceinline__ void sincos_small(double x, double &s, double &c)
{
    const double x2 = x * x;
    double ps = 1.0 / 121645100408832000.0;               // 1/19!
    ps = fma(ps, x2, -1.0 / 355687428096000.0);           // 1/17!
    ps = fma(ps, x2, 1.0 / 1307674368000.0);              // 1/15!
    ps = fma(ps, x2, -1.0 / 6227020800.0);                // 1/13!
    ps = fma(ps, x2, 1.0 / 39916800.0);                   // 1/11!
    ps = fma(ps, x2, -1.0 / 362880.0);                    // 1/9!
    ps = fma(ps, x2, 1.0 / 5040.0);                       // 1/7!
    ps = fma(ps, x2, -1.0 / 120.0);                       // 1/5!
    ps = fma(ps, x2, 1.0 / 6.0);                          // 1/3!
    s = fma(-x * x2, ps, x);
    double pc = 1.0 / 6402373705728000.0;                 // 1/18!
    pc = fma(pc, x2, -1.0 / 20922789888000.0);            // 1/16!
    pc = fma(pc, x2, 1.0 / 87178291200.0);                // 1/14!
    pc = fma(pc, x2, -1.0 / 479001600.0);                 // 1/12!
    pc = fma(pc, x2, 1.0 / 3628800.0);                    // 1/10!
    pc = fma(pc, x2, -1.0 / 40320.0);                     // 1/8!
    pc = fma(pc, x2, 1.0 / 720.0);                        // 1/6!
    pc = fma(pc, x2, -1.0 / 24.0);                        // 1/4!
    pc = fma(pc, x2, 0.5);                                // 1/2!
    c = fma(-x2, pc, 1.0);
}

__device__ __forceinline__ void sym3_eigenvalues(double a00, double a11, double a22, double a01, double a02,
                                                 double a12, double &e0, double &e1, double &e2)
{
    const double q = (a00 + a11 + a22) * (1.0 / 3.0);
    const double b00 = a00 - q, b11 = a11 - q, b22 = a22 - q;
    const double p2 = (b00 * b00 + b11 * b11 + b22 * b22 + 2.0 * (a01 * a01 + a02 * a02 + a12 * a12)) * (1.0 / 6.0);
    if (!(p2 > 0.0)) {
        e0 = e1 = e2 = q;
        return;
    }
    const double p = sqrt(p2);
    const double det = b00 * (b11 * b22 - a12 * a12) - a01 * (a01 * b22 - a12 * a02) + a02 * (a01 * a12 - b11 * a02);
    const double r = fmin(1.0, fmax(-1.0, det / (2.0 * p2 * p)));
    const double phi = acos(r) * (1.0 / 3.0);
    double sphi, cphi;
    sincos_small(phi, sphi, cphi);
    e0 = q + 2.0 * p * cphi;
    // cos(phi + 2 pi / 3) = -cos(phi) / 2 - sin(phi) sqrt(3) / 2
    e2 = q + 2.0 * p * (-0.5 * cphi - 0.86602540378443865 * sphi);
    e1 = 3.0 * q - e0 - e2;
}

__device__ __forceinline__ void swap_if(double &a, double &b, bool c)
{
    const double ta = a;
    a = c ? b : a;
    b = c ? ta : b;
}

// Frangi's tube measure without its S factor, for sigma^2 H: n1, n2, n3 are
// the eigenvalues by ascending magnitude (eigenvalues first in descending
// order, then the exchanges (0,1), (0,2), (1,2) wherever the later one is
// strictly smaller in magnitude); F = 0 where n2 n3 = 0 or the mode's sign
// test fails, else (1 - exp(-R_A^2 / 2 alpha^2)) exp(-R_B^2 / 2 beta^2) with
// R_A = |n2| / |n3|, R_B = |n1| / sqrt|n2 n3|.
__device__ __forceinline__ double tube_factor(double h00, double h11, double h22, double h01, double h02,
                                              double h12, int mode, double inv2beta2)
{
    double e0, e1, e2;
    sym3_eigenvalues(h00, h11, h22, h01, h02, h12, e0, e1, e2);
    swap_if(e0, e1, e1 > e0);   // descending
    swap_if(e0, e2, e2 > e0);
    swap_if(e1, e2, e2 > e1);
    swap_if(e0, e1, fabs(e1) < fabs(e0));   // ascending magnitude
    swap_if(e0, e2, fabs(e2) < fabs(e0));
    swap_if(e1, e2, fabs(e2) < fabs(e1));
    if (e1 * e2 == 0.0) return 0.0;
    if (mode == MF4D_RIDGE && (e1 > 0.0 || e2 > 0.0)) return 0.0;
    if (mode == MF4D_VALLEY && (e1 < 0.0 || e2 < 0.0)) return 0.0;
    const double a1 = fabs(e1), a2 = fabs(e2), inv = 1.0 / (a1 * a2 * a2);
    const double ra2 = a1 * a1 * a1 * inv;   // R_A^2 = n2^2 / n3^2
    const double rb2 = e0 * e0 * a2 * inv;   // R_B^2 = n1^2 / |n2 n3|
    // the two factors in float (F is stored as float): 1 - e^-x as -expm1
    const float fa = -expm1f(-(float)(ra2 * (0.5 / (kAlpha3 * kAlpha3))));
    const float fb = expf(-(float)(rb2 * inv2beta2));
    return (double)(fa * fb);
}

// Pass along x and the per-voxel outputs of one scale: the gradient and
// Hessian of u_sigma, S = |sigma^2 H|_F and the tube factor F (SF [m] pairs),
// N = H / sqrt(1 + |grad u_sigma|) (planes xx, yy, zz, xy, xz, yz), and the
// largest S into *smax_bits.
__global__ __launch_bounds__(256) void sweep3_x_kernel(const float *__restrict__ Y, float2 *__restrict__ SF,
                                                       float *__restrict__ N, unsigned *__restrict__ smax_bits,
                                                       int D, int H, int W, WinTaps t, float sigma2, int mode,
                                                       double inv2beta2)
{
    // the block's 4 rows of the six planes, columns x0 - R .. x0 + 63 + R
    // (reflected), staged in LDS: [6][kBY][SW]
    extern __shared__ float sy[];
    const Vox v = voxel(D, H, W);
    const int R = t.R, SW = kBX + 2 * R;
    const size_t m = (size_t)D * H * W;
    {
        // every load of a chunk of two columns per thread is issued before its
        // LDS stores (from clamped, in-bounds addresses; rows past the volume
        // store 0), so the thread waits for them once
        const int x0 = blockIdx.x * kBX;
        const bool row_in = v.y < H;
        const size_t row = ((size_t)v.z * H + (row_in ? v.y : 0)) * W;
        auto col = [&](int i) {
            const int gx = x0 - R + i;
            return (gx >= 0 && gx < W) ? gx : sym_index(gx, W);
        };
        for (int base = 0; base < SW; base += 2 * kBX) {
            const int ia = base + threadIdx.x, ib = ia + kBX;
            const size_t xa = row + col(min(ia, SW - 1)), xb = row + col(min(ib, SW - 1));
            float va[6], vb[6];
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                va[j] = Y[j * m + xa];
                vb[j] = Y[j * m + xb];
            }
            float *dst = sy + threadIdx.y * SW;
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                if (ia < SW) dst[j * kBY * SW + ia] = row_in ? va[j] : 0.f;
                if (ib < SW) dst[j * kBY * SW + ib] = row_in ? vb[j] : 0.f;
            }
        }
    }
    __syncthreads();
    float Sv = 0.f;
    if (v.inside) {
        const float *base = sy + threadIdx.y * SW + threadIdx.x;   // column x - R of plane 0
        const int PS = kBY * SW;                                    // plane stride
        float r[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) r[j] = base[j * PS + R];
        float gx = 0.f, gy = 0.f, gz = 0.f, hxx = 0.f, hyy = 0.f, hzz = 0.f, hxy = 0.f, hxz = 0.f, hyz = 0.f;
        for (int k = 0; k <= 2 * R; ++k) {
            const float *q = base + k;
            const float b00 = q[0] - r[0], b01 = q[PS] - r[1], b02 = q[2 * PS] - r[2];
            const float b10 = q[3 * PS] - r[3], b11 = q[4 * PS] - r[4], b20 = q[5 * PS] - r[5];
            const float g = t.g[k], d1 = t.d1[k], d2 = t.d2[k];
            gx = fmaf(d1, b00, gx);
            hxx = fmaf(d2, b00, hxx);
            gy = fmaf(g, b01, gy);
            hxy = fmaf(d1, b01, hxy);
            hyy = fmaf(g, b02, hyy);
            gz = fmaf(g, b10, gz);
            hxz = fmaf(d1, b10, hxz);
            hyz = fmaf(g, b11, hyz);
            hzz = fmaf(g, b20, hzz);
        }
        gy += r[1] * t.gsum;
        hyy += r[2] * t.gsum;
        gz += r[3] * t.gsum;
        hyz += r[4] * t.gsum;
        hzz += r[5] * t.gsum;
        const double s2 = sigma2;
        const double a00 = s2 * hxx, a11 = s2 * hyy, a22 = s2 * hzz, a01 = s2 * hxy, a02 = s2 * hxz, a12 = s2 * hyz;
        const double S = sqrt(a00 * a00 + a11 * a11 + a22 * a22 + 2.0 * (a01 * a01 + a02 * a02 + a12 * a12));
        const double F = tube_factor(a00, a11, a22, a01, a02, a12, mode, inv2beta2);
        Sv = (float)S;
        // written once and read once after every scale is done (SF by the
        // argmax, N gathered by the integration): nontemporal, so that they do
        // not evict the planes the next passes read
        __builtin_nontemporal_store(vf2{Sv, (float)F}, (vf2 *)(SF + v.o));
        const float f = 1.f / sqrtf(1.f + sqrtf(gx * gx + gy * gy + gz * gz));
        __builtin_nontemporal_store(hxx * f, N + v.o);
        __builtin_nontemporal_store(hyy * f, N + m + v.o);
        __builtin_nontemporal_store(hzz * f, N + 2 * m + v.o);
        __builtin_nontemporal_store(hxy * f, N + 3 * m + v.o);
        __builtin_nontemporal_store(hxz * f, N + 4 * m + v.o);
        __builtin_nontemporal_store(hyz * f, N + 5 * m + v.o);
    }
    // block maximum of S, then one atomic (S >= 0: float order = bit order).
    // The maximum only grows, so a block whose value does not exceed the one
    // already stored (possibly an older, smaller one) has nothing to add and
    // skips the atomic: with 65536 blocks per scale at 256^3, atomics on the
    // one address otherwise serialise (~0.36 ms per launch)
    __shared__ float red[kBX * kBY / 64];
    float mx = Sv;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off));
    const int tid = threadIdx.y * kBX + threadIdx.x;
    if ((tid & 63) == 0) red[tid >> 6] = mx;
    __syncthreads();
    if (tid == 0) {
        float b = red[0];
        for (int i = 1; i < kBX * kBY / 64; ++i) b = fmaxf(b, red[i]);
        if (__float_as_uint(b) > __atomic_load_n(smax_bits, __ATOMIC_RELAXED)) atomicMax(smax_bits, __float_as_uint(b));
    }
}

// ----------------------------------------------------------------- select
// V_s = F_s (1 - exp(-S_s^2 / 2 c^2)) with c = params c when > 0, else half
// the largest S over all scales and voxels; the smallest s of maximal V.
__global__ __launch_bounds__(256) void argmax3_kernel(const float2 *__restrict__ SF, int ns, const unsigned *smax_bits,
                                                      float c_param, uint8_t *__restrict__ idx,
                                                      float *__restrict__ vmax, float *__restrict__ c_out, int D,
                                                      int H, int W)
{
    const Vox v = voxel(D, H, W);
    const float c = c_param > 0.f ? c_param : 0.5f * __uint_as_float(*smax_bits);
    if (c_out && v.x == 0 && v.y == 0 && v.z == 0) *c_out = c;
    if (!v.inside) return;
    const size_t m = (size_t)D * H * W;
    int best = 0;
    float bv = 0.f;
    if (c > 0.f) {
        const float inv2c2 = 1.f / (2.f * c * c);
        for (int s = 0; s < ns; ++s) {
            const vf2 sf = __builtin_nontemporal_load((const vf2 *)(SF + s * m + v.o));
            const float val = sf.y * -expm1f(-(sf.x * sf.x) * inv2c2);
            if (s == 0 || val > bv) {
                bv = val;
                best = s;
            }
        }
    }
    idx[v.o] = (uint8_t)best;
    if (vmax) vmax[v.o] = bv;
}

// N at each voxel's scale (clamped to ns - 1), planes [6][m].
__global__ __launch_bounds__(256) void gather3_kernel(const float *__restrict__ N, const uint8_t *__restrict__ idx,
                                                      int ns, float *__restrict__ out, int D, int H, int W)
{
    const Vox v = voxel(D, H, W);
    if (!v.inside) return;
    const size_t m = (size_t)D * H * W;
    const int s = min((int)idx[v.o], ns - 1);
    const float *src = N + (size_t)s * 6 * m;
#pragma unroll
    for (int k = 0; k < 6; ++k) out[k * m + v.o] = src[k * m + v.o];
}

// G_rho along one axis (0: x, 1: y, 2: z) of the six planes.
template <int AXIS>
__global__ __launch_bounds__(256) void rho3_kernel(const float *__restrict__ in, float *__restrict__ out, int D, int H,
                                                   int W, RhoTaps t)
{
    const Vox v = voxel(D, H, W);
    if (!v.inside) return;
    const size_t plane = (size_t)H * W, m = plane * D;
    const int n = AXIS == 0 ? W : (AXIS == 1 ? H : D);
    const int c = AXIS == 0 ? v.x : (AXIS == 1 ? v.y : v.z);
    const size_t stride = AXIS == 0 ? 1 : (AXIS == 1 ? (size_t)W : plane);
    const size_t base = v.o - (size_t)c * stride;
    float acc[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[k] = t.g[0] * in[k * m + v.o];
    for (int j = 1; j <= t.r; ++j) {
        const size_t qm = base + (size_t)sym_index(c - j, n) * stride;
        const size_t qp = base + (size_t)sym_index(c + j, n) * stride;
#pragma unroll
        for (int k = 0; k < 6; ++k) acc[k] = fmaf(t.g[j], in[k * m + qm] + in[k * m + qp], acc[k]);
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) out[k * m + v.o] = acc[k];
}

// H_rho from N at the chosen scales in one kernel, for integration radii
// RR <= 2: a workgroup owns a kIX x kIY tile of output columns and marches
// along z over a segment of planes. Per plane it gathers N at each voxel's
// chosen scale over the tile and an RR-voxel xy halo into LDS, blurs it along
// x (halo rows included) into LDS and then along y into a per-thread register
// window of the last 2 RR + 1 planes, and blurs the window along z into the
// output plane RR behind. Each voxel takes the same operations in the same
// order as gather3_kernel and the three rho3_kernel passes (x, y, z;
// reflection per axis), so the values are the same, without writing and
// reading the gathered and the partly blurred planes.
// Where neighbouring voxels chose different scales, each 128-byte line of a
// gathered row brings in the lines of every scale present, so the kernel's
// fetch is several times its algorithmic bytes; in a tile 64 voxels wide
// the x halo's extra lines are two of a row's four (32 wide: two of three).
constexpr int kIX = 64, kIY = 16, kIZSeg = 32;

template <int RR>
__global__ __launch_bounds__(kIX * kIY) void integrate3_kernel(const float *__restrict__ N, const uint8_t *__restrict__ idx,
                                                         int ns, float *__restrict__ out, int D, int H, int W,
                                                         RhoTaps t, int tiles_x, int tiles_y)
{
    constexpr int AX = kIX + 2 * RR, AY = kIY + 2 * RR, NR = 2 * RR + 1, NT = kIX * kIY;
    constexpr int NIT = (AY * AX + NT - 1) / NT;   // gathered positions per thread
    __shared__ float sa[6][AY][AX];                // gathered N of one plane with the xy halo
    __shared__ float sb[6][AY][kIX];               // blurred along x
    const int tid = threadIdx.x;
    const int b = xcd_block();
    const int tx = b % tiles_x, ty = (b / tiles_x) % tiles_y, zs = b / (tiles_x * tiles_y);
    const int x0 = tx * kIX, y0 = ty * kIY, z0 = zs * kIZSeg, z1 = min(D, z0 + kIZSeg);
    const int pend = z1 + RR;                      // planes z0 - RR .. pend - 1
    const size_t m = (size_t)D * H * W, plane = (size_t)H * W;
    const int lx = tid % kIX, ly = tid / kIX;      // this thread's output column and row
    // The in-plane offsets of this thread's gathered positions (reflected at
    // the volume's sides), the scale indices loaded two planes ahead and N
    // loaded one plane ahead, so the loads of both are in flight while the
    // planes before them are blurred.
    size_t ofs[NIT];
    int sidx[NIT];
    float pre[NIT][6];
#pragma unroll
    for (int it = 0; it < NIT; ++it) {
        const int i = min(tid + it * NT, AY * AX - 1);
        const int ay = i / AX, ax = i - ay * AX;
        ofs[it] = (size_t)sym_index(y0 - RR + ay, H) * W + sym_index(x0 - RR + ax, W);
    }
    // (the indices are clamped only where they are used: a use right after
    // the load would wait for every load issued before it, N's included)
    auto fetch_idx = [&](int q) {
        const size_t zo = (size_t)sym_index(q, D) * plane;
#pragma unroll
        for (int it = 0; it < NIT; ++it) sidx[it] = idx[zo + ofs[it]];
    };
    auto fetch_n = [&](int q) {
        const size_t zo = (size_t)sym_index(q, D) * plane;
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const float *src = N + (size_t)min(sidx[it], ns - 1) * 6 * m + zo + ofs[it];
#pragma unroll
            for (int k = 0; k < 6; ++k) pre[it][k] = src[k * m];
        }
    };
    fetch_idx(z0 - RR);
    fetch_n(z0 - RR);
    if (z0 - RR + 1 < pend) fetch_idx(z0 - RR + 1);
    float win[NR][6];   // plane q blurred along x and y, in slot (q - z0 + RR) mod NR
    for (int pb = z0 - RR; pb < pend; pb += NR) {
#pragma unroll
        for (int u = 0; u < NR; ++u) {
            const int p = pb + u;
            if (p >= pend) break;
#pragma unroll
            for (int it = 0; it < NIT; ++it) {
                const int i = tid + it * NT;
                if (i < AY * AX) {
                    const int ay = i / AX, ax = i - ay * AX;
#pragma unroll
                    for (int k = 0; k < 6; ++k) sa[k][ay][ax] = pre[it][k];
                }
            }
            __syncthreads();
            if (p + 1 < pend) {
                fetch_n(p + 1);
                if (p + 2 < pend) fetch_idx(p + 2);
            }
            for (int i = tid; i < AY * kIX; i += NT) {
                const int ay = i / kIX, ox = i - ay * kIX;
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    float acc = t.g[0] * sa[k][ay][ox + RR];
#pragma unroll
                    for (int j = 1; j <= RR; ++j) acc = fmaf(t.g[j], sa[k][ay][ox + RR - j] + sa[k][ay][ox + RR + j], acc);
                    sb[k][ay][ox] = acc;
                }
            }
            __syncthreads();
            // sb is rewritten only after the next plane's first barrier, and
            // sa only after every thread has passed this one
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                float acc = t.g[0] * sb[k][ly + RR][lx];
#pragma unroll
                for (int j = 1; j <= RR; ++j) acc = fmaf(t.g[j], sb[k][ly + RR - j][lx] + sb[k][ly + RR + j][lx], acc);
                win[u][k] = acc;
            }
            // output plane z = p - RR from the window's planes z - RR .. z + RR
            const int z = p - RR;
            if (z >= z0) {
                const int x = x0 + lx, y = y0 + ly;
                const int c = (u + NR - RR) % NR;   // a constant once unrolled
#pragma unroll
                for (int k = 0; k < 6; ++k) {
                    float acc = t.g[0] * win[c][k];
#pragma unroll
                    for (int j = 1; j <= RR; ++j)
                        acc = fmaf(t.g[j], win[(c + NR - j) % NR][k] + win[(c + j) % NR][k], acc);
                    if (x < W && y < H) out[k * m + (size_t)z * plane + (size_t)y * W + x] = acc;
                }
            }
        }
    }
}

// ----------------------------------------------------------------- tensor
__device__ __forceinline__ void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Eigenpairs of the symmetric 3 x 3 matrix A (FP64): the eigenvalues from
// the cubic; the eigenvector of the root farthest from the middle one (a
// simple root unless all three coincide) as the longest cross product of two
// rows of A - lambda I; the other two from the symmetric 2 x 2 restriction of
// A to the plane orthogonal to it (its rotation from the half-angle forms),
// which stays well defined when those two roots coincide. nu[k] and column k
// of q.
__device__ __forceinline__ void sym3_eigenpairs(const double (&A)[3][3], double (&nu)[3], double (&q)[3][3])
{
    double e0, e1, e2;
    sym3_eigenvalues(A[0][0], A[1][1], A[2][2], A[0][1], A[0][2], A[1][2], e0, e1, e2);
    const bool top = (e0 - e1) >= (e1 - e2);
    const double lam = top ? e0 : e2;
    double r0[3] = {A[0][0] - lam, A[0][1], A[0][2]};
    double r1[3] = {A[1][0], A[1][1] - lam, A[1][2]};
    double r2[3] = {A[2][0], A[2][1], A[2][2] - lam};
    double c01[3], c02[3], c12[3];
    cross3(r0, r1, c01);
    cross3(r0, r2, c02);
    cross3(r1, r2, c12);
    const double n01 = dot3(c01, c01), n02 = dot3(c02, c02), n12 = dot3(c12, c12);
    double v[3];
    double nb = n01;
    v[0] = c01[0], v[1] = c01[1], v[2] = c01[2];
    if (n02 > nb) nb = n02, v[0] = c02[0], v[1] = c02[1], v[2] = c02[2];
    if (n12 > nb) nb = n12, v[0] = c12[0], v[1] = c12[1], v[2] = c12[2];
    double amax = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) amax = fmax(amax, fabs(A[i][j]));
    if (!(nb > 1e-56 * amax * amax * amax * amax)) {
        // all roots equal to working accuracy: any orthonormal basis
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            nu[i] = A[i][i];
#pragma unroll
            for (int k = 0; k < 3; ++k) q[i][k] = i == k ? 1.0 : 0.0;
        }
        return;
    }
    const double inv = 1.0 / sqrt(nb);
    v[0] *= inv, v[1] *= inv, v[2] *= inv;
    // orthonormal basis (a, b) of the plane orthogonal to v
    double ax[3] = {0.0, 0.0, 0.0};
    ax[fabs(v[0]) < 0.6 ? 0 : 1] = 1.0;
    double a[3], b[3];
    cross3(v, ax, a);
    const double ia = 1.0 / sqrt(dot3(a, a));
    a[0] *= ia, a[1] *= ia, a[2] *= ia;
    cross3(v, a, b);
    double Aa[3], Ab[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Aa[i] = A[i][0] * a[0] + A[i][1] * a[1] + A[i][2] * a[2];
        Ab[i] = A[i][0] * b[0] + A[i][1] * b[1] + A[i][2] * b[2];
    }
    const double saa = dot3(a, Aa), sab = dot3(a, Ab), sbb = dot3(b, Ab);
    // the rotation by theta = atan2(2 sab, saa - sbb) / 2 in (-pi/2, pi/2]
    // from its half-angle forms (cos 2 theta = d / rad, sin 2 theta = sab /
    // rad), each taken where it does not cancel: c = cos theta >= 0, and sn
    // has the sign of sab (of +pi/2 where sab = 0 and d < 0); rad = hypot(d,
    // sab) does not underflow where the two roots nearly coincide
    const double d = 0.5 * (saa - sbb);
    const double mid = 0.5 * (saa + sbb), rad = hypot(d, sab);
    double c = 1.0, sn = 0.0;
    if (rad > 0.0) {
        if (d >= 0.0) {
            c = sqrt((rad + d) / (2.0 * rad));
            sn = sab / (2.0 * rad * c);
        } else {
            sn = copysign(sqrt((rad - d) / (2.0 * rad)), sab);
            c = sab / (2.0 * rad * sn);
        }
    }
    const int kv = top ? 0 : 2, k1 = top ? 1 : 0, k2 = top ? 2 : 1;
    nu[kv] = lam;
    nu[k1] = mid + rad;
    nu[k2] = mid - rad;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        q[i][kv] = v[i];
        q[i][k1] = c * a[i] + sn * b[i];
        q[i][k2] = -sn * a[i] + c * b[i];
    }
}

// Eigenpairs (nu_k, e_k) of H_rho in FP64 and mu_k of Eq. (7) with the mode
// masks, stored as P = sum_k mu_k e_k e_k^T: 6 values per voxel ([m][6], the
// substep reads them together: xx, yy, zz, xy, xz, yz). The tensor's weights
// mu_k on e_k e_k^T and (mu_k + mu_l) / 2 on the symmetric pairs make its
// action on a symmetric h equal to (P h + h P) / 2, so P is all it needs.
__global__ __launch_bounds__(256) void eig3_kernel(const float *__restrict__ hr, float *__restrict__ tens, int mode,
                                                   double inv_lam2, int D, int H, int W)
{
    const Vox v = voxel(D, H, W);
    if (!v.inside) return;
    const size_t m = (size_t)D * H * W;
    const double hxx = hr[v.o], hyy = hr[m + v.o], hzz = hr[2 * m + v.o];
    const double hxy = hr[3 * m + v.o], hxz = hr[4 * m + v.o], hyz = hr[5 * m + v.o];
    float2 *p = (float2 *)(tens + 6 * v.o);   // 24 bytes per voxel, 8-byte aligned
    if (mode == MF4D_BOTH) {
        // Without the mode masks every mu_k is 1 / (1 + nu_k^2 / lambda^2), so
        // P = (I + H^2 / lambda^2)^-1: the inverse of a symmetric positive
        // definite M (eigenvalues >= 1), from its adjugate. The rounding of H^2
        // enters M amplified by 1 / lambda^2, an error of about
        // 1e-16 |H|^2 / lambda^2 in P; where that could exceed 1e-10 the
        // eigenpairs below are used instead.
        const double s = inv_lam2;
        const double f2 = hxx * hxx + hyy * hyy + hzz * hzz + 2.0 * (hxy * hxy + hxz * hxz + hyz * hyz);
        if (s * f2 <= 1e6) {
            const double m00 = 1.0 + s * (hxx * hxx + hxy * hxy + hxz * hxz);
            const double m11 = 1.0 + s * (hxy * hxy + hyy * hyy + hyz * hyz);
            const double m22 = 1.0 + s * (hxz * hxz + hyz * hyz + hzz * hzz);
            const double m01 = s * (hxx * hxy + hxy * hyy + hxz * hyz);
            const double m02 = s * (hxx * hxz + hxy * hyz + hxz * hzz);
            const double m12 = s * (hxy * hxz + hyy * hyz + hyz * hzz);
            const double c00 = m11 * m22 - m12 * m12, c11 = m00 * m22 - m02 * m02, c22 = m00 * m11 - m01 * m01;
            const double c01 = m02 * m12 - m01 * m22, c02 = m01 * m12 - m02 * m11, c12 = m01 * m02 - m00 * m12;
            const double id = 1.0 / (m00 * c00 + m01 * c01 + m02 * c02);
            p[0] = make_float2((float)(c00 * id), (float)(c11 * id));
            p[1] = make_float2((float)(c22 * id), (float)(c01 * id));
            p[2] = make_float2((float)(c02 * id), (float)(c12 * id));
            return;
        }
    }
    const double a[3][3] = {{hxx, hxy, hxz}, {hxy, hyy, hyz}, {hxz, hyz, hzz}};
    double nu[3], q[3][3];
    sym3_eigenpairs(a, nu, q);
    double mu[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double mk = 1.0 / (1.0 + nu[k] * nu[k] * inv_lam2);
        if (mode == MF4D_RIDGE && nu[k] >= 0.0) mk = 1.0;
        if (mode == MF4D_VALLEY && nu[k] <= 0.0) mk = 1.0;
        mu[k] = mk;
    }
    auto Pij = [&](int i, int j) { return mu[0] * q[i][0] * q[j][0] + mu[1] * q[i][1] * q[j][1] + mu[2] * q[i][2] * q[j][2]; };
    p[0] = make_float2((float)Pij(0, 0), (float)Pij(1, 1));
    p[1] = make_float2((float)Pij(2, 2), (float)Pij(0, 1));
    p[2] = make_float2((float)Pij(0, 2), (float)Pij(1, 2));
}

// ---------------------------------------------------------------- substep
// One FED substep u_out = u_in - tau L^T T, T = D h, fused: a workgroup owns
// a tile of 32 x 8 output columns (x, y) and marches along z over a segment
// of planes. For each output plane z it loads u plane z + 2 of the tile with
// a 2-voxel xy halo into an LDS ring of three planes, forms T of plane z + 1
// on the tile with a 1-voxel halo into a ring of three T planes (one thread
// per T position, its 6 tensor values loaded one plane ahead), and then
// gathers L^T T at plane z. T is D h at interior voxels and 0 elsewhere
// (also outside the volume), h the second differences of u (cross stencils
// for the mixed terms). D h = Q (M o (Q^T h Q)) Q^T with M_kk = mu_k and
// M_kl = (mu_k + mu_l) / 2; as M o G = (Lambda G + G Lambda) / 2 for any G,
// that is (P h + h P) / 2 with P = Q Lambda Q^T. Neighbouring tiles
// recompute their shared halo, so u_out must not alias u_in.
constexpr int kFX = 32, kFY = 8;                  // output tile
constexpr int kTX = kFX + 2, kTY = kFY + 2;       // T region
constexpr int kUX = kFX + 4, kUY = kFY + 4;       // u region
constexpr int kZSeg = 64;                         // planes per workgroup
constexpr int kFThreads = 384;                    // >= the T region's 340 positions

// T = D h = (P h + h P) / 2 for symmetric h and P (xx, yy, zz, xy, xz, yz)
__device__ __forceinline__ void tensor_action(const float (&h)[3][3], const float (&P)[6], float (&T)[6])
{
    const float p00 = P[0], p11 = P[1], p22 = P[2], p01 = P[3], p02 = P[4], p12 = P[5];
    const float h00 = h[0][0], h11 = h[1][1], h22 = h[2][2], h01 = h[0][1], h02 = h[0][2], h12 = h[1][2];
    T[0] = p00 * h00 + p01 * h01 + p02 * h02;
    T[1] = p01 * h01 + p11 * h11 + p12 * h12;
    T[2] = p02 * h02 + p12 * h12 + p22 * h22;
    T[3] = 0.5f * ((p00 * h01 + p01 * h11 + p02 * h12) + (p01 * h00 + p11 * h01 + p12 * h02));
    T[4] = 0.5f * ((p00 * h02 + p01 * h12 + p02 * h22) + (p02 * h00 + p12 * h01 + p22 * h02));
    T[5] = 0.5f * ((p01 * h02 + p11 * h12 + p12 * h22) + (p02 * h01 + p12 * h11 + p22 * h12));
}

__global__ __launch_bounds__(kFThreads) void fed3_kernel(const float *__restrict__ u, float *__restrict__ uo,
                                                   const float *__restrict__ tens, float tau, int D, int H, int W,
                                                   int tiles_x, int tiles_y)
{
    __shared__ float su[3][kUY][kUX];
    __shared__ float sT[3][6][kTY][kTX];
    const int tid = threadIdx.x;
    const int b = xcd_block();
    const int tx = b % tiles_x, ty = (b / tiles_x) % tiles_y, zs = b / (tiles_x * tiles_y);
    const int x0 = tx * kFX, y0 = ty * kFY, z0 = zs * kZSeg, z1 = min(D, z0 + kZSeg);
    const size_t plane = (size_t)H * W;
    auto slot = [](int z) { return (z + 3) % 3; };   // z >= -3
    // u of the u region, one plane ahead in registers: this thread's
    // positions (their in-plane offsets, clamped into the volume, and whether
    // they lie inside it) do not change with z. The loads are unconditional
    // and the zero outside the volume is applied only at the LDS store, so
    // nothing waits for them before then.
    constexpr int kUN = (kUY * kUX + kFThreads - 1) / kFThreads;
    size_t uoff[kUN];
    bool uin[kUN];
#pragma unroll
    for (int k = 0; k < kUN; ++k) {
        const int i = min(tid + k * kFThreads, kUY * kUX - 1);
        const int ly = i / kUX, lx = i - ly * kUX;
        const int gx = x0 - 2 + lx, gy = y0 - 2 + ly;
        uin[k] = tid + k * kFThreads < kUY * kUX && gx >= 0 && gx < W && gy >= 0 && gy < H;
        uoff[k] = (size_t)min(max(gy, 0), H - 1) * W + min(max(gx, 0), W - 1);
    }
    float pu[kUN];
    auto fetch_u = [&](int z) {
        const size_t zo = (size_t)min(max(z, 0), D - 1) * plane;
#pragma unroll
        for (int k = 0; k < kUN; ++k) pu[k] = u[zo + uoff[k]];
    };
    auto store_u = [&](int z) {   // u plane z of the u region (0 outside the volume)
        const bool zin = z >= 0 && z < D;
        float *sp = &su[slot(z)][0][0];
#pragma unroll
        for (int k = 0; k < kUN; ++k)
            if (tid + k * kFThreads < kUY * kUX) sp[tid + k * kFThreads] = zin && uin[k] ? pu[k] : 0.f;
    };
    auto load_u = [&](int z) {
        fetch_u(z);
        store_u(z);
    };
    // this thread's T position and its tensor values at plane z (loaded from
    // voxel 0 where T is 0: make_T does not use them there)
    const int tly = tid / kTX, tlx = tid - tly * kTX;
    const int tgx = x0 - 1 + tlx, tgy = y0 - 1 + tly;
    const bool tpos = tid < kTY * kTX;
    auto load_tens = [&](int z, float (&tq)[6]) {
        const bool in = tpos && z >= 1 && z <= D - 2 && tgx >= 1 && tgx <= W - 2 && tgy >= 1 && tgy <= H - 2;
        const size_t o = in ? (size_t)z * plane + (size_t)tgy * W + tgx : 0;
        const float2 *p = (const float2 *)(tens + 6 * o);   // 24 bytes per voxel, 8-byte aligned
        const float2 a = p[0], b = p[1], c = p[2];
        tq[0] = a.x, tq[1] = a.y, tq[2] = b.x, tq[3] = b.y, tq[4] = c.x, tq[5] = c.y;
    };
    // T plane z of the T region from u planes z - 1 .. z + 1 in the ring
    auto make_T = [&](int z, const float (&tq)[6]) {
        const int s0 = slot(z - 1), s1 = slot(z), s2 = slot(z + 1), st = slot(z);
        if (tpos) {
            const int ly = tly, lx = tlx;
            const int gx = tgx, gy = tgy;
            float T[6] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (z >= 1 && z <= D - 2 && gx >= 1 && gx <= W - 2 && gy >= 1 && gy <= H - 2) {
                const int ux = lx + 1, uy = ly + 1;   // the voxel in the u region
                const float c2 = 2.f * su[s1][uy][ux];
                float h[3][3];
                h[0][0] = su[s1][uy][ux - 1] - c2 + su[s1][uy][ux + 1];
                h[1][1] = su[s1][uy - 1][ux] - c2 + su[s1][uy + 1][ux];
                h[2][2] = su[s0][uy][ux] - c2 + su[s2][uy][ux];
                h[0][1] = 0.25f * ((su[s1][uy - 1][ux - 1] + su[s1][uy + 1][ux + 1]) -
                                   (su[s1][uy + 1][ux - 1] + su[s1][uy - 1][ux + 1]));
                h[0][2] = 0.25f * ((su[s0][uy][ux - 1] + su[s2][uy][ux + 1]) - (su[s2][uy][ux - 1] + su[s0][uy][ux + 1]));
                h[1][2] = 0.25f * ((su[s0][uy - 1][ux] + su[s2][uy + 1][ux]) - (su[s2][uy - 1][ux] + su[s0][uy + 1][ux]));
                h[1][0] = h[0][1];
                h[2][0] = h[0][2];
                h[2][1] = h[1][2];
                tensor_action(h, tq, T);
            }
#pragma unroll
            for (int k = 0; k < 6; ++k) sT[st][k][ly][lx] = T[k];
        }
    };
    // prologue: T of planes z0 - 1 and z0
    float tq[6];
    load_tens(z0 - 1, tq);
    load_u(z0 - 2);
    load_u(z0 - 1);
    load_u(z0);
    __syncthreads();
    make_T(z0 - 1, tq);
    load_tens(z0, tq);
    __syncthreads();
    load_u(z0 + 1);   // into the slot of plane z0 - 2
    __syncthreads();
    make_T(z0, tq);
    load_tens(z0 + 1, tq);
    fetch_u(z0 + 2);
    const bool out = tid < kFX * kFY;
    const int ox = tid % kFX, oy = out ? tid / kFX : 0;   // this thread's output column
    const int gx = x0 + ox, gy = y0 + oy;
    const int lx = ox + 1, ly = oy + 1;         // in the T region
    for (int z = z0; z < z1; ++z) {
        __syncthreads();   // the previous plane's gather has read the ring slots reused below
        store_u(z + 2);    // into the slot of plane z - 1
        fetch_u(z + 3);    // in flight during make_T and the gather
        __syncthreads();
        make_T(z + 1, tq); // into the slot of plane z - 2
        load_tens(z + 2, tq);   // in flight during the gather and the next plane's u load
        __syncthreads();
        if (out && gx < W && gy < H) {
            const int tm = slot(z - 1), t0 = slot(z), tp = slot(z + 1);
            float r = (sT[t0][0][ly][lx - 1] + sT[t0][0][ly][lx + 1]) - 2.f * sT[t0][0][ly][lx];
            r += (sT[t0][1][ly - 1][lx] + sT[t0][1][ly + 1][lx]) - 2.f * sT[t0][1][ly][lx];
            r += (sT[tm][2][ly][lx] + sT[tp][2][ly][lx]) - 2.f * sT[t0][2][ly][lx];
            r += 0.5f * ((sT[t0][3][ly - 1][lx - 1] + sT[t0][3][ly + 1][lx + 1]) -
                         (sT[t0][3][ly + 1][lx - 1] + sT[t0][3][ly - 1][lx + 1]));
            r += 0.5f * ((sT[tm][4][ly][lx - 1] + sT[tp][4][ly][lx + 1]) - (sT[tp][4][ly][lx - 1] + sT[tm][4][ly][lx + 1]));
            r += 0.5f * ((sT[tm][5][ly - 1][lx] + sT[tp][5][ly + 1][lx]) - (sT[tp][5][ly - 1][lx] + sT[tm][5][ly + 1][lx]));
            const size_t o = (size_t)z * plane + (size_t)gy * W + gx;
            uo[o] = su[slot(z)][oy + 2][ox + 2] - tau * r;
        }
    }
}

// ------------------------------------------------------------------ host
dim3 grid3(int D, int H, int W) { return dim3((W + kBX - 1) / kBX, (H + kBY - 1) / kBY, D); }
const dim3 kBlock3(kBX, kBY, 1);

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

bool aligned8(const void *p) { return ((uintptr_t)p & 7) == 0; }

bool valid_dims(int D, int H, int W)
{
    if (D < 3 || H < 3 || W < 3 || D > 65535) return false;
    return (long long)D * H * W < (1LL << 31);
}

// Parameter checks of the 2-D filter, then the 3-D restrictions.
int validate3(int D, int H, int W, const mf4d_params *p)
{
    if (!valid_dims(D, H, W) || !p) return MF4D_EINVAL;
    int st = validate_params(3, 3, p);   // the fields of p (the image size is checked above)
    if (st != MF4D_OK) return st;
    if (p->tau_max > kTauLimit3) return MF4D_EINVAL;
    if (p->model != MF4D_MAFOD || p->postprocess != 0 || p->check != 0 || p->reselect_each_cycle != 1)
        return MF4D_EINVAL;
    return MF4D_OK;
}

struct Work3 {
    float *X, *Y;        // planes of the z pass [3][m] and the y pass [6][m]
    float2 *SF;          // [ns][m]
    float *N;            // [ns][6][m]
    uint8_t *idx;
    float *G1, *G2;      // [6][m] each: gathered N and the blur's ping-pong
    float *hrho;         // [6][m]
    float *tens;         // [m][6]: P
    float *utmp;         // [m]: the substeps' ping-pong image
    unsigned *smax;
};

size_t layout3(int D, int H, int W, int ns, Work3 *w, char *base)
{
    const size_t m = (size_t)D * H * W;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *q = base ? base + off : nullptr;
        off += align256(bytes);
        return q;
    };
    Work3 t;
    t.X = (float *)take(3 * m * 4);
    t.Y = (float *)take(6 * m * 4);
    t.SF = (float2 *)take((size_t)ns * m * 8);
    t.N = (float *)take((size_t)ns * 6 * m * 4);
    t.idx = (uint8_t *)take(m);
    t.G1 = (float *)take(6 * m * 4);
    t.G2 = (float *)take(6 * m * 4);
    t.hrho = (float *)take(6 * m * 4);
    t.tens = (float *)take(6 * m * 4);
    t.utmp = (float *)take(m * 4);
    t.smax = (unsigned *)take(256);
    if (w) *w = t;
    return off;
}

#define CHECK_HIP(expr)                         \
    do {                                        \
        hipError_t e_ = (expr);                 \
        if (e_ != hipSuccess) return MF4D_EHIP; \
    } while (0)
#define CHECK_LAUNCH() CHECK_HIP(hipGetLastError())

// All scales: S, F and N per scale, and the largest S (cleared first).
int sweep3(const float *u, int D, int H, int W, const mf4d_params *p, const Work3 &w, hipStream_t s)
{
    const size_t m = (size_t)D * H * W;
    const dim3 g = grid3(D, H, W);
    // z and y passes: kLW outputs per thread along the pass
    const dim3 gz((W + kBX - 1) / kBX, (H + kBY - 1) / kBY, (D + kLW - 1) / kLW);
    const dim3 gy((W + kBX - 1) / kBX, ((H + kLW - 1) / kLW + kBY - 1) / kBY, D);
    CHECK_HIP(launch_fill_u32(w.smax, 0u, 1, s));
    const double inv2beta2 = 1.0 / (2.0 * (double)p->beta * (double)p->beta);
    for (int k = 0; k < p->nscales; ++k) {
        WinTaps t;
        window_taps(p->sigmas[k], &t);
        const float sigma2 = p->sigmas[k] * p->sigmas[k];
        sweep3_z_kernel<<<gz, kBlock3, 0, s>>>(u, w.X, D, H, W, t);
        CHECK_LAUNCH();
        sweep3_y_kernel<<<gy, kBlock3, 0, s>>>(w.X, w.Y, D, H, W, t);
        CHECK_LAUNCH();
        const size_t lds = sizeof(float) * 6 * kBY * (kBX + 2 * t.R);
        sweep3_x_kernel<<<g, kBlock3, lds, s>>>(w.Y, w.SF + k * m, w.N + (size_t)k * 6 * m, w.smax, D, H, W, t,
                                                sigma2, p->mode, inv2beta2);
        CHECK_LAUNCH();
    }
    return MF4D_OK;
}

// H_rho from N at the chosen scales; then (optionally) the tensor planes.
int integrate3(int D, int H, int W, const mf4d_params *p, const uint8_t *idx, const Work3 &w, float *hrho,
               float *tens, hipStream_t s)
{
    const dim3 g = grid3(D, H, W);
    RhoTaps rt;
    rho_taps(p->rho, &rt);
    if (rt.r <= 2) {   // one fused kernel (the same values as the passes below)
        const int tiles_x = (W + kIX - 1) / kIX, tiles_y = (H + kIY - 1) / kIY, segs = (D + kIZSeg - 1) / kIZSeg;
        const dim3 gi(tiles_x * tiles_y * segs);
        switch (rt.r) {
        case 0: integrate3_kernel<0><<<gi, kIX * kIY, 0, s>>>(w.N, idx, p->nscales, hrho, D, H, W, rt, tiles_x, tiles_y); break;
        case 1: integrate3_kernel<1><<<gi, kIX * kIY, 0, s>>>(w.N, idx, p->nscales, hrho, D, H, W, rt, tiles_x, tiles_y); break;
        default: integrate3_kernel<2><<<gi, kIX * kIY, 0, s>>>(w.N, idx, p->nscales, hrho, D, H, W, rt, tiles_x, tiles_y); break;
        }
        CHECK_LAUNCH();
    } else {
        gather3_kernel<<<g, kBlock3, 0, s>>>(w.N, idx, p->nscales, w.G1, D, H, W);
        CHECK_LAUNCH();
        rho3_kernel<0><<<g, kBlock3, 0, s>>>(w.G1, w.G2, D, H, W, rt);
        CHECK_LAUNCH();
        rho3_kernel<1><<<g, kBlock3, 0, s>>>(w.G2, w.G1, D, H, W, rt);
        CHECK_LAUNCH();
        rho3_kernel<2><<<g, kBlock3, 0, s>>>(w.G1, hrho, D, H, W, rt);
        CHECK_LAUNCH();
    }
    if (tens) {
        const double inv_lam2 = 1.0 / ((double)p->lambda * (double)p->lambda);
        eig3_kernel<<<g, kBlock3, 0, s>>>(hrho, tens, p->mode, inv_lam2, D, H, W);
        CHECK_LAUNCH();
    }
    return MF4D_OK;
}

// n substeps from u back into u, ping-ponging through tmp (one plane of
// the T scratch); an odd count ends with a copy back.
int substeps3(float *u, int D, int H, int W, const float *tens, const float *taus32, int n, float *tmp, hipStream_t s)
{
    const int tiles_x = (W + kFX - 1) / kFX, tiles_y = (H + kFY - 1) / kFY, segs = (D + kZSeg - 1) / kZSeg;
    const dim3 grid(tiles_x * tiles_y * segs);
    float *src = u, *dst = tmp;
    for (int i = 0; i < n; ++i) {
        fed3_kernel<<<grid, kFThreads, 0, s>>>(src, dst, tens, taus32[i], D, H, W, tiles_x, tiles_y);
        CHECK_LAUNCH();
        float *t = src;
        src = dst;
        dst = t;
    }
    if (src != u) CHECK_HIP(launch_copy_f32(src, u, (size_t)D * H * W, s));
    return MF4D_OK;
}

}  // namespace

extern "C" {

size_t mf4d3d_workspace_bytes(int D, int H, int W, const mf4d_params *p)
{
    if (validate3(D, H, W, p) != MF4D_OK) return 0;
    return layout3(D, H, W, p->nscales, nullptr, nullptr);
}

int mf4d3d_scale_select(const float *u, int D, int H, int W, const mf4d_params *p, uint8_t *idx_out,
                        float *vmax_out, float *c_out, void *ws, size_t ws_bytes, void *stream)
{
    int st = validate3(D, H, W, p);
    if (st != MF4D_OK) return st;
    if (!u || !idx_out || !ws) return MF4D_EINVAL;
    if (ws_bytes < layout3(D, H, W, p->nscales, nullptr, nullptr)) return MF4D_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    Work3 w;
    layout3(D, H, W, p->nscales, &w, (char *)ws);
    st = sweep3(u, D, H, W, p, w, s);
    if (st != MF4D_OK) return st;
    argmax3_kernel<<<grid3(D, H, W), kBlock3, 0, s>>>(w.SF, p->nscales, w.smax, p->c, idx_out, vmax_out, c_out, D, H,
                                                      W);
    CHECK_LAUNCH();
    return MF4D_OK;
}

int mf4d3d_tensor(const float *u, int D, int H, int W, const uint8_t *idx, const mf4d_params *p, float *hrho_out,
                  float *dparams_out, void *ws, size_t ws_bytes, void *stream)
{
    int st = validate3(D, H, W, p);
    if (st != MF4D_OK) return st;
    if (!u || !idx || !hrho_out || !ws || (dparams_out && !aligned8(dparams_out))) return MF4D_EINVAL;
    if (ws_bytes < layout3(D, H, W, p->nscales, nullptr, nullptr)) return MF4D_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    Work3 w;
    layout3(D, H, W, p->nscales, &w, (char *)ws);
    st = sweep3(u, D, H, W, p, w, s);
    if (st != MF4D_OK) return st;
    return integrate3(D, H, W, p, idx, w, hrho_out, dparams_out, s);
}

int mf4d3d_dtensor(const float *hrho, int D, int H, int W, const mf4d_params *p, float *dparams_out, void *stream)
{
    int st = validate3(D, H, W, p);
    if (st != MF4D_OK) return st;
    if (!hrho || !dparams_out || !aligned8(dparams_out)) return MF4D_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const double inv_lam2 = 1.0 / ((double)p->lambda * (double)p->lambda);
    eig3_kernel<<<grid3(D, H, W), kBlock3, 0, s>>>(hrho, dparams_out, p->mode, inv_lam2, D, H, W);
    CHECK_LAUNCH();
    return MF4D_OK;
}

int mf4d3d_fed_cycle_tensor(float *u, float *u_tmp, int D, int H, int W, const float *dparams, const double *taus,
                            int n, void *stream)
{
    if (!valid_dims(D, H, W) || !u || !u_tmp || u == u_tmp || !dparams || !aligned8(dparams) || !taus || n < 1 ||
        n > MF4D_MAX_SUBSTEPS)
        return MF4D_EINVAL;
    for (int i = 0; i < n; ++i)
        if (!(taus[i] > 0.0) || !std::isfinite(taus[i])) return MF4D_EINVAL;
    std::vector<float> t32(n);
    for (int i = 0; i < n; ++i) t32[i] = (float)taus[i];
    return substeps3(u, D, H, W, dparams, t32.data(), n, u_tmp, (hipStream_t)stream);
}

int mf4d3d_filter(const float *u_in, float *u_out, int D, int H, int W, const mf4d_params *p, void *ws,
                  size_t ws_bytes, void *stream)
{
    int st = validate3(D, H, W, p);
    if (st != MF4D_OK) return st;
    if (!u_in || !u_out || !ws) return MF4D_EINVAL;
    if (ws_bytes < layout3(D, H, W, p->nscales, nullptr, nullptr)) return MF4D_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    const size_t m = (size_t)D * H * W;
    Work3 w;
    layout3(D, H, W, p->nscales, &w, (char *)ws);
    if (u_in != u_out) CHECK_HIP(launch_copy_f32(u_in, u_out, m, s));
    if (p->cycles == 0) return MF4D_OK;
    std::vector<double> ordered;
    int n = 0;
    st = fed_plan_host(p, &n, ordered);
    if (st != MF4D_OK) return st;
    std::vector<float> t32(n);
    for (int i = 0; i < n; ++i) t32[i] = (float)ordered[i];
    const dim3 g = grid3(D, H, W);
    for (int k = 0; k < p->cycles; ++k) {
        st = sweep3(u_out, D, H, W, p, w, s);
        if (st != MF4D_OK) return st;
        argmax3_kernel<<<g, kBlock3, 0, s>>>(w.SF, p->nscales, w.smax, p->c, w.idx, nullptr, nullptr, D, H, W);
        CHECK_LAUNCH();
        st = integrate3(D, H, W, p, w.idx, w, w.hrho, w.tens, s);
        if (st != MF4D_OK) return st;
        st = substeps3(u_out, D, H, W, w.tens, t32.data(), n, w.utmp, s);
        if (st != MF4D_OK) return st;
    }
    return MF4D_OK;
}

}  // extern "C"
