// Wave-level device code of the row-streaming FED substep kernel, shared by
// the single-image and the batched launches.
#pragma once

#include "mf4d_internal.h"

namespace mf4d {
namespace tiles {

// ------------------------------------------------------------ row streaming
// fed_stream_kernel<S>: S consecutive substeps per launch without LDS or
// barriers. A wave owns 64 adjacent columns (lane = column) and walks down a
// segment of rows; every intermediate quantity lives in per-lane register
// rings indexed by row, and x-neighbours come from lane shifts. Each level
// of the substep pipeline (flux T_k, then u_k) lags the previous one by one
// row and spoils one more lane at each wave edge, so a wave owns 64 - 4 S
// output columns and reads u and the tensor planes with a 2 S lane and 2 S
// row halo.
//
// With D(x) = T_xy(p-1, x) - T_xy(p+1, x) the divergence at row p is
//   r = [T_xx(p) + D/2](x-1) + [T_xx(p) - D/2](x+1) - 2 T_xx(p)(x)
//       + T_yy(p-1) - 2 T_yy(p) + T_yy(p+1),
// i.e. L_xx^T T_xx + 2 L_xy^T T_xy + L_yy^T T_yy with two lane shifts.

// lane i receives the value of lane i - 1 (x - 1) / lane i + 1 (x + 1); the
// wave's edge lanes receive 0, which only ever reaches halo lanes.
__device__ __forceinline__ float from_left(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_right(float v)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}

typedef float nt_f2 __attribute__((ext_vector_type(2)));   // 8-byte nontemporal loads
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Raw buffer resource over n floats at p (n < 2^29): a load or store through
// it takes the lane's byte offset as a vector operand and the row's as a
// scalar one, so no per-lane address arithmetic is spent on a row. The third
// descriptor word is the one of the gfx9 family (untyped 32-bit data).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const float *p, size_t n)
{
    return __builtin_amdgcn_make_buffer_rsrc((void *)p, (short)0, (int)(n * 4), 0x00020000);
}
constexpr int kBufNontemporal = 2;   // cache-policy bit of a buffer access: nontemporal

// v where m is all ones, +0 where m is 0 (a bitwise select the compiler
// cannot turn into a branch; for finite v the same values as a conditional)
__device__ __forceinline__ float keep(float v, unsigned m) { return __uint_as_float(__float_as_uint(v) & m); }
__device__ __forceinline__ unsigned mask_of(bool b) { return b ? 0xffffffffu : 0u; }

template <int S>
__device__ __forceinline__ void fed_stream_wave(const float *__restrict__ u, float *__restrict__ uo,
                                                const float *__restrict__ coef, int H, int W, const FedTaus &taus,
                                                int strip, int seg, int seg_rows)
{
#pragma clang fp contract(off)   // fused multiply-adds are written out: every launch shape rounds alike
    constexpr int HALO = 2 * S;
    constexpr int OUTW = 64 - 2 * HALO;
    constexpr int D = 8;                                  // rows loaded ahead
    constexpr int NC = 2 * S;                             // tensor rows kept
    constexpr int U = kStreamUnroll;                      // unroll: multiple of 3, NC and D
    const int lane = threadIdx.x & 63;
    const int x = strip * OUTW - HALO + lane;
    const int ys = seg * seg_rows;
    const int ye = min(ys + seg_rows, H);
    const bool xin = x >= 0 && x < W;
    const bool xint = x >= 1 && x <= W - 2;
    const bool store = lane >= HALO && lane < 64 - HALO && x < W;
    const size_t plane = (size_t)H * W;
    const int xc = min(max(x, 0), W - 1);

    float uL[S][3], uC[S][3], uR[S][3];   // u_k rows, k < S: left / centre / right
    float txx[S][3], txy[S][3], tyy[S][3];   // T_k rows, k = 1..S
    float cm[NC], ca[NC], cb[NC];         // tensor planes of the last NC rows
    float qu[D], qm[D], qa[D], qb[D];     // rows in flight
#pragma unroll
    for (int k = 0; k < S; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            uL[k][j] = uC[k][j] = uR[k][j] = txx[k][j] = txy[k][j] = tyy[k][j] = 0.f;
#pragma unroll
    for (int j = 0; j < NC; ++j) cm[j] = ca[j] = cb[j] = 0.f;

    const int y0 = ys - HALO;           // first row loaded
    const int y1 = ye + HALO;           // one past the last row needed
    // rows are loaded from a clamped address and masked when consumed
    auto issue = [&](int y, float &vu, float &vm, float &va, float &vb) {
        const size_t o = (size_t)min(max(y, 0), H - 1) * W + xc;
        vu = __builtin_nontemporal_load(u + o);   // the launch's input image is read here for the last time
        vm = coef[o];
        va = coef[plane + o];
        vb = coef[2 * plane + o];
    };
#pragma unroll
    for (int d = 0; d < D; ++d) issue(y0 + d, qu[d], qm[d], qa[d], qb[d]);

    for (int yb = y0; yb < y1; yb += U) {
#pragma clang loop unroll(full)
        for (int t = 0; t < U; ++t) {
            const int y = yb + t;
            // arrival of row y of u_0 and of the tensor planes
            const int qs = t % D;
            const float nu = keep(qu[qs], mask_of(xin && y >= 0 && y < H));
            // zero tensor off the interior: the flux T = D h vanishes there
            const unsigned on = mask_of(xint && y >= 1 && y <= H - 2);
            cm[t % NC] = keep(qm[qs], on);
            ca[t % NC] = keep(qa[qs], on);
            cb[t % NC] = keep(qb[qs], on);
            issue(y + D, qu[qs], qm[qs], qa[qs], qb[qs]);
            {
                const int w0 = t % 3;
                uC[0][w0] = nu;
                uL[0][w0] = from_left(nu);
                uR[0][w0] = from_right(nu);
            }
#pragma unroll
            for (int k = 1; k <= S; ++k) {
                // flux T_k at row q = y - (2k - 1) from u_{k-1} rows q-1, q, q+1
                const int wn = (t - 2 * (k - 1) + 300) % 3;        // u_{k-1} row q+1
                const int wc = (t - 2 * (k - 1) - 1 + 300) % 3;    // row q
                const int wo = (t - 2 * (k - 1) - 2 + 300) % 3;    // row q-1
                const int ci = (t - (2 * k - 1) + 2 * NC * 50) % NC;
                const float v = uC[k - 1][wc];
                const float hxx = fmaf(-2.f, v, uL[k - 1][wc] + uR[k - 1][wc]);
                const float hyy = fmaf(-2.f, v, uC[k - 1][wo] + uC[k - 1][wn]);
                const float hxy = 0.25f * ((uL[k - 1][wo] + uR[k - 1][wn]) - (uL[k - 1][wn] + uR[k - 1][wo]));
                const float mb = cm[ci], al = ca[ci], be = cb[ci];
                const int tw = (t - (2 * k - 1) + 300) % 3;
                const float bxy = be * hxy;
                txx[k - 1][tw] = fmaf(mb + al, hxx, bxy);
                txy[k - 1][tw] = fmaf(mb, hxy, (be * 0.5f) * (hxx + hyy));
                tyy[k - 1][tw] = fmaf(mb - al, hyy, bxy);
                // u_k at row p = y - 2k from T_k rows p-1, p, p+1 and u_{k-1} row p
                const int p = y - 2 * k;
                const int sn = tw;                            // T_k row p+1
                const int sc = (t - 2 * k + 300) % 3;         // row p
                const int so = (t - 2 * k - 1 + 300) % 3;     // row p-1
                const float dxy = txy[k - 1][so] - txy[k - 1][sn];
                const float el = fmaf(0.5f, dxy, txx[k - 1][sc]);
                const float er = fmaf(-0.5f, dxy, txx[k - 1][sc]);
                const float rx = fmaf(-2.f, txx[k - 1][sc], from_left(el) + from_right(er));
                const float ry = fmaf(-2.f, tyy[k - 1][sc], tyy[k - 1][so] + tyy[k - 1][sn]);
                const float r = rx + ry;
                const float nv = fmaf(-taus.t[k - 1], r, uC[k - 1][(t - 2 * k + 300) % 3]);
                if (k < S) {
                    const int w = (t - 2 * k + 300) % 3;
                    uC[k][w] = nv;
                    uL[k][w] = from_left(nv);
                    uR[k][w] = from_right(nv);
                } else if (store && p >= ys && p < ye) {
                    uo[(size_t)p * W + x] = nv;
                }
            }
        }
    }
}


// fed_stream_wave2<S>: the same S substeps with two adjacent columns per
// lane (lane l owns columns 2l and 2l+1 of a 128-column strip), so a wave
// owns 128 - 4 S output columns. Each column's neighbour inside the lane is
// a register; only the outer neighbours cross lanes, which halves the lane
// shifts per pixel and the share of halo columns. Every column runs the
// arithmetic of fed_stream_wave in the same order, so both forms give the
// same values bit for bit.
// Odd segments walk their rows upwards (up = true). The 2 S halo rows two
// neighbouring segments share are then read by both at about the same time
// (both at the end of their walks, or both at the start), so the second read
// finds them in the L2 cache instead of HBM. Walking up, the ring slots of the
// older and newer rows hold rows p + 1 and p - 1 instead of p - 1 and p + 1:
// the sums over the two are unchanged (addition commutes) and the two
// differences (the cross derivative, and T_xy(p - 1) - T_xy(p + 1)) change
// sign exactly, which the direction-signed factors (+-1/4, +-1/2) undo
// exactly. Both directions therefore give the same values (an exact zero may
// differ in sign).
// PAIR: the strip lies inside the image, W is even, the planes are 8-byte
// aligned and hold fewer than 2^29 pixels, so each lane loads and stores its
// two columns as one 8-byte buffer access (the same values as two 4-byte
// accesses), addressed as the row's offset (scalar) plus the lane's.
// INNER (with PAIR): every column of the strip and every row the segment
// loads is an interior pixel, so no value needs masking: the masks of the
// general form are all ones there, and skipping them gives the same bits.
template <int S, bool PAIR, bool INNER>
__device__ __forceinline__ void fed_stream_wave2_body(const float *__restrict__ u, float *__restrict__ uo,
                                                      const float *__restrict__ coef, int H, int W,
                                                      const FedTaus &taus, int strip, int seg, int seg_rows,
                                                      bool up)
{
#pragma clang fp contract(off)   // fused multiply-adds are written out: every launch shape rounds alike
    constexpr int HALO = 2 * S;                           // columns
    constexpr int OUTW = 128 - 2 * HALO;
    constexpr int D = 4;                                  // rows loaded ahead
    constexpr int NC = 2 * S;                             // tensor rows kept
    constexpr int U = kStreamUnroll;                      // unroll: multiple of 3, NC and D
    const int lane = threadIdx.x & 63;
    const int xa = strip * OUTW - HALO + 2 * lane, xb = xa + 1;
    const int ys = seg * seg_rows;
    const int ye = min(ys + seg_rows, H);
    const bool ina = xa >= 0 && xa < W, inb = xb >= 0 && xb < W;
    const bool inta = xa >= 1 && xa <= W - 2, intb = xb >= 1 && xb <= W - 2;
    const bool own = lane >= S && lane < 64 - S;          // both columns are outputs of this strip
    const bool sta = own && xa < W, stb = own && xb < W;
    const size_t plane = (size_t)H * W;
    const int xca = min(max(xa, 0), W - 1), xcb = min(max(xb, 0), W - 1);

    // u_k rows, k < S, of column a and column b; the outer neighbours (column
    // b of the lane to the left, column a of the lane to the right) are lane
    // shifts taken where they are used, which the compiler folds into the adds
    float ua[S][3], ub[S][3];
    float txa[S][3], tya[S][3], tza[S][3];   // T_k rows (xx, xy, yy), column a
    float txb[S][3], tyb[S][3], tzb[S][3];   // column b
    // tensor rows: m, be and the sums m + al, m - al and be / 2 the flux uses,
    // formed once per pixel (the same roundings as forming them per substep)
    float cma[NC], cea[NC], cpa[NC], cqa[NC], cha[NC];
    float cmb[NC], ceb[NC], cpb[NC], cqb[NC], chb[NC];
    float qa0[D], qa1[D], qa2[D], qa3[D], qb0[D], qb1[D], qb2[D], qb3[D];   // rows in flight
#pragma unroll
    for (int k = 0; k < S; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            ua[k][j] = ub[k][j] = 0.f;
            txa[k][j] = tya[k][j] = tza[k][j] = txb[k][j] = tyb[k][j] = tzb[k][j] = 0.f;
        }
#pragma unroll
    for (int j = 0; j < NC; ++j)
        cma[j] = cea[j] = cpa[j] = cqa[j] = cha[j] = cmb[j] = ceb[j] = cpb[j] = cqb[j] = chb[j] = 0.f;

    const int y0 = ys - 2 * S;          // first row needed
    const int y1 = ye + 2 * S;          // one past the last row needed
    const int dir = up ? -1 : 1;        // row step of the walk
    const int yfirst = up ? y1 - 1 : y0;
    const float q4 = up ? -0.25f : 0.25f, h2 = up ? -0.5f : 0.5f;
    const unsigned lbyte = 4u * (unsigned)xa;   // PAIR: 0 <= xa < W
    __amdgpu_buffer_rsrc_t bu, bm, ba, be, bo;
    if (PAIR) {
        bu = plane_rsrc(u, plane);
        bm = plane_rsrc(coef, plane);
        ba = plane_rsrc(coef + plane, plane);
        be = plane_rsrc(coef + 2 * plane, plane);
        bo = plane_rsrc(uo, plane);
    }
    auto issue = [&](int y, int d) {
        const size_t r = (size_t)min(max(y, 0), H - 1) * W;
        if (PAIR) {
            const unsigned rb = 4u * (unsigned)r;   // r < 2^29
            // the launch's input image is read here for the last time (the
            // tensor planes are read again by the cycle's later launches)
            const u32x2 v0 = __builtin_amdgcn_raw_buffer_load_b64(bu, lbyte, rb, kBufNontemporal);
            const u32x2 v1 = __builtin_amdgcn_raw_buffer_load_b64(bm, lbyte, rb, 0);
            const u32x2 v2 = __builtin_amdgcn_raw_buffer_load_b64(ba, lbyte, rb, 0);
            const u32x2 v3 = __builtin_amdgcn_raw_buffer_load_b64(be, lbyte, rb, 0);
            qa0[d] = __uint_as_float(v0.x);
            qb0[d] = __uint_as_float(v0.y);
            qa1[d] = __uint_as_float(v1.x);
            qb1[d] = __uint_as_float(v1.y);
            qa2[d] = __uint_as_float(v2.x);
            qb2[d] = __uint_as_float(v2.y);
            qa3[d] = __uint_as_float(v3.x);
            qb3[d] = __uint_as_float(v3.y);
        } else {
            const size_t oa = r + xca, ob = r + xcb;
            qa0[d] = __builtin_nontemporal_load(u + oa);
            qb0[d] = __builtin_nontemporal_load(u + ob);
            qa1[d] = coef[oa];
            qb1[d] = coef[ob];
            qa2[d] = coef[plane + oa];
            qb2[d] = coef[plane + ob];
            qa3[d] = coef[2 * plane + oa];
            qb3[d] = coef[2 * plane + ob];
        }
    };
#pragma unroll
    for (int d = 0; d < D; ++d) issue(yfirst + dir * d, d);

    // flux of one column from its u_{k-1} rows: the sums of the left and
    // right neighbours of the old, centre and new rows (lco, lcn, lcc: left
    // old + right new, left new + right old, left + right of the centre row),
    // the centre column's old, centre and new values, and the tensor
    auto flux = [&](float lorn, float lnro, float lcrc, float co, float cc, float cn, float mb, float be,
                    float mpa, float mma, float beh, float &txx, float &txy, float &tyy) {
#pragma clang fp contract(off)
        const float hxx = fmaf(-2.f, cc, lcrc);
        const float hyy = fmaf(-2.f, cc, co + cn);
        const float hxy = q4 * (lorn - lnro);
        const float bxy = be * hxy;
        txx = fmaf(mpa, hxx, bxy);
        txy = fmaf(mb, hxy, beh * (hxx + hyy));
        tyy = fmaf(mma, hyy, bxy);
    };

    for (int sb = 0; sb < y1 - y0; sb += U) {
#pragma clang loop unroll(full)
        for (int t = 0; t < U; ++t) {
            const int y = yfirst + dir * (sb + t);
            const int qs = t % D;
            const bool yin = y >= 0 && y < H;
            const float na = INNER ? qa0[qs] : keep(qa0[qs], mask_of(ina && yin));
            const float nb = INNER ? qb0[qs] : keep(qb0[qs], mask_of(inb && yin));
            // zero tensor off the interior: the flux T = D h vanishes there
            const bool yint = y >= 1 && y <= H - 2;
            const unsigned ona = mask_of(inta && yint), onb = mask_of(intb && yint);
            {
                const int ci = t % NC;
                const float ma = INNER ? qa1[qs] : keep(qa1[qs], ona);
                const float aa = INNER ? qa2[qs] : keep(qa2[qs], ona);
                const float ea = INNER ? qa3[qs] : keep(qa3[qs], ona);
                const float mb = INNER ? qb1[qs] : keep(qb1[qs], onb);
                const float ab = INNER ? qb2[qs] : keep(qb2[qs], onb);
                const float eb = INNER ? qb3[qs] : keep(qb3[qs], onb);
                cma[ci] = ma;
                cea[ci] = ea;
                cpa[ci] = ma + aa;
                cqa[ci] = ma - aa;
                cha[ci] = ea * 0.5f;
                cmb[ci] = mb;
                ceb[ci] = eb;
                cpb[ci] = mb + ab;
                cqb[ci] = mb - ab;
                chb[ci] = eb * 0.5f;
            }
            issue(y + dir * D, qs);
            {
                const int w0 = t % 3;
                ua[0][w0] = na;
                ub[0][w0] = nb;
            }
#pragma unroll
            for (int k = 1; k <= S; ++k) {
                const int wn = (t - 2 * (k - 1) + 300) % 3;        // u_{k-1} row q+1
                const int wc = (t - 2 * (k - 1) - 1 + 300) % 3;    // row q
                const int wo = (t - 2 * (k - 1) - 2 + 300) % 3;    // row q-1
                const int ci = (t - (2 * k - 1) + 2 * NC * 50) % NC;
                const int tw = (t - (2 * k - 1) + 300) % 3;
                const float *pa = ua[k - 1], *pb = ub[k - 1];
                // column a: left neighbour from_left(b), right neighbour b;
                // column b: left neighbour a, right neighbour from_right(a)
                flux(from_left(pb[wo]) + pb[wn], from_left(pb[wn]) + pb[wo], from_left(pb[wc]) + pb[wc], pa[wo],
                     pa[wc], pa[wn], cma[ci], cea[ci], cpa[ci], cqa[ci], cha[ci], txa[k - 1][tw], tya[k - 1][tw],
                     tza[k - 1][tw]);
                flux(pa[wo] + from_right(pa[wn]), pa[wn] + from_right(pa[wo]), pa[wc] + from_right(pa[wc]), pb[wo],
                     pb[wc], pb[wn], cmb[ci], ceb[ci], cpb[ci], cqb[ci], chb[ci], txb[k - 1][tw], tyb[k - 1][tw],
                     tzb[k - 1][tw]);
                // u_k at row p = y - 2k (walking up: y + 2k)
                const int p = y - dir * 2 * k;
                const int sn = tw;
                const int sc = (t - 2 * k + 300) % 3;
                const int so = (t - 2 * k - 1 + 300) % 3;
                const float dxa = tya[k - 1][so] - tya[k - 1][sn];
                const float dxb = tyb[k - 1][so] - tyb[k - 1][sn];
                const float ela = fmaf(h2, dxa, txa[k - 1][sc]);
                const float era = fmaf(-h2, dxa, txa[k - 1][sc]);
                const float elb = fmaf(h2, dxb, txb[k - 1][sc]);
                const float erb = fmaf(-h2, dxb, txb[k - 1][sc]);
                // column a: el at x-1 is column b of the lane to the left, er at x+1 is column b
                const float rxa = fmaf(-2.f, txa[k - 1][sc], from_left(elb) + erb);
                const float rxb = fmaf(-2.f, txb[k - 1][sc], ela + from_right(era));
                const float rya = fmaf(-2.f, tza[k - 1][sc], tza[k - 1][so] + tza[k - 1][sn]);
                const float ryb = fmaf(-2.f, tzb[k - 1][sc], tzb[k - 1][so] + tzb[k - 1][sn]);
                const float ra = rxa + rya, rb = rxb + ryb;
                const int wp = (t - 2 * k + 300) % 3;
                const float nva = fmaf(-taus.t[k - 1], ra, ua[k - 1][wp]);
                const float nvb = fmaf(-taus.t[k - 1], rb, ub[k - 1][wp]);
                if (k < S) {
                    ua[k][wp] = nva;
                    ub[k][wp] = nvb;
                } else if (p >= ys && p < ye) {
                    const size_t r = (size_t)p * W;
                    if (PAIR) {
                        const u32x2 o = {__float_as_uint(nva), __float_as_uint(nvb)};
                        if (own) __builtin_amdgcn_raw_buffer_store_b64(o, bo, lbyte, 4u * (unsigned)r, 0);
                    } else {
                        if (sta) uo[r + xa] = nva;
                        if (stb) uo[r + xb] = nvb;
                    }
                }
            }
        }
    }
}

template <int S>
__device__ __forceinline__ void fed_stream_wave2(const float *__restrict__ u, float *__restrict__ uo,
                                                 const float *__restrict__ coef, int H, int W,
                                                 const FedTaus &taus, int strip, int seg, int seg_rows)
{
    const int x0 = strip * (128 - 4 * S) - 2 * S;   // first column of the strip
    const bool pair = (W & 1) == 0 && x0 >= 0 && x0 + 128 <= W && (size_t)H * W < ((size_t)1 << 29) &&
                      (((uintptr_t)u | (uintptr_t)uo | (uintptr_t)coef) & 7) == 0;
    // interior: columns x0 .. x0 + 127 and the loaded rows ys - 2 S .. ye + 2 S - 1
    // all lie in 1 .. W - 2 and 1 .. H - 2
    const int ys = seg * seg_rows, ye = min(ys + seg_rows, H);
    const bool inner = pair && x0 >= 1 && x0 + 128 <= W - 1 && ys - 2 * S >= 1 && ye + 2 * S <= H - 1;
    const bool up = (seg & 1) != 0;
    if (inner) fed_stream_wave2_body<S, true, true>(u, uo, coef, H, W, taus, strip, seg, seg_rows, up);
    else if (pair) fed_stream_wave2_body<S, true, false>(u, uo, coef, H, W, taus, strip, seg, seg_rows, up);
    else fed_stream_wave2_body<S, false, false>(u, uo, coef, H, W, taus, strip, seg, seg_rows, up);
}

}  // namespace tiles
}  // namespace mf4d
