// Learned scale surrogate: a 5-layer 3x3 convolutional network (channels
// 1 -> 32 -> 32 -> 32 -> 32 -> 9, zero padding) that predicts, per pixel, the
// index of the Gaussian scale the exact sweep would select (8 logits) and a
// confidence logit. Weights and activations are BF16, products accumulate
// in FP32 on the matrix cores (v_mfma_f32_16x16x16_bf16).
//
// Convolutions are implicit GEMMs over a 16 x 16 pixel tile: M = pixels,
// N = output channels, K = 9 taps x input channels. The input tile and its
// 1-pixel halo are staged in LDS (pixel-major, channels contiguous); each
// wave owns 4 rows of the tile (4 M-tiles) and every output channel.
// Backward: input gradients are the same convolution with transposed,
// flipped weights and a ReLU-mask epilogue; weight gradients are per-tile
// GEMMs over the tile's pixels (channel-major LDS), reduced over tiles in a
// fixed order.
//
// Parameter vector theta (FP32, the optimizer's master copy): for each layer
// W[cout][cin][3][3] then b[cout]. Kernel layouts are built from it per call.
#include <cmath>
#include <cstring>
#include <vector>

#include "mf4d_internal.h"
#include "scale_tiles.h"

namespace mf4d {

namespace net {

constexpr int kLayers = 5;
constexpr int kC[6] = {1, 32, 32, 32, 32, 9};
constexpr int kCP[6] = {16, 32, 32, 32, 32, 16};   // padded to MFMA K / N multiples

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__host__ __device__ constexpr int param_count()
{
    int n = 0;
    for (int l = 0; l < kLayers; ++l) n += kC[l + 1] * kC[l] * 9 + kC[l + 1];
    return n;
}
__host__ __device__ constexpr int theta_offset(int l)
{
    int n = 0;
    for (int k = 0; k < l; ++k) n += kC[k + 1] * kC[k] * 9 + kC[k + 1];
    return n;
}
__host__ __device__ constexpr int wsize(int l) { return 9 * kCP[l + 1] * kCP[l]; }   // kernel layout size

__device__ __forceinline__ uint16_t to_bf16(float f)
{
    // round to nearest even: one v_cvt_pk_bf16_f32 on gfx950
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// EPI_SELECT: the logits of the last layer, reduced per pixel to one byte
// (see conv_kernel) instead of being written out
enum { EPI_RELU = 0, EPI_LINEAR = 1, EPI_MASK = 2, EPI_SELECT = 3 };

// ------------------------------------------------------------------ forward
template <int CINP, int COUTP, int EPI>
__global__ __launch_bounds__(256, 4) void conv_kernel(const uint16_t *__restrict__ in, const uint16_t *__restrict__ wt,
                                                   const float *__restrict__ bias, const uint16_t *__restrict__ mask,
                                                   void *__restrict__ out, int H, int W, int tiles_per_img,
                                                   float thr = 0.f, int ns = 0)
{
    constexpr int NT = COUTP / 16, KC = CINP / 16, CH4 = CINP / 4;
    constexpr int ESZ = (EPI == EPI_LINEAR || EPI == EPI_SELECT) ? 4 : 2;   // output element bytes in LDS
    constexpr int OUT_BYTES = 256 * COUTP * ESZ;                    // the tile's output, pixel-major
    constexpr int IN_ELEMS = 18 * 18 * CINP;
    static_assert(EPI != EPI_SELECT || IN_ELEMS * 2 >= 256 * (COUTP + 1) * 4, "padded logits tile exceeds the LDS");
    // the input patch, then (after the products) the output tile on its way to HBM
    __shared__ __align__(16) uint16_t sIn[IN_ELEMS > OUT_BYTES / 2 ? IN_ELEMS : OUT_BYTES / 2];
    const int img = blockIdx.x / tiles_per_img, t = blockIdx.x % tiles_per_img;
    const int tx = W / 16;
    const int x0 = (t % tx) * 16, y0 = (t / tx) * 16;
    const size_t base = (size_t)img * H * W;
    // the 18 x 18 input patch (zero outside the image): every load is issued
    // before the first LDS store, so the block waits for one memory round trip
    constexpr int NST = (18 * 18 * CH4 + 255) / 256;
    uint2 v[NST];
#pragma unroll
    for (int it = 0; it < NST; ++it) {
        const int i = threadIdx.x + 256 * it;
        const int q = i / CH4, c4 = i % CH4;
        const int gy = y0 - 1 + q / 18, gx = x0 - 1 + q % 18;
        v[it] = make_uint2(0u, 0u);
        if (i < 18 * 18 * CH4 && gy >= 0 && gy < H && gx >= 0 && gx < W)
            v[it] = *(const uint2 *)(in + (base + (size_t)gy * W + gx) * CINP + c4 * 4);
    }
#pragma unroll
    for (int it = 0; it < NST; ++it) {
        const int i = threadIdx.x + 256 * it;
        const int q = i / CH4, c4 = i % CH4;
        if (i < 18 * 18 * CH4) *(uint2 *)(sIn + q * CINP + c4 * 4) = v[it];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    f4 acc[4][NT];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            s4 bfr[NT];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                bfr[nt] = *(const s4 *)(wt + (size_t)(tap * COUTP + nt * 16 + lr) * CINP + kc * 16 + lk * 4);
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                const int r = wv * 4 + mt;
                const s4 afr = *(const s4 *)(sIn + ((r + 1 + dy) * 18 + lr + 1 + dx) * CINP + kc * 16 + lk * 4);
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
                    acc[mt][nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(afr, bfr[nt], acc[mt][nt], 0, 0, 0);
            }
        }
    }
    // lane holds D[m = 4 lk + i][n = lr]: pixel x0 + 4 lk + i of row r, channel 16 nt + lr.
    // The tile's outputs go to LDS in the global pixel-major order, then to
    // HBM in 16-byte chunks (one tile row of 16 pixels is contiguous there).
    __syncthreads();   // every wave has finished reading the input patch
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        const int prow = (wv * 4 + mt) * 16 + lk * 4;   // pixel index inside the tile
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int c = nt * 16 + lr;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // pixel-major; EPI_SELECT pads the pixel stride by one float so
                // that thread t reading pixel t meets no bank conflict
                const int o = (prow + i) * (EPI == EPI_SELECT ? COUTP + 1 : COUTP) + c;
                const float v = acc[mt][nt][i];
                if (EPI == EPI_RELU) sIn[o] = to_bf16(fmaxf(v + bias[c], 0.f));
                else if (EPI == EPI_LINEAR || EPI == EPI_SELECT) ((float *)sIn)[o] = v + bias[c];
                else sIn[o] = to_bf16(v);
            }
        }
    }
    __syncthreads();
    if (EPI == EPI_SELECT) {
        // thread t takes pixel t of the tile: the network's scale (argmax of the
        // first min(ns, 8) logits, smallest index among equal maxima) in the low
        // bits, bit 7 set where the confidence sigmoid(z_8) reaches thr
        const float *zz = (const float *)sIn + threadIdx.x * (COUTP + 1);
        int best = 0;
        float mx = zz[0];
        for (int k = 1; k < ns && k < 8; ++k)
            if (zz[k] > mx) { mx = zz[k]; best = k; }
        const float conf = 1.f / (1.f + expf(-zz[8]));
        ((uint8_t *)out)[base + (size_t)(y0 + threadIdx.x / 16) * W + x0 + threadIdx.x % 16] =
            (uint8_t)(best | (conf >= thr ? 0x80 : 0));
        return;
    }
    constexpr int NCH = OUT_BYTES / 16, CPR = NCH / 16;   // 16-byte chunks, per tile row
#pragma unroll
    for (int it = 0; it < NCH / 256; ++it) {
        const int c = threadIdx.x + 256 * it;
        const int r = c / CPR, k = c - r * CPR;
        const size_t go = ((base + (size_t)(y0 + r) * W + x0) * COUTP) * ESZ + (size_t)k * 16;   // bytes
        uint4 val = ((const uint4 *)sIn)[c];
        if (EPI == EPI_MASK) {   // zero where the forward activation (ReLU output) is not positive
            const uint4 mk = *(const uint4 *)((const char *)mask + go);
            const uint32_t mw[4] = {mk.x, mk.y, mk.z, mk.w};
            uint32_t vw[4] = {val.x, val.y, val.z, val.w};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint32_t lo = from_bf16((uint16_t)(mw[q] & 0xffffu)) > 0.f ? 0x0000ffffu : 0u;
                const uint32_t hi = from_bf16((uint16_t)(mw[q] >> 16)) > 0.f ? 0xffff0000u : 0u;
                vw[q] &= lo | hi;
            }
            val = make_uint4(vw[0], vw[1], vw[2], vw[3]);
        }
        *(uint4 *)((char *)out + go) = val;
    }
}

// ---------------------------------------------------------- weight gradient
// Per 16 x 16 tile: dW[tap][co][ci] = sum_p dout[p][co] in[p + tap][ci] and
// db[co] = sum_p dout[p][co], written to the tile's partial slot.
template <int CINP, int COUTP>
__global__ __launch_bounds__(256) void wgrad_kernel(const uint16_t *__restrict__ in, const uint16_t *__restrict__ dout,
                                                    float *__restrict__ partial, int H, int W, int tiles_per_img)
{
    constexpr int MT = COUTP / 16, NT = CINP / 16, COMBOS = 9 * MT * NT;
    constexpr int PER = (COMBOS + 3) / 4;
    __shared__ uint16_t sI[CINP][18 * 18 + 4];
    __shared__ uint16_t sD[COUTP][256 + 4];
    const int img = blockIdx.x / tiles_per_img, t = blockIdx.x % tiles_per_img;
    const int tx = W / 16;
    const int x0 = (t % tx) * 16, y0 = (t / tx) * 16;
    const size_t base = (size_t)img * H * W;
    for (int i = threadIdx.x; i < 18 * 18 * CINP; i += 256) {
        const int q = i / CINP, c = i % CINP;
        const int gy = y0 - 1 + q / 18, gx = x0 - 1 + q % 18;
        uint16_t v = 0;
        if (gy >= 0 && gy < H && gx >= 0 && gx < W) v = in[(base + (size_t)gy * W + gx) * CINP + c];
        sI[c][q] = v;
    }
    for (int i = threadIdx.x; i < 256 * COUTP; i += 256) {
        const int q = i / COUTP, c = i % COUTP;
        sD[c][q] = dout[(base + (size_t)(y0 + q / 16) * W + x0 + q % 16) * COUTP + c];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    float *dst = partial + (size_t)blockIdx.x * (9 * COUTP * CINP + COUTP);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        const int combo = wv * PER + j;
        if (combo >= COMBOS) break;
        const int tap = combo / (MT * NT), mt = (combo / NT) % MT, nt = combo % NT;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        f4 acc = f4{0.f, 0.f, 0.f, 0.f};
        for (int r = 0; r < 16; ++r) {   // K-step: the 16 pixels of tile row r
            s4 a, b;
            const uint16_t *pa = &sD[mt * 16 + lr][r * 16 + lk * 4];
            const uint16_t *pb = &sI[nt * 16 + lr][(r + 1 + dy) * 18 + lk * 4 + 1 + dx];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                a[i] = (short)pa[i];
                b[i] = (short)pb[i];
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
        }
        // D[m = 4 lk + i][n = lr]: co = 16 mt + 4 lk + i, ci = 16 nt + lr
#pragma unroll
        for (int i = 0; i < 4; ++i)
            dst[(tap * COUTP + mt * 16 + lk * 4 + i) * CINP + nt * 16 + lr] = acc[i];
    }
    if (threadIdx.x < COUTP) {
        float s = 0.f;
        for (int q = 0; q < 256; ++q) s += from_bf16(sD[threadIdx.x][q]);
        dst[9 * COUTP * CINP + threadIdx.x] = s;
    }
}

// sums the per-tile partials in tile order (deterministic) and scatters
// them into theta order for layer l
__global__ void reduce_grad_kernel(const float *__restrict__ partial, int nblocks, int cinp, int coutp, int cin,
                                   int cout, float *__restrict__ grad_layer)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = 9 * coutp * cinp, stride = nw + coutp;
    if (j >= stride) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += partial[(size_t)b * stride + j];
    if (j < nw) {
        const int tap = j / (coutp * cinp), co = (j / cinp) % coutp, ci = j % cinp;
        if (co < cout && ci < cin) grad_layer[(co * cin + ci) * 9 + tap] = s;
    } else {
        const int co = j - nw;
        if (co < cout) grad_layer[cout * cin * 9 + co] = s;
    }
}

// ----------------------------------------------------------------- helpers
// theta -> forward weights [9][coutp][cinp], transposed-flipped weights
// [9][cinp][coutp] (input-gradient convolution) and padded biases
__global__ void pack_kernel(const float *__restrict__ th, uint16_t *__restrict__ wf, uint16_t *__restrict__ wb,
                            float *__restrict__ bias, int cin, int cout, int cinp, int coutp)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int nw = 9 * coutp * cinp;
    if (j < nw) {
        const int tap = j / (coutp * cinp), co = (j / cinp) % coutp, ci = j % cinp;
        const float v = (co < cout && ci < cin) ? th[(co * cin + ci) * 9 + tap] : 0.f;
        wf[j] = to_bf16(v);
        wb[((8 - tap) * cinp + ci) * coutp + co] = to_bf16(v);
    } else if (j < nw + coutp) {
        const int co = j - nw;
        bias[co] = co < cout ? th[cout * cin * 9 + co] : 0.f;
    }
}

__global__ void input_kernel(const float *__restrict__ u, uint16_t *__restrict__ a0, size_t P)
{
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    uint16_t *d = a0 + p * 16;
    d[0] = to_bf16(u[p]);
#pragma unroll
    for (int c = 1; c < 16; ++c) d[c] = 0;
}

__device__ __forceinline__ void softmax8(const float *z, float *pk, int *am)
{
    float mx = z[0];
    int a = 0;
    for (int k = 1; k < 8; ++k)
        if (z[k] > mx) { mx = z[k]; a = k; }
    float se = 0.f;
    for (int k = 0; k < 8; ++k) {
        pk[k] = expf(z[k] - mx);
        se += pk[k];
    }
    for (int k = 0; k < 8; ++k) pk[k] /= se;
    *am = a;
}

// loss, dLoss/dz (BF16) and per-block sums of the loss and of correct argmaxes
__global__ __launch_bounds__(256) void loss_kernel(const float *__restrict__ z, const uint8_t *__restrict__ label,
                                                   size_t P, float w_conf, uint16_t *__restrict__ dz,
                                                   float *__restrict__ part)
{
    __shared__ float sl[256], sc[256];
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    float loss = 0.f, corr = 0.f;
    if (p < P) {
        const float *zz = z + p * 16;
        float pk[8];
        int am;
        softmax8(zz, pk, &am);
        const int y = label[p];
        const float tgt = am == y ? 1.f : 0.f;
        const float zc = zz[8];
        loss = -logf(fmaxf(pk[y], 1e-30f)) + w_conf * (fmaxf(zc, 0.f) - zc * tgt + log1pf(expf(-fabsf(zc))));
        corr = tgt;
        const float inv = 1.f / (float)P;
        uint16_t *d = dz + p * 16;
        for (int k = 0; k < 8; ++k) d[k] = to_bf16((pk[k] - (k == y ? 1.f : 0.f)) * inv);
        d[8] = to_bf16(w_conf * (1.f / (1.f + expf(-zc)) - tgt) * inv);
        for (int k = 9; k < 16; ++k) d[k] = 0;
    }
    sl[threadIdx.x] = loss;
    sc[threadIdx.x] = corr;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            sl[threadIdx.x] += sl[threadIdx.x + s];
            sc[threadIdx.x] += sc[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = sl[0];
        part[2 * blockIdx.x + 1] = sc[0];
    }
}

__global__ void sum_parts_kernel(const float *__restrict__ part, int n, float P, float *__restrict__ out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float l = 0.f, c = 0.f;
    for (int i = 0; i < n; ++i) {
        l += part[2 * i];
        c += part[2 * i + 1];
    }
    out[0] = l / P;
    out[1] = c / P;
}

__global__ void predict_kernel(const float *__restrict__ z, size_t P, uint8_t *__restrict__ idx,
                               float *__restrict__ conf)
{
    const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= P) return;
    const float *zz = z + p * 16;
    int a = 0;
    float mx = zz[0];
    for (int k = 1; k < 8; ++k)
        if (zz[k] > mx) { mx = zz[k]; a = k; }
    if (idx) idx[p] = (uint8_t)a;
    if (conf) conf[p] = 1.f / (1.f + expf(-zz[8]));
}

__global__ void adam_kernel(float *__restrict__ th, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float gj = g[j];
    const float mj = b1 * m[j] + (1.f - b1) * gj;
    const float vj = b2 * v[j] + (1.f - b2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    th[j] -= lr * (mj / c1) / (sqrtf(vj / c2) + eps);
}

// learned selection: the network's scale where its confidence reaches the
// threshold, the exact argmax elsewhere (the integration then gathers N at
// that scale through idx)
__global__ __launch_bounds__(256) void learned_select_kernel(const uint8_t *__restrict__ sel,
                                                             const float *__restrict__ SA,
                                                             int ns, size_t plane,
                                                             const unsigned *__restrict__ smax_bits, float c_param,
                                                             uint8_t *__restrict__ idx, unsigned *__restrict__ fallback)
{
    __shared__ unsigned cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    const size_t o = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o < plane) {
        const unsigned code = sel[o];   // network scale, bit 7: confident
        int best = (int)(code & 0x7fu);
        if (!(code & 0x80u)) {
            const float c = c_param > 0.f ? c_param : 0.5f * __uint_as_float(*smax_bits);
            float bv;
            best = tiles::argmax_px(SA, ns, plane, o, c, &bv);
            atomicAdd(&cnt, 1u);
        }
        idx[o] = (uint8_t)best;
    }
    __syncthreads();
    // one of kFallbackSlots counters per block, so the blocks' atomics spread
    // over that many addresses instead of all meeting on one
    if (threadIdx.x == 0 && cnt) atomicAdd(fallback + blockIdx.x % kFallbackSlots, cnt);
}

// one workgroup per 32 x 32 block: the scales its pixels need
__global__ __launch_bounds__(256) void need_flags_kernel(const uint8_t *__restrict__ sel, int H, int W, int ns,
                                                         int bx, uint8_t *__restrict__ need)
{
    __shared__ unsigned bits;
    if (threadIdx.x == 0) bits = 0u;
    __syncthreads();
    const int x0 = (blockIdx.x % bx) * 32, y0 = (blockIdx.x / bx) * 32;
    const unsigned all = (1u << ns) - 1u;
    unsigned m = 0u;
    for (int i = threadIdx.x; i < 1024; i += 256) {
        const int x = x0 + (i & 31), y = y0 + (i >> 5);
        if (x >= W || y >= H) continue;
        const unsigned code = sel[(size_t)y * W + x];
        m |= (code & 0x80u) ? (1u << (code & 0x7fu)) : all;
    }
    if (m) atomicOr(&bits, m);
    __syncthreads();
    if (threadIdx.x == 0) need[blockIdx.x] = (uint8_t)bits;
}

// the total of the fallback counters
__global__ void fallback_sum_kernel(const unsigned *__restrict__ slots, unsigned *__restrict__ total)
{
    if (threadIdx.x == 0) {
        unsigned t = 0;
        for (int i = 0; i < kFallbackSlots; ++i) t += slots[i];
        *total = t;
    }
}

// --------------------------------------------------------------- workspace
struct NetWs {
    uint16_t *wf[kLayers], *wb[kLayers];
    float *bias[kLayers];
    uint16_t *act[kLayers];   // act[0] = input [P][16], act[l] = output of layer l-1 [P][32]
    float *z;                 // [P][16]
    uint16_t *dz;             // [P][16]
    uint16_t *d[2];           // [P][32] ping-pong input gradients
    float *partial;           // [tiles][9*32*32+32]
    float *lossparts;         // [2 * ceil(P/256)]
};

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t net_layout(int B, int H, int W, bool train, NetWs *w, char *base)
{
    const size_t P = (size_t)B * H * W;
    const size_t tiles = P / 256;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + off : nullptr;
        off += al256(bytes);
        return p;
    };
    NetWs t;
    for (int l = 0; l < kLayers; ++l) {
        t.wf[l] = (uint16_t *)take(2 * wsize(l));
        t.wb[l] = (uint16_t *)take(2 * wsize(l));
        t.bias[l] = (float *)take(4 * kCP[l + 1]);
    }
    t.act[0] = (uint16_t *)take(P * 16 * 2);
    for (int l = 1; l < kLayers; ++l) t.act[l] = (uint16_t *)take(P * 32 * 2);
    t.z = (float *)take(P * 16 * 4);
    if (train) {
        t.dz = (uint16_t *)take(P * 16 * 2);
        t.d[0] = (uint16_t *)take(P * 32 * 2);
        t.d[1] = (uint16_t *)take(P * 32 * 2);
        t.partial = (float *)take(tiles * (9 * 32 * 32 + 32) * 4);
        t.lossparts = (float *)take(((P + 255) / 256) * 2 * 4 + 16);
    } else {
        t.dz = nullptr;
        t.d[0] = t.d[1] = nullptr;
        t.partial = t.lossparts = nullptr;
    }
    if (w) *w = t;
    return off;
}

#define NCHECK(expr)                                  \
    do {                                              \
        if ((expr) != hipSuccess) return MF4D_EHIP;   \
    } while (0)

int pack_all(const float *theta, const NetWs &w, hipStream_t s)
{
    for (int l = 0; l < kLayers; ++l) {
        const int n = wsize(l) + kCP[l + 1];
        hipLaunchKernelGGL(pack_kernel, dim3((n + 255) / 256), dim3(256), 0, s, theta + theta_offset(l), w.wf[l],
                           w.wb[l], w.bias[l], kC[l], kC[l + 1], kCP[l], kCP[l + 1]);
        NCHECK(hipGetLastError());
    }
    return MF4D_OK;
}

int forward_all(const float *u, int B, int H, int W, const NetWs &w, hipStream_t s)
{
    const size_t P = (size_t)B * H * W;
    const int tpi = (H / 16) * (W / 16);
    const dim3 grid(B * tpi), blk(256);
    hipLaunchKernelGGL(input_kernel, dim3((unsigned)((P + 255) / 256)), blk, 0, s, u, w.act[0], P);
    hipLaunchKernelGGL((conv_kernel<16, 32, EPI_RELU>), grid, blk, 0, s, w.act[0], w.wf[0], w.bias[0], nullptr,
                       (void *)w.act[1], H, W, tpi);
    for (int l = 1; l < 4; ++l)
        hipLaunchKernelGGL((conv_kernel<32, 32, EPI_RELU>), grid, blk, 0, s, w.act[l], w.wf[l], w.bias[l], nullptr,
                           (void *)w.act[l + 1], H, W, tpi);
    hipLaunchKernelGGL((conv_kernel<32, 16, EPI_LINEAR>), grid, blk, 0, s, w.act[4], w.wf[4], w.bias[4], nullptr,
                       (void *)w.z, H, W, tpi);
    NCHECK(hipGetLastError());
    return MF4D_OK;
}

// forward_all with the last layer reduced to the selection byte per pixel
// (EPI_SELECT) in sel
int forward_select(const float *u, int H, int W, const NetWs &w, float thr, int ns, uint8_t *sel, hipStream_t s)
{
    const int B = 1;
    const size_t P = (size_t)B * H * W;
    const int tpi = (H / 16) * (W / 16);
    const dim3 grid(B * tpi), blk(256);
    hipLaunchKernelGGL(input_kernel, dim3((unsigned)((P + 255) / 256)), blk, 0, s, u, w.act[0], P);
    hipLaunchKernelGGL((conv_kernel<16, 32, EPI_RELU>), grid, blk, 0, s, w.act[0], w.wf[0], w.bias[0], nullptr,
                       (void *)w.act[1], H, W, tpi);
    for (int l = 1; l < 4; ++l)
        hipLaunchKernelGGL((conv_kernel<32, 32, EPI_RELU>), grid, blk, 0, s, w.act[l], w.wf[l], w.bias[l], nullptr,
                           (void *)w.act[l + 1], H, W, tpi);
    hipLaunchKernelGGL((conv_kernel<32, 16, EPI_SELECT>), grid, blk, 0, s, w.act[4], w.wf[4], w.bias[4], nullptr,
                       (void *)sel, H, W, tpi, thr, ns);
    NCHECK(hipGetLastError());
    return MF4D_OK;
}

bool shape_ok(int B, int H, int W)
{
    return B >= 1 && H >= 16 && W >= 16 && H % 16 == 0 && W % 16 == 0 && (long long)B * H * W < (1LL << 31);
}

}  // namespace net

// network forward for the learned filter: returns the logits [P][16]
int net_select_into(const float *theta, const float *u, int H, int W, char *ws, hipStream_t s, float thr, int ns,
                    const uint8_t **sel, bool pack)
{
    using namespace net;
    NetWs w;
    net_layout(1, H, W, false, &w, ws);
    int st = pack ? pack_all(theta, w, s) : MF4D_OK;
    uint8_t *out = (uint8_t *)w.z;   // the logits' space holds the selection bytes
    if (st == MF4D_OK) st = forward_select(u, H, W, w, thr, ns, out, s);
    *sel = out;
    return st;
}

size_t net_forward_bytes(int H, int W) { return net::net_layout(1, H, W, false, nullptr, nullptr); }

hipError_t launch_fallback_sum(const unsigned *slots, unsigned *total, hipStream_t s)
{
    hipLaunchKernelGGL(net::fallback_sum_kernel, dim3(1), dim3(64), 0, s, slots, total);
    return hipGetLastError();
}

hipError_t launch_need_flags(const uint8_t *sel, int H, int W, int ns, uint8_t *need, hipStream_t s)
{
    const int bx = (W + 31) / 32, by = (H + 31) / 32;
    hipLaunchKernelGGL(net::need_flags_kernel, dim3(bx * by), dim3(256), 0, s, sel, H, W, ns, bx, need);
    return hipGetLastError();
}

hipError_t launch_learned_select(const uint8_t *sel, const SelectArgs &a, int H, int W, unsigned *fallback,
                                 hipStream_t s)
{
    const size_t plane = (size_t)H * W;
    hipLaunchKernelGGL(net::learned_select_kernel, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, s, sel, a.SA,
                       a.ns, plane, a.smax_bits, a.c_param, a.idx_out, fallback);
    return hipGetLastError();
}

// learned-filter helpers defined in mf4d_api.hip
int validate_params(int H, int W, const mf4d_params *p);
size_t image_workspace_bytes(int H, int W, int ns);
void image_workspace(int H, int W, int ns, char *base, float **hA, float **SA, float **N,
                     uint8_t **idx, float **tens, float **utmp, unsigned **smax);
void window_taps(double sigma, WinTaps *t);
void rho_taps(double rho, RhoTaps *t);
int fed_plan_host(const mf4d_params *p, int *n_out, std::vector<double> &ordered);
int default_stream_rows(int H, int W, int steps);

}  // namespace mf4d

using namespace mf4d;
using namespace mf4d::net;

extern "C" {

size_t mf4d_net_param_count(void) { return (size_t)param_count(); }

size_t mf4d_net_workspace_bytes(int B, int H, int W, int train)
{
    if (!shape_ok(B, H, W)) return 0;
    return net_layout(B, H, W, train != 0, nullptr, nullptr);
}

int mf4d_net_forward(const float *theta, const float *u, int B, int H, int W, float *logits, uint8_t *idx_out,
                     float *conf_out, void *ws, size_t ws_bytes, void *stream)
{
    if (!theta || !u || !ws || !shape_ok(B, H, W)) return MF4D_EINVAL;
    if (ws_bytes < net_layout(B, H, W, false, nullptr, nullptr)) return MF4D_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    NetWs w;
    net_layout(B, H, W, false, &w, (char *)ws);
    int st = pack_all(theta, w, s);
    if (st == MF4D_OK) st = forward_all(u, B, H, W, w, s);
    if (st != MF4D_OK) return st;
    const size_t P = (size_t)B * H * W;
    if (logits) NCHECK(hipMemcpyAsync(logits, w.z, P * 16 * 4, hipMemcpyDeviceToDevice, s));
    if (idx_out || conf_out) {
        hipLaunchKernelGGL(predict_kernel, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, w.z, P, idx_out,
                           conf_out);
        NCHECK(hipGetLastError());
    }
    return MF4D_OK;
}

int mf4d_net_backward(const float *theta, const float *u, const uint8_t *labels, int B, int H, int W, float w_conf,
                      float *grad, float *stats_out, void *ws, size_t ws_bytes, void *stream)
{
    if (!theta || !u || !labels || !grad || !ws || !shape_ok(B, H, W) || !(w_conf >= 0.f)) return MF4D_EINVAL;
    if (ws_bytes < net_layout(B, H, W, true, nullptr, nullptr)) return MF4D_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    NetWs w;
    net_layout(B, H, W, true, &w, (char *)ws);
    int st = pack_all(theta, w, s);
    if (st == MF4D_OK) st = forward_all(u, B, H, W, w, s);
    if (st != MF4D_OK) return st;
    const size_t P = (size_t)B * H * W;
    const int tpi = (H / 16) * (W / 16), nb = B * tpi;
    const dim3 grid(nb), blk(256);
    const int lblocks = (int)((P + 255) / 256);
    hipLaunchKernelGGL(loss_kernel, dim3(lblocks), blk, 0, s, w.z, labels, P, w_conf, w.dz, w.lossparts);
    if (stats_out)
        hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(64), 0, s, w.lossparts, lblocks, (float)P, stats_out);
    NCHECK(hipGetLastError());
    // layer 4: weight gradient, then input gradient through the ReLU of act[4]
    auto reduce = [&](int l) {
        const int stride = wsize(l) + kCP[l + 1];
        hipLaunchKernelGGL(reduce_grad_kernel, dim3((stride + 255) / 256), blk, 0, s, w.partial, nb, kCP[l],
                           kCP[l + 1], kC[l], kC[l + 1], grad + theta_offset(l));
    };
    hipLaunchKernelGGL((wgrad_kernel<32, 16>), grid, blk, 0, s, w.act[4], w.dz, w.partial, H, W, tpi);
    reduce(4);
    hipLaunchKernelGGL((conv_kernel<16, 32, EPI_MASK>), grid, blk, 0, s, w.dz, w.wb[4], nullptr, w.act[4],
                       (void *)w.d[0], H, W, tpi);
    int cur = 0;
    for (int l = 3; l >= 1; --l) {
        hipLaunchKernelGGL((wgrad_kernel<32, 32>), grid, blk, 0, s, w.act[l], w.d[cur], w.partial, H, W, tpi);
        reduce(l);
        hipLaunchKernelGGL((conv_kernel<32, 32, EPI_MASK>), grid, blk, 0, s, w.d[cur], w.wb[l], nullptr, w.act[l],
                           (void *)w.d[1 - cur], H, W, tpi);
        cur = 1 - cur;
    }
    hipLaunchKernelGGL((wgrad_kernel<16, 32>), grid, blk, 0, s, w.act[0], w.d[cur], w.partial, H, W, tpi);
    reduce(0);
    NCHECK(hipGetLastError());
    return MF4D_OK;
}

int mf4d_net_step(float *theta, const float *grad, float *adam_m, float *adam_v, int step, float lr, void *stream)
{
    if (!theta || !grad || !adam_m || !adam_v || step < 1 || !(lr > 0.f)) return MF4D_EINVAL;
    const int n = param_count();
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - std::pow(b1, (float)step), c2 = 1.f - std::pow(b2, (float)step);
    hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, theta, grad, adam_m,
                       adam_v, n, lr, b1, b2, 1e-8f, c1, c2);
    NCHECK(hipGetLastError());
    return MF4D_OK;
}

}  // extern "C"
