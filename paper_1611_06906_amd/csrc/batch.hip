// Batched filter: many images of different sizes in one hipGraph.
//
// All images advance through the FED cycles together. Every stage (sweep
// passes, argmax, integration, streaming substeps) is one launch for the
// whole batch: a prefix table maps the launch's blocks to (image, tile), and
// the tile-level code is the same device code the single-image kernels run,
// on the same tile grid, so each image's result is bit-identical to a
// single-image mf4d_filter call. Images are ordered by decreasing cycle
// count, so the images still active in cycle k are a prefix of the tables and
// a launch simply covers fewer blocks once short images have finished. The
// whole launch sequence is captured once into a hipGraph (no memset nodes:
// counters are cleared by a kernel) and replayed per call.
//
// The streaming substep kernel's decomposition (substeps per launch and rows
// per wave) does not change any value; mf4d_batch_autotune times candidate
// decompositions on the batch's shapes and keeps the fastest.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "fed_tiles.h"
#include "scale_mfma.h"

namespace mf4d {

// Device record of one image of the batch.
struct BImg {
    const float *user_in;   // caller's input
    const float *in;        // source of the first launch (user_in, or its copy in tmp)
    float *out, *tmp;       // launch j writes (j + parity) odd ? tmp : out
    float *hA;              // 3 planes: horizontal pass of the split and register-window sweep forms
    float *SA, *N;          // per-scale (S, blob) pairs and N
    uint8_t *idx;
    float *tens;
    unsigned *smax;
    int H, W, mode, parity, copy_in, copy_out;
    int strips[5], segs[5], seg_rows[5];   // streaming decomposition per substeps-per-launch
};

enum { PT_HV = 0, PT_PX, PT_RHO, PT_ST1, PT_ST2, PT_ST3, PT_ST4, PT_HM, PT_VM, PT_FU, PT_COUNT };

// rows per workgroup of the batched matrix-core vertical pass and of the
// batched fused kernel (any multiple of the step gives the same values)
constexpr int kBatchVSegRows = 256;
constexpr int kBatchFusedSegRows = 1024;

namespace {

using namespace tiles;

__device__ __forceinline__ int image_of(const int *pre, int nact, int b)
{
    int lo = 0, hi = nact;   // pre[lo] <= b < pre[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (pre[mid] <= b) lo = mid;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ const float *state_src(const BImg &im, int j)
{
    if (j == 0) return im.in;
    return ((j - 1 + im.parity) & 1) ? im.tmp : im.out;
}

__device__ __forceinline__ float *state_dst(const BImg &im, int j)
{
    return ((j + im.parity) & 1) ? im.tmp : im.out;
}

__global__ void batch_fill_kernel(const BImg *imgs, int nact)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nact) *imgs[i].smax = 0u;
}

__global__ __launch_bounds__(256) void batch_copy_kernel(const BImg *imgs, const int *pre, int nact)
{
    const int i = image_of(pre, nact, blockIdx.x);
    const BImg &im = imgs[i];
    if (!im.copy_in && !im.copy_out) return;
    const size_t o = (size_t)(blockIdx.x - pre[i]) * 256 + threadIdx.x;
    if (o >= (size_t)im.H * im.W) return;
    if (im.copy_in) im.tmp[o] = im.user_in[o];
    else im.out[o] = im.user_in[o];   // an image with no cycles
}

__global__ __launch_bounds__(256) void batch_hpass_kernel(const BImg *imgs, const int *pre, int nact, WinTaps t,
                                                          int jsrc)
{
    extern __shared__ float tile[];
    const int i = image_of(pre, nact, blockIdx.x);
    const BImg &im = imgs[i];
    const int lt = blockIdx.x - pre[i];
    const int tx = (im.W + 63) / 64;
    const size_t m = (size_t)im.H * im.W;
    hpass_tile(state_src(im, jsrc), im.hA, im.hA + m, im.hA + 2 * m, im.H, im.W, t, (lt % tx) * 64,
               (lt / tx) * 64, tile);
}

__global__ __launch_bounds__(256) void batch_vpass_kernel(const BImg *imgs, const int *pre, int nact, WinTaps t,
                                                          float sigma2, float inv2beta2, int s)
{
    const int i = image_of(pre, nact, blockIdx.x);
    const BImg &im = imgs[i];
    const int lt = blockIdx.x - pre[i];
    const int tx = (im.W + 63) / 64;
    const size_t m = (size_t)im.H * im.W;
    const float *A = im.hA, *B = im.hA + m, *C = im.hA + 2 * m;
    float *SA = im.SA + 2 * s * m, *No = im.N + 3 * s * m;
    const int x0 = (lt % tx) * 64, y0 = (lt / tx) * 64;
    float v;
    if (im.mode == MF4D_RIDGE) v = vpass_tile<MF4D_RIDGE>(A, B, C, im.H, im.W, t, sigma2, inv2beta2, SA, No, x0, y0);
    else if (im.mode == MF4D_VALLEY) v = vpass_tile<MF4D_VALLEY>(A, B, C, im.H, im.W, t, sigma2, inv2beta2, SA, No, x0, y0);
    else v = vpass_tile<MF4D_BOTH>(A, B, C, im.H, im.W, t, sigma2, inv2beta2, SA, No, x0, y0);
    block_max_to(v, im.smax);
}

template <int NC>
__global__ __launch_bounds__(256) void batch_hpass_mfma_kernel(const BImg *imgs, const int *pre, int nact, WinTaps t,
                                                               int jsrc, int per_xcd)
{
    extern __shared__ f4 lds4[];
    const int b = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (b >= pre[nact]) return;
    const int i = image_of(pre, nact, b);
    const BImg &im = imgs[i];
    const int lt = b - pre[i];
    const int tx = (im.W + kHMW - 1) / kHMW;
    const size_t m = (size_t)im.H * im.W;
    hpass_mfma_tile<NC>(state_src(im, jsrc), im.hA, im.hA + m, im.hA + 2 * m, im.H, im.W, t, (lt % tx) * kHMW,
                        (lt / tx) * kHMH, (float *)lds4);
}

template <int NC>
__global__ __launch_bounds__(256) void batch_vpass_mfma_kernel(const BImg *imgs, const int *pre, int nact, WinTaps t,
                                                               float sigma2, float inv2beta2, int s, int per_xcd)
{
    extern __shared__ f4 lds4[];
    const int b = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (b >= pre[nact]) return;
    const int i = image_of(pre, nact, b);
    const BImg &im = imgs[i];
    const int lt = b - pre[i];
    const int segs = (im.H + kBatchVSegRows - 1) / kBatchVSegRows;
    const int strip = lt / segs, seg = lt - strip * segs;
    const int ys = seg * kBatchVSegRows, ye = min(im.H, ys + kBatchVSegRows);
    const size_t m = (size_t)im.H * im.W;
    const float v = vpass_mfma_tile<NC>(im.hA, im.hA + m, im.hA + 2 * m, im.H, im.W, t, sigma2, inv2beta2, im.mode,
                                        im.SA + 2 * s * m, im.N + 3 * s * m, strip * kVMW, ys, ye,
                                        (float *)lds4);
    block_max_to(v, im.smax);
}

template <int NC>
__global__ __launch_bounds__(256, 2) void batch_sweep_fused_kernel(const BImg *imgs, const int *pre, int nact, WinTaps t,
                                                                float sigma2, float inv2beta2, int s, int jsrc,
                                                                int per_xcd)
{
    extern __shared__ f4 lds4[];
    const int b = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (b >= pre[nact]) return;
    const int i = image_of(pre, nact, b);
    const BImg &im = imgs[i];
    const int lt = b - pre[i];
    const int segs = (im.H + kBatchFusedSegRows - 1) / kBatchFusedSegRows;
    const int strip = lt / segs, seg = lt - strip * segs;
    const int ys = seg * kBatchFusedSegRows, ye = min(im.H, ys + kBatchFusedSegRows);
    const size_t m = (size_t)im.H * im.W;
    const float v = sweep_fused_tile<NC>(state_src(im, jsrc), im.H, im.W, t, sigma2, inv2beta2, im.mode,
                                         im.SA + 2 * s * m, im.N + 3 * s * m, strip * kVMW, ys, ye, (float *)lds4);
    block_max_to(v, im.smax);
}

__global__ __launch_bounds__(256) void batch_argmax_kernel(const BImg *imgs, const int *pre, int nact, int ns,
                                                           float c_param)
{
    const int i = image_of(pre, nact, blockIdx.x);
    const BImg &im = imgs[i];
    const size_t m = (size_t)im.H * im.W;
    const size_t o = (size_t)(blockIdx.x - pre[i]) * 256 + threadIdx.x;
    if (o >= m) return;
    const float c = c_param > 0.f ? c_param : 0.5f * __uint_as_float(*im.smax);
    float bv;
    im.idx[o] = (uint8_t)argmax_px(im.SA, ns, m, o, c, &bv);
}

// H_rho of each image, N gathered through its scale indices
template <int HR>
__global__ __launch_bounds__(256) void batch_rho_kernel(const BImg *imgs, const int *pre, int nact, int ns,
                                                        RhoTaps t, float inv_lam2)
{
    const int i = image_of(pre, nact, blockIdx.x);
    const BImg &im = imgs[i];
    const int lt = blockIdx.x - pre[i];
    const int tx = (im.W + kBTW - 1) / kBTW;
    rho_blur_tile<HR>(im.N, im.idx, ns, nullptr, im.tens, im.mode, inv_lam2, im.H, im.W, t, (lt % tx) * kBTW,
                      (lt / tx) * kBTH);
}

template <int S, int C>
__global__ __launch_bounds__(256) void batch_stream_kernel(const BImg *imgs, const int *pre, int nact, FedTaus taus,
                                                           int j, int per_xcd)
{
    // XCD-aware: each XCD takes a contiguous run of blocks
    const int b = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (b >= pre[nact]) return;
    const int i = image_of(pre, nact, b);
    const BImg &im = imgs[i];
    const int wave = __builtin_amdgcn_readfirstlane((b - pre[i]) * 4 + (threadIdx.x >> 6));   // uniform per wave
    const int strip = wave % im.strips[S], seg = wave / im.strips[S];
    if (seg >= im.segs[S]) return;
    if (C == 2)
        fed_stream_wave2<S>(state_src(im, j), state_dst(im, j), im.tens, im.H, im.W, taus, strip, seg,
                            im.seg_rows[S]);
    else
        fed_stream_wave<S>(state_src(im, j), state_dst(im, j), im.tens, im.H, im.W, taus, strip, seg,
                           im.seg_rows[S]);
}

void launch_batch_stream(int cols, int steps, dim3 grid, hipStream_t s, const BImg *imgs, const int *pt, int nact,
                         const FedTaus &ft, int j, int per)
{
#define MF4D_BS(K)                                                                                            \
    case K:                                                                                                   \
        if (cols == 2)                                                                                        \
            hipLaunchKernelGGL((batch_stream_kernel<K, 2>), grid, dim3(256), 0, s, imgs, pt, nact, ft, j, per);  \
        else                                                                                                  \
            hipLaunchKernelGGL((batch_stream_kernel<K, 1>), grid, dim3(256), 0, s, imgs, pt, nact, ft, j, per);  \
        break;
    switch (steps) {
        MF4D_BS(1) MF4D_BS(2) MF4D_BS(3)
    default:
        MF4D_BS(4)
    }
#undef MF4D_BS
}

}  // namespace

}  // namespace mf4d

using namespace mf4d;

struct mf4d_batch {
    int nimg = 0;
    std::vector<int64_t> off;
    std::vector<int> H, W, mode, cycles;
    std::vector<float> sigmas;
    mf4d_params shared{};
    std::vector<int> order;          // images by decreasing cycle count
    int n = 0, max_cycles = 0;
    std::vector<float> tau32;
    int spl = 4;                     // substeps per launch
    int cols[5] = {1, 1, 1, 1, 2};   // columns per lane of the streaming kernel per substeps (fixed at creation)
    int rows[5] = {0, 0, 0, 0, 0};   // rows per wave (0: default)
    size_t table_bytes = 0, ws_total = 0;
    std::vector<size_t> img_ws;      // per image (sorted order) workspace offset
    // cached graph
    const void *g_in = nullptr;
    void *g_out = nullptr, *g_ws = nullptr;
    bool have_graph = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<char> host_tables;
};

namespace {

size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

void drop_graph(mf4d_batch *b)
{
    if (b->exec) hipGraphExecDestroy(b->exec);
    if (b->graph) hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->have_graph = false;
}

int rows_for(const mf4d_batch *b, int H, int W, int steps)
{
    return b->rows[steps] > 0 ? b->rows[steps] : default_stream_rows(H, W, steps);
}

// Builds the device tables (host image) for the given pointers.
void build_tables(mf4d_batch *b, const float *in, float *out, char *ws, std::vector<int> pre[PT_COUNT])
{
    const int N = b->nimg;
    const int ns = b->shared.nscales;
    const int lpc = (b->n + b->spl - 1) / b->spl;
    b->host_tables.assign(b->table_bytes, 0);
    BImg *imgs = (BImg *)b->host_tables.data();
    for (int k = 0; k < PT_COUNT; ++k) pre[k].assign(N + 1, 0);
    for (int r = 0; r < N; ++r) {
        const int i = b->order[r];
        BImg &im = imgs[r];
        const int H = b->H[i], W = b->W[i];
        im.H = H;
        im.W = W;
        im.mode = b->mode[i];
        float *utmp;
        image_workspace(H, W, ns, ws + b->img_ws[r], &im.hA, &im.SA, &im.N, &im.idx, &im.tens, &utmp,
                        &im.smax);
        im.user_in = in + b->off[i];
        im.out = out + b->off[i];
        im.tmp = utmp;
        const long long L = (long long)b->cycles[i] * lpc;
        im.parity = (int)((L + 1) % 2);
        im.copy_in = (L > 0 && im.user_in == im.out && im.parity == 0) ? 1 : 0;
        im.copy_out = (L == 0 && im.user_in != im.out) ? 1 : 0;
        im.in = im.copy_in ? im.tmp : im.user_in;
        for (int s = 1; s <= 4; ++s) {
            const int outw = 64 * b->cols[s] - 4 * s;
            im.strips[s] = (W + outw - 1) / outw;
            im.seg_rows[s] = rows_for(b, H, W, s);
            im.segs[s] = (H + im.seg_rows[s] - 1) / im.seg_rows[s];
        }
        const int hv = ((W + 63) / 64) * ((H + 63) / 64);
        const int px = (int)(((size_t)H * W + 255) / 256);
        const int rho = ((W + kBTW - 1) / kBTW) * ((H + kBTH - 1) / kBTH);
        pre[PT_HV][r + 1] = pre[PT_HV][r] + hv;
        pre[PT_PX][r + 1] = pre[PT_PX][r] + px;
        pre[PT_RHO][r + 1] = pre[PT_RHO][r] + rho;
        pre[PT_HM][r + 1] = pre[PT_HM][r] + ((W + kHMW - 1) / kHMW) * ((H + kHMH - 1) / kHMH);
        pre[PT_VM][r + 1] = pre[PT_VM][r] + ((W + kVMW - 1) / kVMW) * ((H + kBatchVSegRows - 1) / kBatchVSegRows);
        pre[PT_FU][r + 1] = pre[PT_FU][r] + ((W + kVMW - 1) / kVMW) * ((H + kBatchFusedSegRows - 1) / kBatchFusedSegRows);
        for (int s = 1; s <= 4; ++s)
            pre[PT_ST1 + s - 1][r + 1] = pre[PT_ST1 + s - 1][r] + (im.strips[s] * im.segs[s] + 3) / 4;
    }
    int *tab = (int *)(b->host_tables.data() + al256(sizeof(BImg) * N));
    for (int k = 0; k < PT_COUNT; ++k) std::memcpy(tab + k * (N + 1), pre[k].data(), sizeof(int) * (N + 1));
}

#define BCHECK(expr)                                  \
    do {                                              \
        if ((expr) != hipSuccess) return MF4D_EHIP;   \
    } while (0)

// Enqueues the whole batch on stream s (captured into the graph by the caller).
int enqueue_batch(mf4d_batch *b, char *ws, const std::vector<int> pre[PT_COUNT], hipStream_t s)
{
    const int N = b->nimg;
    const BImg *imgs = (const BImg *)ws;
    const int *tab = (const int *)(ws + al256(sizeof(BImg) * N));
    auto P = [&](int k) { return tab + k * (N + 1); };
    const mf4d_params &p = b->shared;
    const int ns = p.nscales;
    const int lpc = (b->n + b->spl - 1) / b->spl;
    const float inv_lam2 = 1.f / (p.lambda * p.lambda);
    const float inv2beta2 = 1.f / (2.f * p.beta * p.beta);
    std::vector<WinTaps> taps(ns);
    for (int k = 0; k < ns; ++k) window_taps(p.sigmas[k], &taps[k]);
    RhoTaps rt;
    rho_taps(p.rho, &rt);
    // copies: in-place images whose first launch would overwrite the input, and
    // images with no cycles (output = input)
    hipLaunchKernelGGL(batch_copy_kernel, dim3(pre[PT_PX][N]), dim3(256), 0, s, imgs, P(PT_PX), N);
    BCHECK(hipGetLastError());
    int j = 0;
    for (int k = 0; k < b->max_cycles; ++k) {
        int nact = 0;
        while (nact < N && b->cycles[b->order[nact]] > k) ++nact;
        hipLaunchKernelGGL(batch_fill_kernel, dim3((nact + 255) / 256), dim3(256), 0, s, imgs, nact);
        BCHECK(hipGetLastError());
        for (int sc = 0; sc < ns; ++sc) {
            const float sig = p.sigmas[sc];
            if (sweep_engine(taps[sc]) == kSweepFused) {
                const int per_f = (pre[PT_FU][nact] + 7) / 8;
                switch (sweep_chunks(taps[sc])) {
#define MF4D_BFU(NC)                                                                                              \
    case NC:                                                                                                      \
        hipLaunchKernelGGL(batch_sweep_fused_kernel<NC>, dim3(8 * per_f), dim3(256), fused_lds(NC), s, imgs,          \
                           P(PT_FU), nact, taps[sc], sig * sig, inv2beta2, sc, j, per_f);                         \
        break;
                    MF4D_BFU(2) MF4D_BFU(3) MF4D_BFU(4) MF4D_BFU(5) MF4D_BFU(6) MF4D_BFU(7) MF4D_BFU(8)
#undef MF4D_BFU
                default: return MF4D_EINVAL;
                }
                BCHECK(hipGetLastError());
                continue;
            }
            if (const int nc = sweep_chunks(taps[sc])) {
                const int per_h = (pre[PT_HM][nact] + 7) / 8;
                switch (nc) {
#define MF4D_BHM(NC)                                                                                              \
    case NC:                                                                                                      \
        hipLaunchKernelGGL(batch_hpass_mfma_kernel<NC>, dim3(8 * per_h), dim3(256), hpass_mfma_lds(NC), s, imgs,      \
                           P(PT_HM), nact, taps[sc], j, per_h);                                                   \
        break;
                    MF4D_BHM(2) MF4D_BHM(3) MF4D_BHM(4) MF4D_BHM(5) MF4D_BHM(6) MF4D_BHM(7) MF4D_BHM(8) MF4D_BHM(9)
#undef MF4D_BHM
                default: return MF4D_EINVAL;
                }
            } else {
                const size_t lds = (size_t)64 * (taps[sc].ntaps + 65) * sizeof(float);
                hipLaunchKernelGGL(batch_hpass_kernel, dim3(pre[PT_HV][nact]), dim3(256), lds, s, imgs, P(PT_HV), nact,
                                   taps[sc], j);
            }
            BCHECK(hipGetLastError());
            if (const int nc = sweep_chunks(taps[sc])) {
                const int per_v = (pre[PT_VM][nact] + 7) / 8;
                switch (nc) {
#define MF4D_BVM(NC)                                                                                              \
    case NC:                                                                                                      \
        hipLaunchKernelGGL(batch_vpass_mfma_kernel<NC>, dim3(8 * per_v), dim3(256), vpass_mfma_lds(NC), s, imgs,      \
                           P(PT_VM), nact, taps[sc], sig * sig, inv2beta2, sc, per_v);                            \
        break;
                    MF4D_BVM(2) MF4D_BVM(3) MF4D_BVM(4) MF4D_BVM(5) MF4D_BVM(6) MF4D_BVM(7) MF4D_BVM(8) MF4D_BVM(9)
#undef MF4D_BVM
                default: return MF4D_EINVAL;
                }
            } else {
                hipLaunchKernelGGL(batch_vpass_kernel, dim3(pre[PT_HV][nact]), dim3(256), 0, s, imgs, P(PT_HV), nact,
                                   taps[sc], sig * sig, inv2beta2, sc);
            }
            BCHECK(hipGetLastError());
        }
        if (k == 0 || p.reselect_each_cycle) {   // otherwise the indices of the first cycle are kept
            hipLaunchKernelGGL(batch_argmax_kernel, dim3(pre[PT_PX][nact]), dim3(256), 0, s, imgs, P(PT_PX), nact, ns,
                               p.c);
            BCHECK(hipGetLastError());
        }
        switch (rt.r) {
#define MF4D_BRHO(R)                                                                                           \
    case R:                                                                                                    \
        hipLaunchKernelGGL(batch_rho_kernel<R>, dim3(pre[PT_RHO][nact]), dim3(256), 0, s, imgs, P(PT_RHO), nact, ns, \
                           rt, inv_lam2);                                                                      \
        break;
            MF4D_BRHO(0) MF4D_BRHO(1) MF4D_BRHO(2) MF4D_BRHO(3) MF4D_BRHO(4) MF4D_BRHO(5) MF4D_BRHO(6)
            MF4D_BRHO(7) MF4D_BRHO(8)
#undef MF4D_BRHO
        default: return MF4D_EINVAL;
        }
        BCHECK(hipGetLastError());
        for (int i0 = 0, l = 0; l < lpc; ++l) {
            const int steps = std::min(b->spl, b->n - i0);
            FedTaus ft{};
            for (int q = 0; q < steps; ++q) ft.t[q] = b->tau32[i0 + q];
            const int total = pre[PT_ST1 + steps - 1][nact];
            const int per = (total + 7) / 8;
            const int *pt = P(PT_ST1 + steps - 1);
            launch_batch_stream(b->cols[steps], steps, dim3(8 * per), s, imgs, pt, nact, ft, j, per);
            BCHECK(hipGetLastError());
            i0 += steps;
            ++j;
        }
    }
    return MF4D_OK;
}

// Uploads the tables for (in, out, ws) and records the batch into a graph.
int prepare(mf4d_batch *b, const float *in, float *out, char *ws, hipStream_t stream)
{
    std::vector<int> pre[PT_COUNT];
    build_tables(b, in, out, ws, pre);
    drop_graph(b);
    BCHECK(hipMemcpyAsync(ws, b->host_tables.data(), b->table_bytes, hipMemcpyHostToDevice, stream));
    BCHECK(hipStreamSynchronize(stream));
    hipStream_t cs;
    BCHECK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    int st = MF4D_OK;
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) st = MF4D_EHIP;
    if (st == MF4D_OK) st = enqueue_batch(b, ws, pre, cs);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &g);
    if (st == MF4D_OK && e != hipSuccess) st = MF4D_EHIP;
    if (st == MF4D_OK && hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) st = MF4D_EHIP;
    if (st == MF4D_OK) {
        b->graph = g;
        b->have_graph = true;
        b->g_in = in;
        b->g_out = out;
        b->g_ws = ws;
    } else if (g) {
        hipGraphDestroy(g);
    }
    hipStreamDestroy(cs);
    return st;
}

bool same_shared(const mf4d_params &a, const mf4d_params &b)
{
    if (a.nscales != b.nscales) return false;
    for (int k = 0; k < a.nscales; ++k)
        if (a.sigmas[k] != b.sigmas[k]) return false;
    return a.lambda == b.lambda && a.rho == b.rho && a.beta == b.beta && a.c == b.c &&
           a.substeps == b.substeps && a.stop_time == b.stop_time && a.tau_max == b.tau_max &&
           a.reselect_each_cycle == b.reselect_each_cycle && a.postprocess == b.postprocess &&
           (a.substeps > 0 || a.cycles == b.cycles);
}

}  // namespace

extern "C" {

int mf4d_batch_create(int nimg, const int64_t *offsets, const int *H, const int *W, const mf4d_params *per_image,
                      mf4d_batch **plan)
{
    if (!plan) return MF4D_EINVAL;
    *plan = nullptr;
    if (nimg < 1 || !offsets || !H || !W || !per_image) return MF4D_EINVAL;
    for (int i = 0; i < nimg; ++i) {
        if (validate_params(H[i], W[i], &per_image[i]) != MF4D_OK) return MF4D_EINVAL;
        if (per_image[i].model != MF4D_MAFOD || per_image[i].postprocess != 0 || per_image[i].check != 0)
            return MF4D_EINVAL;
        if (offsets[i] < 0 || !same_shared(per_image[0], per_image[i])) return MF4D_EINVAL;
    }
    // images must not overlap in the packed buffer
    std::vector<int> byoff(nimg);
    for (int i = 0; i < nimg; ++i) byoff[i] = i;
    std::sort(byoff.begin(), byoff.end(), [&](int a, int c) { return offsets[a] < offsets[c]; });
    for (int r = 1; r < nimg; ++r) {
        const int a = byoff[r - 1];
        if (offsets[a] + (int64_t)H[a] * W[a] > offsets[byoff[r]]) return MF4D_EINVAL;
    }
    mf4d_batch *b = new mf4d_batch();
    b->nimg = nimg;
    b->off.assign(offsets, offsets + nimg);
    b->H.assign(H, H + nimg);
    b->W.assign(W, W + nimg);
    for (int i = 0; i < nimg; ++i) {
        b->mode.push_back(per_image[i].mode);
        b->cycles.push_back(per_image[i].cycles);
    }
    b->shared = per_image[0];
    for (int q = 1; q <= 4; ++q) b->cols[q] = stream_cols_per_lane(q);
    b->sigmas.assign(per_image[0].sigmas, per_image[0].sigmas + per_image[0].nscales);
    b->shared.sigmas = b->sigmas.data();
    b->max_cycles = *std::max_element(b->cycles.begin(), b->cycles.end());
    std::vector<double> ordered;
    if (b->max_cycles > 0) {
        mf4d_params q = b->shared;
        q.cycles = b->max_cycles;
        if (fed_plan_host(&q, &b->n, ordered) != MF4D_OK) {
            delete b;
            return MF4D_EINVAL;
        }
    }
    for (double t : ordered) b->tau32.push_back((float)t);
    b->order.resize(nimg);
    for (int i = 0; i < nimg; ++i) b->order[i] = i;
    std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) { return b->cycles[a] > b->cycles[c]; });
    b->table_bytes = al256(sizeof(BImg) * nimg) + al256(sizeof(int) * PT_COUNT * (nimg + 1));
    size_t off = b->table_bytes;
    for (int r = 0; r < nimg; ++r) {
        const int i = b->order[r];
        b->img_ws.push_back(off);
        off += al256(image_workspace_bytes(H[i], W[i], b->shared.nscales));
    }
    b->ws_total = off;
    *plan = b;
    return MF4D_OK;
}

size_t mf4d_batch_workspace_bytes(const mf4d_batch *plan) { return plan ? plan->ws_total : 0; }

int mf4d_batch_destroy(mf4d_batch *plan)
{
    if (!plan) return MF4D_EINVAL;
    drop_graph(plan);
    delete plan;
    return MF4D_OK;
}

int mf4d_filter_batch(mf4d_batch *plan, const float *packed_in, float *packed_out, void *ws, size_t ws_bytes,
                      void *stream)
{
    if (!plan || !packed_in || !packed_out || !ws) return MF4D_EINVAL;
    if (ws_bytes < plan->ws_total) return MF4D_ENOMEM;
    hipStream_t s = (hipStream_t)stream;
    if (!plan->have_graph || plan->g_in != packed_in || plan->g_out != packed_out || plan->g_ws != ws) {
        const int st = prepare(plan, packed_in, packed_out, (char *)ws, s);
        if (st != MF4D_OK) return st;
    }
    BCHECK(hipGraphLaunch(plan->exec, s));
    return MF4D_OK;
}

int mf4d_batch_get_tuning(const mf4d_batch *plan, int *substeps_per_launch, int *rows_per_wave)
{
    if (!plan) return MF4D_EINVAL;
    if (substeps_per_launch) *substeps_per_launch = plan->spl;
    if (rows_per_wave) *rows_per_wave = plan->rows[plan->spl];
    return MF4D_OK;
}

int mf4d_batch_set_tuning(mf4d_batch *plan, int substeps_per_launch, int rows_per_wave)
{
    if (!plan || substeps_per_launch < 1 || substeps_per_launch > 4 || rows_per_wave < 0 || rows_per_wave > 4096)
        return MF4D_EINVAL;
    plan->spl = substeps_per_launch;
    for (int s = 1; s <= 4; ++s) plan->rows[s] = rows_per_wave;
    drop_graph(plan);
    return MF4D_OK;
}

int mf4d_batch_autotune(mf4d_batch *plan, void *ws, size_t ws_bytes, void *stream)
{
    if (!plan || !ws) return MF4D_EINVAL;
    if (ws_bytes < plan->ws_total) return MF4D_ENOMEM;
    if (plan->n < 1) return MF4D_OK;
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    const int N = plan->nimg;
    // scratch state: every image filters its own workspace planes (contents
    // are overwritten; values do not affect the kernel's timing)
    const int cand_spl[] = {2, 3, 4};
    const int cand_rows[] = {0, 48, 64, 96, 128, 192, 256};
    hipEvent_t e0, e1;
    BCHECK(hipEventCreate(&e0));
    BCHECK(hipEventCreate(&e1));
    float best = INFINITY;
    int best_spl = plan->spl, best_rows = 0;
    for (int spl : cand_spl) {
        for (int rows : cand_rows) {
            plan->spl = spl;
            for (int q = 1; q <= 4; ++q) plan->rows[q] = rows;
            std::vector<int> pre[PT_COUNT];
            // image buffers inside the workspace: in = out = tmp region of hA planes
            build_tables(plan, nullptr, nullptr, w, pre);
            BImg *imgs = (BImg *)plan->host_tables.data();
            for (int r = 0; r < N; ++r) {
                imgs[r].in = imgs[r].user_in = imgs[r].hA;
                imgs[r].out = imgs[r].hA + (size_t)imgs[r].H * imgs[r].W;
                imgs[r].copy_in = imgs[r].copy_out = 0;
            }
            BCHECK(hipMemcpyAsync(w, plan->host_tables.data(), plan->table_bytes, hipMemcpyHostToDevice, s));
            BCHECK(hipStreamSynchronize(s));
            const int *tab = (const int *)(w + al256(sizeof(BImg) * N));
            const int steps = std::min(spl, plan->n);
            const int *pt = tab + (PT_ST1 + steps - 1) * (N + 1);
            const int total = pre[PT_ST1 + steps - 1][N];
            const int per = (total + 7) / 8;
            FedTaus ft{};
            for (int q = 0; q < steps; ++q) ft.t[q] = plan->tau32[q];
            auto launch = [&](int j) {
                launch_batch_stream(plan->cols[steps], steps, dim3(8 * per), s, (const BImg *)w, pt, N, ft, j, per);
            };
            launch(1);
            launch(2);
            BCHECK(hipEventRecord(e0, s));
            const int reps = 6;
            for (int q = 0; q < reps; ++q) launch(1 + q);
            BCHECK(hipEventRecord(e1, s));
            BCHECK(hipEventSynchronize(e1));
            float ms = 0.f;
            BCHECK(hipEventElapsedTime(&ms, e0, e1));
            const float per_substep = ms / (reps * steps);
            if (per_substep < best) {
                best = per_substep;
                best_spl = spl;
                best_rows = rows;
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    plan->spl = best_spl;
    for (int q = 1; q <= 4; ++q) plan->rows[q] = best_rows;
    drop_graph(plan);
    return MF4D_OK;
}

}  // extern "C"
