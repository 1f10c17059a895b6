// Internal declarations shared by the HIP translation units of libmf4d.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/mf4d.h"

namespace mf4d {

constexpr int kMaxR = MF4D_MAX_RADIUS;   // Gaussian radius limit
constexpr int kMaxRhoR = 8;              // integration-scale radius limit (0: none)

// Full-width tap tables for the register-window passes: entry t holds the
// tap at offset t - R (R = r + 1), zero-padded to a multiple of kWin.
constexpr int kWin = 16;
constexpr int kMaxTaps = ((2 * (kMaxR + 1) + 1 + kWin - 1) / kWin) * kWin;
struct WinTaps {
    int R;       // r + 1
    int ntaps;   // padded tap count, multiple of kWin
    float gsum;  // sum of the float32 Gaussian taps
    float g[kMaxTaps];
    float d1[kMaxTaps];
    float d2[kMaxTaps];
};

// Step sizes of the substeps of one streaming launch.
struct FedTaus {
    float t[4];
};

struct RhoTaps {
    int r;  // 0: identity
    float g[kMaxRhoR + 1];
};

// Per-scale planes written by the scale sweep.
struct ScalePlanes {
    float *SA;  // [H][W][2] per pixel: Frobenius norm S of sigma^2 H(u_sigma), blob factor
                //   exp(-R_B^2 / 2 beta^2) (0 if the sign test fails)
    float *N;   // [H][W][3] H(u_sigma) / sqrt(1 + |grad u_sigma|) per pixel, or nullptr
};

// Horizontal pass of one scale: A = G u, B = D1G u, C = D2G u along x.
hipError_t launch_hpass(const float *u, float *A, float *B, float *C, int H, int W,
                        const WinTaps &t, hipStream_t s);

// Vertical pass of one scale plus the per-pixel vesselness ingredients.
hipError_t launch_vpass(const float *A, const float *B, const float *C, int H, int W,
                        const WinTaps &t, float sigma, int mode, float beta, ScalePlanes out,
                        unsigned *smax_bits, hipStream_t s);

// Matrix-core chunk count (K / 16) used for a scale's passes, 0 for the
// register-window passes (radius beyond the matrix-core tiles, or the
// environment variable MF4D_SWEEP=valu).
int sweep_chunks(const WinTaps &t);
// How a scale's two passes run: one fused matrix-core kernel, two
// matrix-core kernels (MF4D_SWEEP=split, or too many chunks for the fused
// kernel's LDS), or the register-window kernels.
enum { kSweepFused = 0, kSweepSplit = 1, kSweepValu = 2 };
int sweep_engine(const WinTaps &t);
// Which 32 x 32 blocks (the fused sweep's strip width and step) need a
// scale: bit `scale` of bits[by * bx + bx_index]; bits == nullptr: all.
struct ScaleNeed {
    const uint8_t *bits;
    int bx;
    int scale;
};
// Both passes of one scale (the planes hA, hB, hC are used by the split and
// register-window forms only); `shared`: other scales run concurrently. The
// fused kernel skips workgroups whose blocks do not need the scale (the
// other forms compute every block).
hipError_t launch_sweep_scale(const float *u, float *hA, float *hB, float *hC, int H, int W, const WinTaps &t,
                              float sigma, int mode, float beta, ScalePlanes out, unsigned *smax_bits, bool shared,
                              hipStream_t s, ScaleNeed need = ScaleNeed{nullptr, 0, 0});
// Rows per workgroup of the single-image fused kernel (MF4D_VSEG_ROWS
// overrides it; values do not change). `shared`: other scales run concurrently.
int fused_seg_rows(int H, int W, int nc, bool shared);
// Rows per workgroup of the single-image matrix-core vertical pass (the
// environment variable MF4D_VSEG_ROWS overrides it; values do not change).
int vpass_seg_rows(int H, int W);

hipError_t launch_fill_u32(unsigned *p, unsigned v, size_t n, hipStream_t s);
hipError_t launch_copy_f32(const float *src, float *dst, size_t n, hipStream_t s);

// Argmax over scales and/or normalised Hessian integration at the chosen scale.
//   idx_in  != nullptr: use these indices (no argmax)
//   idx_out != nullptr: write indices (tile interior)
//   hrho    != nullptr: write H_rho
//   coef    != nullptr: write the compact tensor planes (m, al, be) of H_rho
struct SelectArgs {
    const float *SA;     // [ns][H][W][2]: S and the blob factor per pixel
    const float *N;      // [ns][H][W][3]
    int ns;
    const unsigned *smax_bits;
    float c_param;
    const uint8_t *idx_in;
    uint8_t *idx_out;
    float *vmax_out;
    float *c_out;
    float *hrho;
    float *coef;
    int mode;
    float inv_lam2;
    RhoTaps rho;
    unsigned *smax_reset;   // nullable: the integration kernel sets it to 0 (the argmax has read it by then)
};
hipError_t launch_select(const SelectArgs &a, int H, int W, hipStream_t s);

// One FED substep u_out = u_in - tau L^T D L u_in with D from H_rho.
hipError_t launch_fed_substep(const float *u_in, float *u_out, const float *hrho, int H, int W,
                              float tau, int mode, float inv_lam2, hipStream_t s);

// `steps` (1..4) consecutive substeps with taus[0..steps-1], one wave per
// 64 c - 4 steps columns x seg_rows rows (c = stream_cols_per_lane(steps)),
// intermediate images in registers. Both forms give the same values;
// MF4D_STREAM_COLS=1 or 2 forces one.
int stream_cols_per_lane(int steps);
// Resident blocks per CU of that kernel for `steps`, and the CU count.
int stream_blocks_per_cu(int steps, int *cus);
constexpr int kStreamUnroll = 24;   // rows per unrolled block of the streaming kernels
hipError_t launch_fed_stream(const float *u_in, float *u_out, const float *coef, int H, int W, int steps,
                             const float *taus, int seg_rows, hipStream_t s);

// Integration with G_rho and tensor planes only: N at the chosen scale is
// gathered through idx_in (else idx_out).
hipError_t launch_rho(const SelectArgs &a, int H, int W, hipStream_t s);

// Learned surrogate (learned.hip): network forward on one H x W image into
// `ws` (net_forward_bytes(H, W) bytes) with the last layer reduced per pixel
// to one byte in *sel: the network's scale among the first min(ns, 8), bit 7
// set where its confidence reaches thr (the weights are packed from theta when
// `pack`, else those of an earlier call with the same ws are used); and the
// learned selection (that scale where confident, the exact argmax elsewhere;
// counts the fallback pixels into *fallback).
int net_select_into(const float *theta, const float *u, int H, int W, char *ws, hipStream_t s, float thr, int ns,
                    const uint8_t **sel, bool pack);
size_t net_forward_bytes(int H, int W);
// fallback: kFallbackSlots counters, summed into *total by launch_fallback_sum
constexpr int kFallbackSlots = 64;
hipError_t launch_learned_select(const uint8_t *sel, const SelectArgs &a, int H, int W, unsigned *fallback,
                                 hipStream_t s);
// Need bits of the learned selection: a 32 x 32 block needs scale s when one
// of its pixels is not confident (the exact argmax reads every scale there)
// or the network chose s for it. need: [ceil(H/32)][ceil(W/32)] bytes.
hipError_t launch_need_flags(const uint8_t *sel, int H, int W, int ns, uint8_t *need, hipStream_t s);
hipError_t launch_fallback_sum(const unsigned *slots, unsigned *total, hipStream_t s);

// ------------------------------------------------------------ aux_kernels.hip
// Per-call device state of the stability monitor and of l2-optimal stopping
// (kept in the workspace; reset by launch_monitor_reset at the start of a call).
struct MonitorState {
    double prev;          // squared l2 norm after the last monitored cycle
    double best;          // smallest distance to the ground truth so far
    unsigned nonfinite;   // a non-finite value was seen
    unsigned growth;      // a cycle grew the l2 norm beyond the tolerance
    unsigned take;        // the last stopping step improved on the best
    int best_k;
};
constexpr int kRedBlocks = 1024;   // partial sums of one l2 reduction (FP64)
enum { kMonitorInit = 0, kMonitorCycle = 1, kStopStep = 2 };
struct ScaleTable {
    float s[MF4D_MAX_SCALES];
};
hipError_t launch_monitor_reset(MonitorState *st, hipStream_t s);
// sum of d^2 over m values (d = u, or u - ref), then the bookkeeping `what`
// (step k of a stopping run writes l2_out[k] and *best_out)
hipError_t launch_l2(const float *u, const float *ref, size_t m, double *partial, MonitorState *st, int what,
                     float growth_tol, int k, double *l2_out, int *best_out, hipStream_t s);
hipError_t launch_take_copy(const float *src, float *dst, size_t m, const MonitorState *st, hipStream_t s);
// isotropic model: g planes (g, 0, 0) from the horizontal planes of one scale
hipError_t launch_ifod_coef(const float *A, const float *B, const float *C, int H, int W, const WinTaps &t,
                            float inv_lam2, float *coef, float *hess, hipStream_t s);
hipError_t launch_postprocess(const uint8_t *idx, const float *vmax, const float *N, int ns, int H, int W,
                              const ScaleTable &sig, float theta, int tmax, uint8_t *out, hipStream_t s);

// ---------------------------------------------------------- crease_kernels.hip
// planes [6][H][W]: g_x, g_y, h_xx, h_xy, h_yy, d = det(g | Hg) of u_sigma,
// from the horizontal planes of one scale
hipError_t launch_crease_field(const float *A, const float *B, const float *C, int H, int W, const WinTaps &t,
                               float *planes, hipStream_t s);
hipError_t launch_marching(const float *planes, int H, int W, float strength, int mode, float *seg, int8_t *type,
                           unsigned *count, hipStream_t s);
hipError_t launch_crease_match(const float *seg, const int8_t *type, int H, int W, const float *gt, const int *gt_type,
                               int n, float radius, float *dist, int *match, hipStream_t s);

// ------------------------------------------------- host helpers (mf4d_api.hip)
// parameter checks of mf4d_filter for an H x W image
int validate_params(int H, int W, const mf4d_params *p);
size_t image_workspace_bytes(int H, int W, int ns);
void image_workspace(int H, int W, int ns, char *base, float **hA, float **SA, float **N,
                     uint8_t **idx, float **tens, float **utmp, unsigned **smax);
// combined taps (G, D1 G, D2 G) of a scale, and the integration taps
void window_taps(double sigma, WinTaps *t);
void rho_taps(double rho, RhoTaps *t);
// the ordered FED steps mf4d_fed_plan returns for p
int fed_plan_host(const mf4d_params *p, int *n_out, std::vector<double> &ordered);
int default_stream_rows(int H, int W, int steps);

}  // namespace mf4d
