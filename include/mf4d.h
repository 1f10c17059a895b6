/*
 * mf4d -- multi-scale anisotropic fourth-order diffusion (MAFOD) on MI355X.
 *
 * C ABI of the GPU library libmf4d.so (HIP, gfx950). The library computes the
 * hot path of the MAFOD ridge/valley filter: a per-pixel Gaussian scale chosen
 * by Frangi vesselness, the normalised integrated Hessian at that scale, and
 * Fast Explicit Diffusion (FED) cycles of the fourth-order anisotropic PDE.
 * Section, equation and table numbers refer to the paper (arXiv:1611.06906).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Images are contiguous row-major float32 [H][W] in DEVICE memory, x = column
 *    (the paper's index i), y = row (index j), pixel spacing 1. The caller owns
 *    all buffers; the library never allocates or frees caller memory. Scratch
 *    space comes from a caller-provided device workspace of at least
 *    mf4d_workspace_bytes() bytes; the one exception is mf4d_filter_noalloc,
 *    whose scratch is a fixed array the library keeps on each GPU.
 *  - mf4d_params, its sigmas array and all double* schedule arrays are HOST
 *    memory; they are read during the call only.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Device work is enqueued asynchronously on it; results are ready when the
 *    stream is synchronised. Calls on different streams must use different
 *    workspaces and outputs.
 *  - Every function returns an int status (MF4D_OK = 0 or a negative code).
 *    Arguments are validated on the host before anything is enqueued; on an
 *    error nothing is enqueued. No exceptions cross the ABI.
 *  - The only state the library keeps is, per host thread and device, three
 *    non-blocking side streams and their events (default priority), created
 *    on the first multi-scale call and kept until the process ends. The
 *    scales of a cycle are forked onto them from `stream` with events and
 *    joined back before anything else is enqueued, so the calls keep the
 *    ordering of `stream`. The environment variable MF4D_FORK=0 keeps all
 *    work on `stream`; if the side streams cannot be created, the thread
 *    keeps all work on `stream` from then on. A call enqueues only kernels
 *    and event edges, so it can be recorded into a hipGraph; make one
 *    eager multi-scale call on the thread first, so that the side streams
 *    are not created during the capture. Calls are thread-safe for distinct
 *    streams and workspaces.
 */
#ifndef MF4D_H
#define MF4D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MF4D_OK 0
#define MF4D_EINVAL (-1)   /* invalid argument (checked before any launch)   */
#define MF4D_ENOMEM (-2)   /* workspace smaller than mf4d_workspace_bytes()  */
#define MF4D_EHIP (-3)     /* a HIP launch or runtime call failed            */
#define MF4D_ENONFINITE (-4) /* check on: u held a non-finite value          */
#define MF4D_EUNSTABLE (-5)  /* check on: a cycle grew the l2 norm of u      */

/* Crease type to enhance (Sec. 3.2, text after Eq. (7); Sec. 3.3 Eq. (9)). */
#define MF4D_RIDGE 0       /* mu_i = 1 where nu_i >= 0; V = 0 where nu~_2 > 0 */
#define MF4D_VALLEY 1      /* mu_i = 1 where nu_i <= 0; V = 0 where nu~_2 < 0 */
#define MF4D_BOTH 2        /* no mask, no sign test (the paper's default)    */

/* Diffusion model (params.model). */
#define MF4D_MAFOD 0       /* anisotropic tensor of Eqs. (7), (8) at the selected scales */
#define MF4D_IFOD 1        /* isotropic: D = g(||H(u_sigma)||_F^2) Id, Eq. (4) with Eq. (1) */

#define MF4D_MAX_SCALES 16
#define MF4D_MAX_RADIUS 64 /* Gaussian radius max(1, ceil(3 sigma)) limit   */
#define MF4D_MAX_SUBSTEPS 1024

/* Filter parameters, in the paper's notation. Zero-initialise the struct (or
 * use mf4d_params_default) so that fields added at its end stay 0.
 *   nscales, sigmas  scale set {sigma_min..sigma_max} of Sec. 3.3; host array,
 *                    strictly ascending, > 0, radius ceil(3 sigma) <= 64.
 *   mode             MF4D_RIDGE / MF4D_VALLEY / MF4D_BOTH.
 *   lambda           Perona-Malik contrast parameter of Eq. (7); > 0, +inf
 *                    allowed (linear isotropic fourth-order diffusion).
 *   rho              integration scale of Eq. (6); >= 0 (0: no integration).
 *                    The paper uses 0.5.
 *   beta, c          Frangi parameters of Eq. (9); beta > 0 (paper: 0.5);
 *                    c <= 0 selects the paper's c = max(S)/2, taken over all
 *                    scales and pixels of the image; c > 0 is used as given.
 *   cycles           number of FED cycles M >= 0 (Eq. (21)).
 *   substeps         n >= 1 substeps per cycle (then T/M = tau_max (n^2+n)/3),
 *                    or 0 to derive n from stop_time by Eq. (22).
 *   stop_time        diffusion stopping time T (used when substeps == 0).
 *   tau_max          stable explicit step, 0 < tau_max <= 1/17 (Eq. (20)).
 *   reselect_each_cycle  1: scales re-selected on u^k every cycle; 0: once on
 *                    u^0 (the Hessian is still re-formed from u^k each cycle).
 *   theta, postprocess   scale-image postprocessing of Sec. 3.3 (text after
 *                    Eq. (9)): postprocess = 1 re-assigns every pixel whose
 *                    max_s V_s >= theta the scale nearest to the mean sigma of
 *                    its cross-section (a march in unit steps, up to
 *                    ceil(3 sigma_max) on each side, across the crease along
 *                    the eigenvector of the stronger eigenvalue of the
 *                    Hessian at the pixel's scale, through vessel pixels
 *                    only; offsets rounded half away from zero; ties to the
 *                    smaller scale). 0: no postprocessing, theta unused.
 *   check            0: none. 1: after every cycle the l2 norm of u is taken
 *                    (FP64 sum) and compared with the previous one; the call
 *                    then synchronises `stream` and returns MF4D_ENONFINITE if
 *                    u (or the input) held a NaN or infinity, else
 *                    MF4D_EUNSTABLE if a cycle grew ||u||_2 by more than a
 *                    relative 1e-5 (exact arithmetic forbids any growth:
 *                    each FED cycle is a contraction for tau_max <= 1/17,
 *                    Sec. 3.4). The environment variable
 *                    MF4D_L2_GROWTH_TOL overrides 1e-5 (a negative value
 *                    forces the growth report, for tests of the error path).
 *                    A call with check = 1 cannot be recorded into a graph.
 *   model            MF4D_MAFOD, or MF4D_IFOD: the isotropic fourth-order
 *                    model of Eq. (4) with g of Eq. (1) on the squared
 *                    Frobenius norm of the Hessian of u_sigma, sigma =
 *                    sigmas[0] (nscales must be 1; mode, rho, beta, c,
 *                    postprocess unused), frozen over each FED cycle.
 */
typedef struct mf4d_params {
    int nscales;
    const float *sigmas;
    int mode;
    float lambda;
    float rho;
    float beta;
    float c;
    int cycles;
    int substeps;
    double stop_time;
    double tau_max;
    int reselect_each_cycle;
    float theta;
    int postprocess;
    int check;
    int model;
} mf4d_params;

/* Human-readable text for a status code. Never NULL. */
const char *mf4d_status_string(int status);

/* Fills *p with the paper's defaults (rho = beta = 0.5, c automatic,
 * tau_max = 0.05, lambda = 0.005, BOTH, reselect each cycle) for the given
 * scale set. Returns MF4D_EINVAL if p is NULL. */
int mf4d_params_default(mf4d_params *p, int nscales, const float *sigmas);

/* ------------------------------------------------------------------ host */

/* FED steps of one cycle, Sec. 3.5 Eq. (23), for n given substeps and
 * T/M = tau_max (n^2+n)/3, i.e. tau_i = tau_max / (2 cos^2(pi (2i+1)/(4n+2))),
 * written to taus_out[0..n-1] (host) in the order they are applied: position j
 * holds tau_{pi(j)} with pi(j) = (kappa j) mod n, kappa the value in [1, n-1]
 * coprime to n that minimises the largest partial-product amplification of
 * the cycle (the paper names kappa-cycle reordering without defining it; this
 * rule is the library's reading). perm_out (nullable) receives pi.
 * Returns kappa (>= 1), or MF4D_EINVAL (n outside [1, MF4D_MAX_SUBSTEPS],
 * tau_max outside (0, 1/17], NULL taus_out). */
int mf4d_fed_schedule(int n, double tau_max, double *taus_out, int *perm_out);

/* Substeps per cycle from the stopping time, Eq. (22). Returns n >= 1 or
 * MF4D_EINVAL (T <= 0, M < 1, bad tau_max, or n > MF4D_MAX_SUBSTEPS). */
int mf4d_fed_substeps(double stop_time, int cycles, double tau_max);

/* Ordered steps for the schedule mf4d_filter will use with these params
 * (Eq. (22) and Eq. (23) when substeps == 0). Writes *n_out; taus_out
 * (nullable) must hold MF4D_MAX_SUBSTEPS doubles. Returns MF4D_OK or
 * MF4D_EINVAL. */
int mf4d_fed_plan(const mf4d_params *p, int *n_out, double *taus_out);

/* Bytes of device workspace needed by mf4d_scale_select, mf4d_tensor and
 * mf4d_filter for an H x W image and these params (0 if invalid). */
size_t mf4d_workspace_bytes(int H, int W, const mf4d_params *p);

/* ---------------------------------------------------------------- device */

/* Scale selection, Sec. 3.3 Eq. (9). For every scale sigma_s the Hessian of
 * u_sigma = u * G_sigma (sampled Gaussian, radius max(1, ceil(3 sigma)),
 * symmetric extension at the border, central differences as in Sec. 3.4) is
 * scale-normalised by sigma^2; S, R_B and the vesselness V_s follow Eq. (9)
 * with c = max over all scales and pixels of S / 2 (or params->c when > 0).
 * The filter products run on the matrix cores at FP32 accuracy: FP32 MFMA,
 * or split BF16 (each value the exact sum of three BF16 parts, six part
 * products, FP32 accumulation), so results match an FP64 evaluation to
 * FP32 rounding, not bit for bit.
 *   u        device, float32 [H][W], read only.
 *   idx_out  device, uint8 [H][W]: smallest s with V_s = max_t V_t, then the
 *            postprocessing of Sec. 3.3 when p->postprocess = 1.
 *   vmax_out device, float32 [H][W] (nullable): max_t V_t.
 *   c_out    device, one float32 (nullable): the c used.
 *   ws       device workspace of ws_bytes >= mf4d_workspace_bytes(H, W, p).
 * Errors: MF4D_EINVAL (bad sizes/params/NULL, or p->model = MF4D_IFOD),
 * MF4D_ENOMEM, MF4D_EHIP. */
int mf4d_scale_select(const float *u, int H, int W, const mf4d_params *p,
                      uint8_t *idx_out, float *vmax_out, float *c_out,
                      void *ws, size_t ws_bytes, void *stream);

/* Normalised, integrated Hessian, Eq. (6): for each pixel,
 * N = H(u_sigma) / sqrt(1 + |grad u_sigma|) at the pixel's scale idx[x,y],
 * then H_rho = G_rho * N per component (symmetric extension).
 *   u         device float32 [H][W]; idx device uint8 [H][W], values < nscales
 *             (larger values are clamped to nscales - 1).
 *   hrho_out  device float32 [3][H][W]: planes (a, b, d) = (xx, xy, yy).
 *   dparams_out (nullable) device float32 [3][H][W]: the fourth-order tensor of
 *             Eqs. (7), (8) in the compact form acting on a symmetric H as
 *             T_xx = (m+al) h_xx + be h_xy, T_xy = m h_xy + be (h_xx+h_yy)/2,
 *             T_yy = (m-al) h_yy + be h_xy; planes (m, al, be), where
 *             m = (mu_1+mu_2)/2 and (al, be) = (mu_1-mu_2)/2 (cos 2t, sin 2t)
 *             for the angle t of the first eigenvector of H_rho.
 * With p->model = MF4D_IFOD, idx is not read (may be NULL), hrho_out
 * receives the Hessian (h_xx, h_xy, h_yy) of u_sigma at sigma = sigmas[0]
 * and dparams_out the planes (g, 0, 0) of D = g Id.
 * Errors as mf4d_scale_select (IFOD allowed). */
int mf4d_tensor(const float *u, int H, int W, const uint8_t *idx, const mf4d_params *p,
                float *hrho_out, float *dparams_out,
                void *ws, size_t ws_bytes, void *stream);

/* One FED cycle, Eq. (21): n explicit steps u <- (I - tau P) u with
 * P = L^T D L frozen for the cycle (Sec. 3.4: Hajiaboli stencils, rows of L
 * only at interior pixels, D from H_rho by Eqs. (7), (8), lambda and mode
 * from p). taus (host, n doubles) are applied in the given order, each cast
 * to float32.
 *   u      device float32 [H][W], in/out: the result always lands here.
 *   u_tmp  device float32 [H][W] scratch (must not alias u).
 *   hrho   device float32 [3][H][W] from mf4d_tensor.
 * Errors: MF4D_EINVAL (also for p->model = MF4D_IFOD: use
 * mf4d_fed_cycle_tensor with the (g, 0, 0) planes), MF4D_EHIP. */
int mf4d_fed_cycle(float *u, float *u_tmp, int H, int W, const float *hrho,
                   const mf4d_params *p, const double *taus, int n, void *stream);

/* n FED substeps as mf4d_fed_cycle, but from the compact tensor planes
 * (dparams_out of mf4d_tensor) computed once for the cycle, so no substep
 * repeats the eigen-decomposition; the values are identical to those of
 * mf4d_fed_cycle given the H_rho the planes were built from.
 *   dparams          device float32 [3][H][W] planes (m, al, be).
 *   steps_per_launch 1..4: consecutive substeps per pass over the image
 *                    (intermediate images stay on chip), dividing the HBM
 *                    traffic per substep by steps_per_launch; same values.
 * Errors: MF4D_EINVAL, MF4D_EHIP. */
int mf4d_fed_cycle_tensor(float *u, float *u_tmp, int H, int W, const float *dparams,
                          const double *taus, int n, int steps_per_launch, void *stream);

/* The whole filter: M cycles of scale selection (Sec. 3.3), normalised
 * Hessian (Eq. (6)) and an FED cycle (Eq. (21)) with the schedule of
 * mf4d_fed_plan.
 *   u_in   device float32 [H][W], read only.
 *   u_out  device float32 [H][W]; may alias u_in.
 * Errors: MF4D_EINVAL, MF4D_ENOMEM, MF4D_EHIP, and with p->check = 1
 * MF4D_ENONFINITE / MF4D_EUNSTABLE (u_out then holds the last state). */
int mf4d_filter(const float *u_in, float *u_out, int H, int W, const mf4d_params *p,
                void *ws, size_t ws_bytes, void *stream);

/* mf4d_filter for callers that cannot allocate device memory (code under
 * hipGraph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation and the same values as mf4d_filter, with the scratch
 * taken from a fixed array of mf4d_noalloc_max_bytes() bytes (128 MiB) that
 * the library keeps on each GPU it runs on until the process ends, instead
 * of a workspace argument. The call allocates nothing (no hipMalloc, no
 * side streams: every scale runs on `stream`) and enqueues kernels only
 * (with p->check = 1 it also synchronises and copies the status back, as
 * mf4d_filter does). All calls on one GPU share that array: calls that
 * overlap in time on one GPU (other streams, other host threads) race and
 * must be serialised by the caller. Everything a call reads from the array
 * it first writes (or clears) itself.
 * Errors: MF4D_EINVAL, MF4D_ENOMEM (mf4d_workspace_bytes(H, W, p) exceeds
 * mf4d_noalloc_max_bytes()), MF4D_EHIP, and with p->check = 1
 * MF4D_ENONFINITE / MF4D_EUNSTABLE. */
int mf4d_filter_noalloc(const float *u_in, float *u_out, int H, int W, const mf4d_params *p,
                        void *stream);

/* Bytes of the fixed scratch array of mf4d_filter_noalloc. */
size_t mf4d_noalloc_max_bytes(void);

/* The filter with l2-optimal stopping against a noise-free image (Sec. 4:
 * the evolution is stopped where the l2 difference between the filtered and
 * the noise-free image is smallest), evaluated at the ends of FED cycles,
 * the states the scheme defines (Eq. (21)). Runs p->cycles cycles.
 *   ground_truth  device float32 [H][W], the noise-free image.
 *   u_out         device float32 [H][W], receives u^k* (must not alias u_in or
 *                 ground_truth).
 *   l2_out        device double [p->cycles + 1] (nullable): e_k = ||u^k - gt||_2,
 *                 u^0 = u_in (sum in FP64 of the FP32 differences).
 *   best_out      device int (nullable): k* = the smallest k of minimal e_k.
 * Everything stays on the device (no synchronisation), so a call can be
 * recorded into a graph; p->check = 1 is honoured as in mf4d_filter.
 * Errors as mf4d_filter. */
int mf4d_filter_l2stop(const float *u_in, float *u_out, int H, int W, const mf4d_params *p,
                       const float *ground_truth, double *l2_out, int *best_out,
                       void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------ crease extraction */

/* Device workspace bytes of mf4d_creases for an H x W image (0 if invalid). */
size_t mf4d_creases_workspace_bytes(int H, int W);

/* Creases of an (already filtered) image, Sec. 3.6: the zero contour of
 * d = det(g | Hg), g and H the gradient and Hessian of u_sigma (sigma =
 * sigma_d; the Gaussian, symmetric extension and central differences of
 * the scale stack), by marching squares on the pixel grid: a corner is
 * inside when d >= 0, crossings are interpolated linearly in d along each
 * edge, saddle cells are split by the sign of the mean of their corners.
 * The zero set of d is a superset of the creases; a segment is kept when H,
 * interpolated likewise, gives both ends the same type -- ridge where its
 * eigenvalue of larger magnitude is negative, valley where positive, that
 * magnitude >= strength -- allowed by mode (MF4D_RIDGE / MF4D_VALLEY /
 * MF4D_BOTH), and the segment runs closer to the eigenvector of the weaker
 * eigenvalue (at the mean Hessian of its ends) than to the other.
 *   u         device float32 [H][W].
 *   seg_out   device float32 [H-1][W-1][2][4]: per cell (x, y) (corners
 *             (x,y), (x+1,y), (x+1,y+1), (x,y+1); pixel centres at integer
 *             coordinates, x = column) up to two segments (x0, y0, x1, y1)
 *             in slots sorted by their first crossed edge (top, right,
 *             bottom, left); unused slots are zero.
 *   type_out  device int8 [H-1][W-1][2]: +1 ridge, -1 valley, 0 empty slot.
 *   count_out device uint32 (nullable): the number of segments is ADDED to it.
 *   field_out device float32 [6][H][W] (nullable): the planes g_x, g_y, h_xx,
 *             h_xy, h_yy, d.
 *   ws        device workspace of mf4d_creases_workspace_bytes(H, W) bytes.
 * Every slot is written, so the result does not depend on scheduling.
 * Errors: MF4D_EINVAL (H, W < 3, sigma_d outside (0, 21.3], strength < 0 or
 * not finite, bad mode, NULL), MF4D_ENOMEM, MF4D_EHIP. */
int mf4d_creases(const float *u, int H, int W, float sigma_d, float strength, int mode, float *seg_out,
                 int8_t *type_out, unsigned *count_out, float *field_out, void *ws, size_t ws_bytes,
                 void *stream);

/* Evaluation of extracted creases against ground-truth segments, Sec. 4:
 * each ground-truth segment gt[i] = (x0, y0, x1, y1) of type gt_type[i]
 * (+1 ridge, -1 valley) is matched to the segment of seg / type (as written
 * by mf4d_creases for an H x W image) of the same type with the least
 * directed Hausdorff distance from gt[i] (the largest distance of a point of
 * gt[i] to it), if that distance is at most radius (the neighbourhood: the
 * paper uses 6 px on synthetic data); ties go to the first cell in row-major
 * order, then slot 0. dist_out[i] = distance from gt[i]'s midpoint to its
 * match, -1 if none; match_out[i] = 2 * (y (W-1) + x) + slot, or -1. The mean
 * of the non-negative distances is the paper's E, their share its p.
 * All arrays are device memory; n >= 0. Errors: MF4D_EINVAL, MF4D_EHIP. */
int mf4d_crease_match(const float *seg, const int8_t *type, int H, int W, const float *gt, const int *gt_type,
                      int n, float radius, float *dist_out, int *match_out, void *stream);

/* ------------------------------------------------------------ volumes */

/* The filter on volumes, the 3-D extension the paper names as its next step
 * (Sec. 5), with every definition of the 2-D filter carried to three axes:
 *  - volumes are float32 [D][H][W] on the device, x fastest, unit spacing;
 *    D, H, W >= 3, D <= 65535, D H W < 2^31;
 *  - scale selection: the Hessian of u_sigma (separable Gaussian, central
 *    differences, the cross stencil of Sec. 3.4 in each coordinate plane for
 *    the mixed terms, symmetric extension) scaled by sigma^2, with
 *    eigenvalues n1, n2, n3 by ascending magnitude; Frangi's tube measure
 *    V = (1 - exp(-R_A^2 / 2 alpha^2)) exp(-R_B^2 / 2 beta^2)
 *    (1 - exp(-S^2 / 2 c^2)) with R_A = |n2|/|n3|, R_B = |n1|/sqrt|n2 n3|,
 *    S the Frobenius norm, alpha = 1/2, beta and c as in 2-D (c = half the
 *    largest S over all scales and voxels unless p->c > 0); V = 0 where
 *    n2 n3 = 0 or, in RIDGE (VALLEY) mode, where n2 or n3 is positive
 *    (negative); the smallest scale index of maximal V;
 *  - Eq. (6) per component: N = H(u_sigma) / sqrt(1 + |grad u_sigma|) at
 *    each voxel's scale, H_rho = G_rho * N (planes xx, yy, zz, xy, xz, yz);
 *  - the tensor: eigenpairs (nu_k, e_k) of H_rho, mu_k of Eq. (7) with the
 *    mode masks of Sec. 3.2; weight mu_k on e_k e_k^T, (mu_k + mu_l)/2 on the
 *    symmetric pairs, 0 on the antisymmetric ones;
 *  - P = L^T D L with the nine second-difference stencils, rows of L only at
 *    voxels whose 3x3x3 neighbourhood lies inside; its largest eigenvalue is
 *    at most 3 * 16 + 6 * 1 = 54, so 0 < tau_max <= 1/27.
 * Parameters are those of mf4d_params with tau_max <= 1/27, model =
 * MF4D_MAFOD, postprocess = 0, check = 0 and reselect_each_cycle = 1
 * (other values: MF4D_EINVAL). The eigen-solves (in BOTH mode, where every
 * mu_k is 1 / (1 + nu_k^2 / lambda^2), mostly the inverse of
 * I + H_rho^2 / lambda^2 instead) run in FP64, everything else in FP32. */

/* Device workspace bytes of the calls below for a D x H x W volume (0 if the
 * sizes or params are invalid). */
size_t mf4d3d_workspace_bytes(int D, int H, int W, const mf4d_params *p);

/* Scale selection over the stack (the tube measure above).
 *   u        device float32 [D][H][W], read only.
 *   idx_out  device uint8 [D][H][W]: smallest s of maximal V_s.
 *   vmax_out device float32 [D][H][W] (nullable): max_s V_s.
 *   c_out    device, one float32 (nullable): the c used.
 * Errors: MF4D_EINVAL, MF4D_ENOMEM (ws_bytes too small), MF4D_EHIP. */
int mf4d3d_scale_select(const float *u, int D, int H, int W, const mf4d_params *p, uint8_t *idx_out,
                        float *vmax_out, float *c_out, void *ws, size_t ws_bytes, void *stream);

/* Normalised, integrated Hessian at the scales idx (device uint8
 * [D][H][W], values >= nscales clamped to nscales - 1).
 *   hrho_out    device float32 [6][D][H][W]: xx, yy, zz, xy, xz, yz.
 *   dparams_out device float32 [D][H][W][6] (nullable): the tensor as
 *               mf4d3d_dtensor writes it.
 * Errors as mf4d3d_scale_select. */
int mf4d3d_tensor(const float *u, int D, int H, int W, const uint8_t *idx, const mf4d_params *p, float *hrho_out,
                  float *dparams_out, void *ws, size_t ws_bytes, void *stream);

/* The tensor of each voxel from its H_rho (device float32 [6][D][H][W]):
 * dparams_out device float32 [D][H][W][6], 6 values per voxel (8-byte
 * aligned base): the symmetric P = sum_k mu_k e_k e_k^T as xx, yy, zz, xy,
 * xz, yz (mu_k from lambda and mode of p). With the weights above, the
 * tensor's action on a symmetric h is (P h + h P) / 2, so P determines it.
 * Errors: MF4D_EINVAL (also for a base not 8-byte aligned), MF4D_EHIP. */
int mf4d3d_dtensor(const float *hrho, int D, int H, int W, const mf4d_params *p, float *dparams_out, void *stream);

/* n FED substeps (Eq. (21)) u <- u - tau_i L^T D L u, with D from dparams
 * (device float32 [D][H][W][6] as mf4d3d_dtensor writes it, 8-byte
 * aligned); taus host, n doubles in the order applied (each cast to
 * float32).
 *   u      device float32 [D][H][W], in/out: the result always lands here.
 *   u_tmp  device float32 [D][H][W] scratch (must not alias u).
 * Errors: MF4D_EINVAL (sizes, NULL, aliasing, n outside
 * [1, MF4D_MAX_SUBSTEPS], a tau not positive and finite), MF4D_EHIP. */
int mf4d3d_fed_cycle_tensor(float *u, float *u_tmp, int D, int H, int W, const float *dparams, const double *taus,
                            int n, void *stream);

/* The whole filter on a volume: M cycles of scale selection, integrated
 * Hessian, tensor and n FED substeps (the schedule of mf4d_fed_plan).
 *   u_in   device float32 [D][H][W], read only.
 *   u_out  device float32 [D][H][W]; may alias u_in.
 * Errors: MF4D_EINVAL, MF4D_ENOMEM, MF4D_EHIP. */
int mf4d3d_filter(const float *u_in, float *u_out, int D, int H, int W, const mf4d_params *p, void *ws,
                  size_t ws_bytes, void *stream);

/* ------------------------------------------------------------ batches */

/* A batch plan: many images of different sizes filtered together. Every
 * stage of the filter is one launch over all images of the batch and the
 * whole launch sequence is recorded once into a hipGraph that each
 * mf4d_filter_batch call replays; each image's result is identical to a
 * separate mf4d_filter call with its own parameters. */
typedef struct mf4d_batch mf4d_batch;

/* Creates a plan for nimg images packed in one device buffer: image i is
 * float32 [H[i]][W[i]] starting at element offsets[i] (images must not
 * overlap). per_image[i] are its filter parameters: mode and cycles may
 * differ between images; every other field (scales, lambda, rho, beta, c,
 * substeps, stop_time, tau_max, reselect_each_cycle) must equal image 0's
 * (with substeps == 0, cycles must match too). All arrays are host memory
 * and are copied. *plan receives the plan (destroy with mf4d_batch_destroy).
 * Batches run the anisotropic model without postprocessing or checks
 * (model, postprocess and check must be 0).
 * Errors: MF4D_EINVAL. */
int mf4d_batch_create(int nimg, const int64_t *offsets, const int *H, const int *W,
                      const mf4d_params *per_image, mf4d_batch **plan);

/* Device workspace bytes mf4d_filter_batch and mf4d_batch_autotune need. */
size_t mf4d_batch_workspace_bytes(const mf4d_batch *plan);

/* Runs the filter on every image of the plan. packed_in / packed_out are
 * device buffers laid out as given to mf4d_batch_create; packed_out may alias
 * packed_in. The first call for a given (packed_in, packed_out, ws) uploads
 * the plan's tables into ws, synchronises `stream` and records the graph;
 * later calls only launch the graph on `stream`. Calls on one plan must not
 * overlap. Errors: MF4D_EINVAL, MF4D_ENOMEM, MF4D_EHIP. */
int mf4d_filter_batch(mf4d_batch *plan, const float *packed_in, float *packed_out, void *ws,
                      size_t ws_bytes, void *stream);

/* Autotuner: times the fused substep kernel on the plan's shapes for each
 * candidate decomposition (substeps per launch 2..4, rows per wave) and keeps
 * the fastest in the plan; no result value depends on this choice. Uses ws
 * as scratch (its contents are overwritten) and synchronises `stream`.
 * Errors: MF4D_EINVAL, MF4D_ENOMEM, MF4D_EHIP. */
int mf4d_batch_autotune(mf4d_batch *plan, void *ws, size_t ws_bytes, void *stream);

/* Reads / sets the substep decomposition of a plan (substeps per launch 1..4,
 * rows per wave, 0 = default). Errors: MF4D_EINVAL. */
int mf4d_batch_get_tuning(const mf4d_batch *plan, int *substeps_per_launch, int *rows_per_wave);
int mf4d_batch_set_tuning(mf4d_batch *plan, int substeps_per_launch, int rows_per_wave);

/* Releases a plan and its recorded graph. Errors: MF4D_EINVAL (NULL). */
int mf4d_batch_destroy(mf4d_batch *plan);

/* ------------------------------------------------------ learned surrogate */

/* A small convolutional network standing in for the scale selection: five
 * 3x3 convolutions with zero padding, channels 1 -> 32 -> 32 -> 32 -> 32 -> 9,
 * ReLU between layers; outputs 8 scale logits and 1 confidence logit per
 * pixel. Products use BF16 weights and activations with FP32 accumulation on
 * the matrix cores. theta is the FP32 parameter vector (device memory): for
 * each layer W[cout][cin][3][3] then b[cout]. Images are [B][H][W] float32
 * with H and W multiples of 16. Not part of the paper: a project extension. */

/* Number of floats in theta. */
size_t mf4d_net_param_count(void);

/* Workspace bytes for B images of H x W (train != 0: also for the backward
 * pass); 0 if the shape is invalid. */
size_t mf4d_net_workspace_bytes(int B, int H, int W, int train);

/* Forward pass. logits (nullable): [B*H*W][16] float32 (entries 0..7 scale
 * logits, 8 confidence logit, 9..15 zero); idx_out (nullable): argmax of the
 * scale logits, uint8 [B][H][W]; conf_out (nullable): sigmoid of the
 * confidence logit, float32 [B][H][W]. Errors: MF4D_EINVAL, MF4D_ENOMEM,
 * MF4D_EHIP. */
int mf4d_net_forward(const float *theta, const float *u, int B, int H, int W, float *logits,
                     uint8_t *idx_out, float *conf_out, void *ws, size_t ws_bytes, void *stream);

/* Gradient of the training loss with respect to theta (written to grad,
 * device float32, param_count entries). Loss, averaged over pixels: softmax
 * cross-entropy of the scale logits against labels (uint8 [B][H][W], the
 * exact sweep's indices), plus w_conf times the binary cross-entropy of the
 * confidence against "the predicted scale is the label". stats_out
 * (nullable, device float32[2]): the loss and the fraction of correct
 * predictions. Errors: MF4D_EINVAL, MF4D_ENOMEM, MF4D_EHIP. */
int mf4d_net_backward(const float *theta, const float *u, const uint8_t *labels, int B, int H, int W,
                      float w_conf, float *grad, float *stats_out, void *ws, size_t ws_bytes, void *stream);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on theta with moment
 * buffers adam_m, adam_v (device float32, zero-initialised before step 1);
 * step counts from 1. Errors: MF4D_EINVAL, MF4D_EHIP. */
int mf4d_net_step(float *theta, const float *grad, float *adam_m, float *adam_v, int step, float lr,
                  void *stream);

/* Workspace bytes for mf4d_filter_learned (0 if invalid). */
size_t mf4d_learned_workspace_bytes(int H, int W, const mf4d_params *p);

/* The filter with the network's scale where its confidence reaches
 * conf_threshold (0..1) and the exact argmax of Eq. (9) elsewhere. The first
 * cycle sweeps every scale over every pixel and fixes the image-wide c
 * (with params c <= 0); the later cycles keep that c and their sweeps skip
 * the 32 x 32 blocks (in whole workgroups of the sweep: a strip segment) in
 * which no pixel needs a scale -- a block needs every scale where a pixel is
 * not confident, and the network's scale where it is (for the normalised
 * Hessian at that scale). With params c > 0, c is used as given throughout.
 * conf_threshold = 1 with an unsure network reproduces mf4d_filter for one
 * cycle (and for more cycles with params c > 0). H, W multiples of 16, nscales <= 8,
 * reselect_each_cycle = 1, model, postprocess and check 0. fallback_count (nullable, device uint32): number
 * of pixel-cycles that fell back to the exact argmax. Errors: MF4D_EINVAL,
 * MF4D_ENOMEM, MF4D_EHIP. */
int mf4d_filter_learned(const float *u_in, float *u_out, int H, int W, const mf4d_params *p,
                        const float *theta, float conf_threshold, unsigned *fallback_count, void *ws,
                        size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MF4D_H */
