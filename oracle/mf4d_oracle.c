/*
 * FP64 CPU oracle of the MAFOD hot path (multi-scale anisotropic
 * fourth-order diffusion integrated by Fast Explicit Diffusion cycles).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow reference that the
 * GPU library is checked against. Only tests/, __graft_entry__.smoke() and
 * the cpu_baseline leg of bench.py may load it. It shares no code, headers,
 * tables or helpers with the GPU library under paper_1611_06906_amd/.
 *
 * Everything is double precision, round-to-nearest, no fast-math, no FMA
 * contraction (built with -O2 -ffp-contract=off). Loops follow the paper's
 * definitions directly; OpenMP only splits independent pixel rows.
 *
 * Layout: images are row-major [H][W], x = column (the paper's index i),
 * y = row (the paper's index j).
 *
 * Readings taken where the paper is silent are marked "reading:" and listed
 * in the design notes of the repository.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define REF_RIDGE 0
#define REF_VALLEY 1
#define REF_BOTH 2

/* ------------------------------------------------------------------------ */
/* FED schedule: Sec. 3.5 (Implementation Using Fast Explicit Diffusion)     */
/* ------------------------------------------------------------------------ */

/* Number of substeps per cycle from stopping time T, M cycles and the
 * stable step limit tau_max: Eq. (22). */
int ref_fed_n(double T, int M, double tau_max)
{
    double v = -0.5 + 0.5 * sqrt(1.0 + 12.0 * T / ((double)M * tau_max));
    return (int)ceil(v);
}

/* Step sizes of one cycle, Eq. (23), in their natural (ascending) order. */
void ref_fed_taus(int n, double T, int M, double *tau)
{
    for (int i = 0; i < n; ++i) {
        double c = cos(M_PI * (double)(2 * i + 1) / (double)(4 * n + 2));
        tau[i] = 3.0 * T / (2.0 * (double)M * ((double)n * n + n) * c * c);
    }
}

static int gcd_int(int a, int b)
{
    while (b) { int t = a % b; a = b; b = t; }
    return a;
}

/* Largest modulus of the partial products of (1 - tau_l z) over the grid
 * z = 2q / (Q tau_max), q = 0..Q, taken over all prefixes l = 0..j and all
 * suffixes l = j..n-1 of the ordered steps. */
static double ref_partial_amplification(int n, const double *ordered, double tau_max, int Q)
{
    double worst = 0.0;
    for (int q = 0; q <= Q; ++q) {
        double z = 2.0 * (double)q / ((double)Q * tau_max);
        double p = 1.0;
        for (int j = 0; j < n; ++j) {
            p *= (1.0 - ordered[j] * z);
            if (fabs(p) > worst) worst = fabs(p);
        }
        p = 1.0;
        for (int j = n - 1; j >= 0; --j) {
            p *= (1.0 - ordered[j] * z);
            if (fabs(p) > worst) worst = fabs(p);
        }
    }
    return worst;
}

/* Reordering of the cycle's steps (Sec. 3.5 names kappa-cycles without
 * defining them). reading: the steps are visited as pi(j) = (kappa * j) mod n
 * for the kappa in [1, n-1] coprime to n that minimises the largest partial
 * amplification (above, Q = 8192); ties within 1e-12 relative keep the
 * smaller kappa; n <= 2 uses kappa = 1. Returns kappa; writes the
 * permutation and the ordered steps. */
int ref_kappa_order(int n, const double *tau, double tau_max, int *perm, double *ordered)
{
    const int Q = 8192;
    int best_k = 1;
    double best = INFINITY;
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (n > 2) {
        for (int k = 1; k < n; ++k) {
            if (gcd_int(k, n) != 1) continue;
            for (int j = 0; j < n; ++j) tmp[j] = tau[(int)(((long)k * j) % n)];
            double a = ref_partial_amplification(n, tmp, tau_max, Q);
            if (a < best * (1.0 - 1e-12)) { best = a; best_k = k; }
        }
    }
    for (int j = 0; j < n; ++j) {
        perm[j] = (int)(((long)best_k * j) % n);
        ordered[j] = tau[perm[j]];
    }
    free(tmp);
    return best_k;
}

/* Ordered steps for a cycle of n substeps when n is given: T/M then equals
 * tau_max (n^2 + n) / 3, so Eq. (23) gives tau_i = tau_max / (2 cos^2(.)). */
int ref_fed_schedule(int n, double tau_max, double *ordered, int *perm)
{
    double *tau = (double *)malloc(sizeof(double) * (size_t)n);
    double T = tau_max * ((double)n * n + n) / 3.0;
    ref_fed_taus(n, T, 1, tau);
    int k = ref_kappa_order(n, tau, tau_max, perm, ordered);
    free(tau);
    return k;
}

/* ------------------------------------------------------------------------ */
/* Gaussian regularisation u_sigma = u * G_sigma (Sec. 3.1, Eq. (6))          */
/* ------------------------------------------------------------------------ */

/* reading: sampled Gaussian exp(-j^2 / (2 sigma^2)), |j| <= r with
 * r = max(1, ceil(3 sigma)), normalised to unit sum. Returns r. */
int ref_gauss_taps(double sigma, double *g /* 2r+1 */)
{
    int r = (int)ceil(3.0 * sigma);
    if (r < 1) r = 1;
    double s = 0.0;
    for (int j = -r; j <= r; ++j) {
        g[j + r] = exp(-(double)j * j / (2.0 * sigma * sigma));
        s += g[j + r];
    }
    for (int j = 0; j <= 2 * r; ++j) g[j] /= s;
    return r;
}

int ref_gauss_radius(double sigma)
{
    int r = (int)ceil(3.0 * sigma);
    return r < 1 ? 1 : r;
}

/* reading: half-sample symmetric extension (... b a | a b ... y z | z y ...),
 * periodic with period 2n so that it also covers radii larger than n. */
static int sym_index(int i, int n)
{
    int p = 2 * n;
    i %= p;
    if (i < 0) i += p;
    return i < n ? i : p - 1 - i;
}

/* Separable Gaussian blur of a [H][W] image with symmetric extension. */
void ref_blur(const double *u, int H, int W, double sigma, double *out)
{
    int r = ref_gauss_radius(sigma);
    double *g = (double *)malloc(sizeof(double) * (size_t)(2 * r + 1));
    ref_gauss_taps(sigma, g);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)H * W);
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            double s = 0.0;
            for (int j = -r; j <= r; ++j) s += g[j + r] * u[(size_t)y * W + sym_index(x + j, W)];
            tmp[(size_t)y * W + x] = s;
        }
    }
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            double s = 0.0;
            for (int j = -r; j <= r; ++j) s += g[j + r] * tmp[(size_t)sym_index(y + j, H) * W + x];
            out[(size_t)y * W + x] = s;
        }
    }
    free(tmp);
    free(g);
}

/* Central-difference gradient and Hessian of a smoothed image (reading: the
 * Hajiaboli stencils of Sec. 3.4 applied to u_sigma, with the same symmetric
 * extension at the border):
 *   u_x  = (v[x+1] - v[x-1]) / 2,                 u_y likewise,
 *   u_xx = v[x-1] - 2 v[x] + v[x+1],             u_yy likewise,
 *   u_xy = (v[x-1,y-1] + v[x+1,y+1] - v[x-1,y+1] - v[x+1,y-1]) / 4. */
void ref_derivatives(const double *v, int H, int W, double *ux, double *uy,
                     double *uxx, double *uxy, double *uyy)
{
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        int ym = sym_index(y - 1, H), yp = sym_index(y + 1, H);
        for (int x = 0; x < W; ++x) {
            int xm = sym_index(x - 1, W), xp = sym_index(x + 1, W);
            size_t c = (size_t)y * W + x;
#define V(yy, xx) v[(size_t)(yy) * W + (xx)]
            if (ux) ux[c] = (V(y, xp) - V(y, xm)) / 2.0;
            if (uy) uy[c] = (V(yp, x) - V(ym, x)) / 2.0;
            if (uxx) uxx[c] = V(y, xm) - 2.0 * V(y, x) + V(y, xp);
            if (uyy) uyy[c] = V(ym, x) - 2.0 * V(y, x) + V(yp, x);
            if (uxy) uxy[c] = (V(ym, xm) + V(yp, xp) - V(yp, xm) - V(ym, xp)) / 4.0;
#undef V
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Scale selection: Sec. 3.3, Eq. (9)                                        */
/* ------------------------------------------------------------------------ */

/* Eigenvalues of the symmetric 2x2 matrix [[a, b], [b, d]], larger first. */
static void eig2_values(double a, double b, double d, double *l1, double *l2)
{
    double m = 0.5 * (a + d);
    double r = hypot(0.5 * (a - d), b);
    *l1 = m + r;
    *l2 = m - r;
}

/* Frangi vesselness of one pixel from the Hessian of u_sigma, Eq. (9).
 * nt1, nt2: the scale-normalised eigenvalues sigma^2 nu_i sorted so that
 * |nt1| <= |nt2|. Returns V for the given c; writes S.
 * reading (magnitude tie |nt1| == |nt2| with nt1 != nt2, i.e. zero trace):
 *   the order is the one under which the mode's sign test passes.
 * reading (modes): RIDGE: V = 0 if nt2 > 0; VALLEY (analogue): V = 0 if
 *   nt2 < 0; BOTH: no sign test. V = 0 when nt2 == 0 or c == 0. */
static double vesselness_px(double hxx, double hxy, double hyy, double sigma,
                            int mode, double beta, double c, double *S_out)
{
    double s2 = sigma * sigma;
    double la, lb;
    eig2_values(s2 * hxx, s2 * hxy, s2 * hyy, &la, &lb);
    double nt1, nt2;
    if (fabs(la) < fabs(lb)) { nt1 = la; nt2 = lb; }
    else if (fabs(la) > fabs(lb)) { nt1 = lb; nt2 = la; }
    else {
        /* |la| == |lb|: either la == lb, or la == -lb > 0 */
        if (mode == REF_VALLEY) { nt2 = la; nt1 = lb; }   /* positive one */
        else { nt2 = lb; nt1 = la; }                       /* negative one */
    }
    double S = sqrt(nt1 * nt1 + nt2 * nt2);
    if (S_out) *S_out = S;
    if (nt2 == 0.0 || c == 0.0) return 0.0;
    if (mode == REF_RIDGE && nt2 > 0.0) return 0.0;
    if (mode == REF_VALLEY && nt2 < 0.0) return 0.0;
    double RB = nt1 / nt2;
    return exp(-(RB * RB) / (2.0 * beta * beta)) * (1.0 - exp(-(S * S) / (2.0 * c * c)));
}

/* Full scale sweep: Hessians at every scale, c = max(S)/2 over all scales
 * and pixels (reading: one c per image; a positive c_param is used as
 * given), V per scale, and per pixel the smallest scale index attaining the
 * maximum V (reading for ties).
 * Outputs (nullable except idx): V_all [ns][H][W], S_all [ns][H][W],
 * vmax [H][W], c_out (scalar). Returns 0. */
int ref_scale_select(const double *u, int H, int W, int ns, const double *sigmas,
                     int mode, double beta, double c_param,
                     uint8_t *idx, double *V_all, double *S_all, double *vmax, double *c_out)
{
    size_t m = (size_t)H * W;
    double *hxx = (double *)malloc(sizeof(double) * m * ns);
    double *hxy = (double *)malloc(sizeof(double) * m * ns);
    double *hyy = (double *)malloc(sizeof(double) * m * ns);
    double *S = (double *)malloc(sizeof(double) * m * ns);
    double *V = (double *)malloc(sizeof(double) * m * ns);
    double *us = (double *)malloc(sizeof(double) * m);
    for (int s = 0; s < ns; ++s) {
        ref_blur(u, H, W, sigmas[s], us);
        ref_derivatives(us, H, W, NULL, NULL, hxx + s * m, hxy + s * m, hyy + s * m);
    }
    double smax = 0.0;
    for (int s = 0; s < ns; ++s) {
        #pragma omp parallel for schedule(static) reduction(max:smax)
        for (size_t p = 0; p < m; ++p) {
            double Sv;
            vesselness_px(hxx[s * m + p], hxy[s * m + p], hyy[s * m + p], sigmas[s], mode, beta, 1.0, &Sv);
            S[s * m + p] = Sv;
            if (Sv > smax) smax = Sv;
        }
    }
    double c = c_param > 0.0 ? c_param : 0.5 * smax;
    if (c_out) *c_out = c;
    for (int s = 0; s < ns; ++s) {
        #pragma omp parallel for schedule(static)
        for (size_t p = 0; p < m; ++p)
            V[s * m + p] = vesselness_px(hxx[s * m + p], hxy[s * m + p], hyy[s * m + p],
                                         sigmas[s], mode, beta, c, NULL);
    }
    #pragma omp parallel for schedule(static)
    for (size_t p = 0; p < m; ++p) {
        int best = 0;
        double bv = V[p];
        for (int s = 1; s < ns; ++s)
            if (V[s * m + p] > bv) { bv = V[s * m + p]; best = s; }
        idx[p] = (uint8_t)best;
        if (vmax) vmax[p] = bv;
    }
    if (V_all) memcpy(V_all, V, sizeof(double) * m * ns);
    if (S_all) memcpy(S_all, S, sizeof(double) * m * ns);
    free(hxx); free(hxy); free(hyy); free(S); free(V); free(us);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Normalised, integrated Hessian H_rho(u_sigma): Eq. (6)                    */
/* ------------------------------------------------------------------------ */

/* For each pixel, N = H(u_sigma) / sqrt(1 + |grad u_sigma|) at that pixel's
 * selected scale (reading: the gradient norm enters unsquared, as printed),
 * then H_rho = G_rho * N per component (symmetric extension; rho = 0 means
 * no integration). Output planes hrho[0..2] = (a, b, d) = (xx, xy, yy). */
int ref_tensor(const double *u, int H, int W, const uint8_t *idx, int ns,
               const double *sigmas, double rho, double *hrho /* 3*H*W */)
{
    size_t m = (size_t)H * W;
    double *us = (double *)malloc(sizeof(double) * m);
    double *ux = (double *)malloc(sizeof(double) * m);
    double *uy = (double *)malloc(sizeof(double) * m);
    double *uxx = (double *)malloc(sizeof(double) * m);
    double *uxy = (double *)malloc(sizeof(double) * m);
    double *uyy = (double *)malloc(sizeof(double) * m);
    double *N = (double *)calloc(3 * m, sizeof(double));
    for (int s = 0; s < ns; ++s) {
        int used = 0;
        for (size_t p = 0; p < m && !used; ++p) used = (idx[p] == s);
        if (!used) continue;
        ref_blur(u, H, W, sigmas[s], us);
        ref_derivatives(us, H, W, ux, uy, uxx, uxy, uyy);
        #pragma omp parallel for schedule(static)
        for (size_t p = 0; p < m; ++p) {
            if (idx[p] != s) continue;
            double f = 1.0 / sqrt(1.0 + sqrt(ux[p] * ux[p] + uy[p] * uy[p]));
            N[p] = uxx[p] * f;
            N[m + p] = uxy[p] * f;
            N[2 * m + p] = uyy[p] * f;
        }
    }
    for (int k = 0; k < 3; ++k) {
        if (rho > 0.0) ref_blur(N + k * m, H, W, rho, hrho + k * m);
        else memcpy(hrho + k * m, N + k * m, sizeof(double) * m);
    }
    free(us); free(ux); free(uy); free(uxx); free(uxy); free(uyy); free(N);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Fourth-order diffusion tensor: Sec. 3.2, Eqs. (7), (8); 4x4 form Sec. 3.4 */
/* ------------------------------------------------------------------------ */

/* Perona-Malik diffusivity of Eq. (1) applied to an eigenvalue, Eq. (7). */
static double pm(double nu, double lambda)
{
    return 1.0 / (1.0 + (nu * nu) / (lambda * lambda));
}

/* The 4x4 matrix D_i = E M E^T acting on (xx, xy, yx, yy), built literally:
 * eigenvectors e1, e2 of H_rho, eigentensors E1 = e1 (x) e1, E2 = e2 (x) e2,
 * E3 = (e1 (x) e2 + e2 (x) e1)/sqrt2, E4 = (e1 (x) e2 - e2 (x) e1)/sqrt2,
 * mu_1,2 from Eq. (7) with the mode's mask (RIDGE: mu_i = 1 where
 * nu_i >= 0; VALLEY: mu_i = 1 where nu_i <= 0; BOTH: none), mu_3 the mean of
 * mu_1 and mu_2, mu_4 = 0. (x) is the outer product, (a (x) b)_kl = a_k b_l.
 * Writes D row-major 4x4; optional e[4] = (e1x, e1y, e2x, e2y), mu[4]. */
void ref_dtensor_px(double a, double b, double d, double lambda, int mode,
                    double *D, double *e_out, double *mu_out)
{
    double theta = 0.5 * atan2(2.0 * b, a - d);
    double e1x = cos(theta), e1y = sin(theta);
    double e2x = -e1y, e2y = e1x;
    double nu1, nu2;
    eig2_values(a, b, d, &nu1, &nu2);
    double mu[4];
    mu[0] = pm(nu1, lambda);
    mu[1] = pm(nu2, lambda);
    if (mode == REF_RIDGE) {
        if (nu1 >= 0.0) mu[0] = 1.0;
        if (nu2 >= 0.0) mu[1] = 1.0;
    } else if (mode == REF_VALLEY) {
        if (nu1 <= 0.0) mu[0] = 1.0;
        if (nu2 <= 0.0) mu[1] = 1.0;
    }
    mu[2] = 0.5 * (mu[0] + mu[1]);
    mu[3] = 0.0;
    double e1[2] = {e1x, e1y}, e2[2] = {e2x, e2y};
    double E[4][4]; /* E[component][i]: column i is vec(E_i) */
    const double rs2 = 1.0 / sqrt(2.0);
    for (int k = 0; k < 2; ++k)
        for (int l = 0; l < 2; ++l) {
            int c = 2 * k + l; /* vec order (xx, xy, yx, yy) */
            E[c][0] = e1[k] * e1[l];
            E[c][1] = e2[k] * e2[l];
            E[c][2] = rs2 * (e1[k] * e2[l] + e2[k] * e1[l]);
            E[c][3] = rs2 * (e1[k] * e2[l] - e2[k] * e1[l]);
        }
    for (int r = 0; r < 4; ++r)
        for (int c = 0; c < 4; ++c) {
            double s = 0.0;
            for (int i = 0; i < 4; ++i) s += E[r][i] * mu[i] * E[c][i];
            D[4 * r + c] = s;
        }
    if (e_out) { e_out[0] = e1x; e_out[1] = e1y; e_out[2] = e2x; e_out[3] = e2y; }
    if (mu_out) for (int i = 0; i < 4; ++i) mu_out[i] = mu[i];
}

/* D for every pixel: out [H*W][16]. */
void ref_dtensor(const double *hrho, int H, int W, double lambda, int mode, double *Dall)
{
    size_t m = (size_t)H * W;
    #pragma omp parallel for schedule(static)
    for (size_t p = 0; p < m; ++p)
        ref_dtensor_px(hrho[p], hrho[m + p], hrho[2 * m + p], lambda, mode, Dall + 16 * p, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* Discrete operator P = L^T D L with natural boundaries: Sec. 3.4           */
/* ------------------------------------------------------------------------ */

/* L has rows only at pixels where the whole 3x3 stencil fits (natural
 * boundary condition): 1 <= x <= W-2, 1 <= y <= H-2. At such a pixel
 *   [L_xx u] = u(x-1,y) - 2u(x,y) + u(x+1,y)
 *   [L_yy u] = u(x,y-1) - 2u(x,y) + u(x,y+1)
 *   [L_xy u] = [L_yx u] = (u(x-1,y-1) + u(x+1,y+1) - u(x-1,y+1) - u(x+1,y-1)) / 4.
 * r = P u is formed as L^T (D (L u)): t = D_p h at each interior pixel, then
 * scattered back through the transposed stencils. */
void ref_apply_P(const double *u, const double *Dall, int H, int W, double *r)
{
    size_t m = (size_t)H * W;
    double *t = (double *)calloc(4 * m, sizeof(double));
    memset(r, 0, sizeof(double) * m);
    #pragma omp parallel for schedule(static)
    for (int y = 1; y < H - 1; ++y) {
        for (int x = 1; x < W - 1; ++x) {
#define U(yy, xx) u[(size_t)(yy) * W + (xx)]
            double h[4];
            h[0] = U(y, x - 1) - 2.0 * U(y, x) + U(y, x + 1);
            h[1] = (U(y - 1, x - 1) + U(y + 1, x + 1) - U(y + 1, x - 1) - U(y - 1, x + 1)) / 4.0;
            h[2] = h[1];
            h[3] = U(y - 1, x) - 2.0 * U(y, x) + U(y + 1, x);
#undef U
            size_t p = (size_t)y * W + x;
            const double *D = Dall + 16 * p;
            for (int i = 0; i < 4; ++i) {
                double s = 0.0;
                for (int j = 0; j < 4; ++j) s += D[4 * i + j] * h[j];
                t[4 * p + i] = s;
            }
        }
    }
    /* scatter r += L^T t; rows three apart never touch the same output row */
    for (int phase = 0; phase < 3; ++phase) {
        #pragma omp parallel for schedule(static)
        for (int y = 1 + phase; y < H - 1; y += 3) {
            for (int x = 1; x < W - 1; ++x) {
                size_t p = (size_t)y * W + x;
                const double *tp = t + 4 * p;
#define R(yy, xx) r[(size_t)(yy) * W + (xx)]
                /* L_xx row */
                R(y, x - 1) += tp[0];
                R(y, x) += -2.0 * tp[0];
                R(y, x + 1) += tp[0];
                /* L_xy row and L_yx row (same stencil) */
                for (int k = 1; k <= 2; ++k) {
                    R(y - 1, x - 1) += tp[k] / 4.0;
                    R(y + 1, x + 1) += tp[k] / 4.0;
                    R(y + 1, x - 1) -= tp[k] / 4.0;
                    R(y - 1, x + 1) -= tp[k] / 4.0;
                }
                /* L_yy row */
                R(y - 1, x) += tp[3];
                R(y, x) += -2.0 * tp[3];
                R(y + 1, x) += tp[3];
#undef R
            }
        }
    }
    free(t);
}

/* One explicit step u <- (I - tau P) u, Eq. (10) in the form of Eq. (17). */
void ref_explicit_step(double *u, const double *Dall, int H, int W, double tau)
{
    size_t m = (size_t)H * W;
    double *r = (double *)malloc(sizeof(double) * m);
    ref_apply_P(u, Dall, H, W, r);
    #pragma omp parallel for schedule(static)
    for (size_t p = 0; p < m; ++p) u[p] -= tau * r[p];
    free(r);
}

/* One FED cycle, Eq. (21): P is frozen for the whole cycle and the n steps
 * are applied in the given order. */
void ref_fed_cycle(double *u, const double *Dall, int H, int W, const double *ordered_tau, int n)
{
    for (int i = 0; i < n; ++i) ref_explicit_step(u, Dall, H, W, ordered_tau[i]);
}

/* ------------------------------------------------------------------------ */
/* Isotropic fourth-order diffusion (IFOD): Sec. 3.1, Eq. (4)                */
/* ------------------------------------------------------------------------ */

/* Diffusivity of the isotropic model of Eq. (4): g = 1 / (1 + F / lambda^2)
 * with F = ||H(u_sigma)||_F^2 = h_xx^2 + h_xy^2 + h_yx^2 + h_yy^2 (Eq. (1)
 * with the squared Frobenius norm of the Hessian as its argument).
 * reading: the Hessian is taken of u_sigma = u * G_sigma (the comparison
 * experiments of Sec. 4.1 regularise IFOD with sigma = 1), with the same
 * Gaussian, symmetric extension and central differences as the scale stack.
 * Optional hess (nullable) receives (h_xx, h_xy, h_yy) planes. */
void ref_ifod_diffusivity(const double *u, int H, int W, double sigma, double lambda,
                          double *g, double *hess /* 3*H*W or NULL */)
{
    size_t m = (size_t)H * W;
    double *us = (double *)malloc(sizeof(double) * m);
    double *hxx = (double *)malloc(sizeof(double) * m);
    double *hxy = (double *)malloc(sizeof(double) * m);
    double *hyy = (double *)malloc(sizeof(double) * m);
    ref_blur(u, H, W, sigma, us);
    ref_derivatives(us, H, W, NULL, NULL, hxx, hxy, hyy);
    #pragma omp parallel for schedule(static)
    for (size_t p = 0; p < m; ++p) {
        double F = hxx[p] * hxx[p] + 2.0 * hxy[p] * hxy[p] + hyy[p] * hyy[p];
        g[p] = 1.0 / (1.0 + F / (lambda * lambda));
    }
    if (hess) {
        memcpy(hess, hxx, sizeof(double) * m);
        memcpy(hess + m, hxy, sizeof(double) * m);
        memcpy(hess + 2 * m, hyy, sizeof(double) * m);
    }
    free(us); free(hxx); free(hxy); free(hyy);
}

/* The isotropic model as a fourth-order tensor: D = g Id on (xx, xy, yx, yy),
 * i.e. every component of the Hessian is scaled by g (Eq. (4)). */
void ref_ifod_dtensor(const double *g, int H, int W, double *Dall)
{
    size_t m = (size_t)H * W;
    #pragma omp parallel for schedule(static)
    for (size_t p = 0; p < m; ++p) {
        double *D = Dall + 16 * p;
        for (int k = 0; k < 16; ++k) D[k] = 0.0;
        for (int k = 0; k < 4; ++k) D[5 * k] = g[p];
    }
}

/* ------------------------------------------------------------------------ */
/* Scale-image postprocessing: Sec. 3.3, the text after Eq. (9)              */
/* ------------------------------------------------------------------------ */

/* Direction across the crease at every pixel: the unit eigenvector of the
 * eigenvalue of larger magnitude of H(u_sigma) at the pixel's selected scale
 * sigma_{idx}. reading: at equal magnitudes the eigenvector of the larger
 * eigenvalue, at angle t = atan2(2 h_xy, h_xx - h_yy) / 2, is taken (for
 * h_xx = h_yy, h_xy = 0 that is (1, 0)). */
void ref_cross_direction(const double *u, int H, int W, int ns, const double *sigmas,
                         const uint8_t *idx, double *ex, double *ey)
{
    size_t m = (size_t)H * W;
    double *us = (double *)malloc(sizeof(double) * m);
    double *hxx = (double *)malloc(sizeof(double) * m);
    double *hxy = (double *)malloc(sizeof(double) * m);
    double *hyy = (double *)malloc(sizeof(double) * m);
    for (int s = 0; s < ns; ++s) {
        int used = 0;
        for (size_t p = 0; p < m && !used; ++p) used = (idx[p] == s);
        if (!used) continue;
        ref_blur(u, H, W, sigmas[s], us);
        ref_derivatives(us, H, W, NULL, NULL, hxx, hxy, hyy);
        #pragma omp parallel for schedule(static)
        for (size_t p = 0; p < m; ++p) {
            if (idx[p] != s) continue;
            double l1, l2;
            eig2_values(hxx[p], hxy[p], hyy[p], &l1, &l2);
            double t = 0.5 * atan2(2.0 * hxy[p], hxx[p] - hyy[p]);
            double e1x = cos(t), e1y = sin(t);
            if (fabs(l2) > fabs(l1)) { ex[p] = -e1y; ey[p] = e1x; }
            else { ex[p] = e1x; ey[p] = e1y; }
        }
    }
    free(us); free(hxx); free(hxy); free(hyy);
}

/* Rounds half away from zero, so that a march and its mirror image visit
 * mirrored pixels. */
static double round_away(double v)
{
    return v >= 0.0 ? floor(v + 0.5) : -floor(-v + 0.5);
}

/* The postprocessing of the scale image. A pixel is on a vessel when its
 * vesselness max_s V_s reaches theta. For every vessel pixel p, its
 * cross-section is sampled by marching from p along +e(p) and -e(p) (the
 * direction across the crease, above) in unit steps, t = 1, 2, ..., tmax,
 * visiting the pixel nearest to p + t e (each coordinate offset rounded
 * half away from zero), and stopping in each direction at the first sample
 * that leaves the image or is not a vessel pixel. p then takes the scale
 * closest to the mean sigma over the samples (p itself and every visited
 * sample, repeats counted); ties go to the smaller scale. Other pixels keep
 * their scale. reading: the march follows the straight line through p along
 * p's own direction; tmax = ceil(3 sigma_max), the support radius of the
 * largest scale. The comparison |mean - sigma_s| is made as |sum - n sigma_s|
 * (the same order after multiplying by n > 0; exact in double, as every
 * term is a float32 sigma times a small integer). */
void ref_postprocess(int H, int W, int ns, const double *sigmas, const uint8_t *idx_in,
                     const double *vmax, const double *ex, const double *ey, double theta,
                     int tmax, uint8_t *idx_out)
{
    #pragma omp parallel for schedule(static)
    for (int y = 0; y < H; ++y) {
        for (int x = 0; x < W; ++x) {
            size_t p = (size_t)y * W + x;
            if (!(vmax[p] >= theta)) { idx_out[p] = idx_in[p]; continue; }
            double sum = sigmas[idx_in[p]];
            double n = 1.0;
            for (int dir = -1; dir <= 1; dir += 2) {
                for (int t = 1; t <= tmax; ++t) {
                    int xx = x + (int)round_away(dir * t * ex[p]);
                    int yy = y + (int)round_away(dir * t * ey[p]);
                    if (xx < 0 || xx >= W || yy < 0 || yy >= H) break;
                    size_t q = (size_t)yy * W + xx;
                    if (!(vmax[q] >= theta)) break;
                    sum += sigmas[idx_in[q]];
                    n += 1.0;
                }
            }
            int best = 0;
            double bd = fabs(sum - n * sigmas[0]);
            for (int s = 1; s < ns; ++s) {
                double d = fabs(sum - n * sigmas[s]);
                if (d < bd) { bd = d; best = s; }
            }
            idx_out[p] = (uint8_t)best;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* The whole filter: M FED cycles, each re-forming P from u^k (Eq. (21))     */
/* ------------------------------------------------------------------------ */

/* Options of ref_filter beyond the paper's core parameters (NULL = all 0). */
typedef struct ref_opts {
    int model;                  /* 0: the anisotropic model, Eqs. (5)-(8); 1: IFOD, Eq. (4) */
    int postprocess;            /* 1: scale-image postprocessing after each scale selection */
    double theta;               /* vessel threshold of the postprocessing */
    const uint8_t *idx_inject;  /* [M][H][W] or NULL: the scale indices of each cycle are
                                   taken from here instead of being selected (teacher
                                   forcing of stage parity) */
} ref_opts;

/* reading: scales are re-selected on u^k at every cycle when reselect != 0,
 * otherwise once on u^0 (the normalised Hessian is still re-formed from u^k
 * each cycle at the kept scales).
 * n_substeps > 0: n given and T/M = tau_max (n^2+n)/3; otherwise n from
 * Eq. (22) with stop_time T and the steps from Eq. (23).
 * Optional records (nullable): idx_rec [M][H][W], c_rec [M],
 * hrho_rec [M][3][H][W], u_rec [M][H][W] (state after each cycle).
 * With opts->model == 1 (IFOD) no scale is selected: D = g Id with g from
 * H(u_sigma) at sigma = sigmas[0]; hrho_rec then records that Hessian.
 * Returns n, or -1 on invalid schedule. */
int ref_filter(const double *u_in, double *u_out, int H, int W,
               int ns, const double *sigmas, int mode, double lambda, double rho,
               double beta, double c_param, int M, int n_substeps, double stop_time,
               double tau_max, int reselect,
               uint8_t *idx_rec, double *c_rec, double *hrho_rec, double *u_rec,
               const ref_opts *opts)
{
    ref_opts none = {0, 0, 0.0, NULL};
    if (!opts) opts = &none;
    size_t m = (size_t)H * W;
    int n = n_substeps;
    double *tau, *ordered;
    int *perm;
    if (n > 0) {
        ordered = (double *)malloc(sizeof(double) * n);
        perm = (int *)malloc(sizeof(int) * n);
        ref_fed_schedule(n, tau_max, ordered, perm);
    } else {
        if (!(stop_time > 0.0) || M <= 0) return -1;
        n = ref_fed_n(stop_time, M, tau_max);
        tau = (double *)malloc(sizeof(double) * n);
        ordered = (double *)malloc(sizeof(double) * n);
        perm = (int *)malloc(sizeof(int) * n);
        ref_fed_taus(n, stop_time, M, tau);
        ref_kappa_order(n, tau, tau_max, perm, ordered);
        free(tau);
    }
    memcpy(u_out, u_in, sizeof(double) * m);
    uint8_t *idx = (uint8_t *)malloc(m);
    double *hrho = (double *)malloc(sizeof(double) * 3 * m);
    double *Dall = (double *)malloc(sizeof(double) * 16 * m);
    double *vmax = (double *)malloc(sizeof(double) * m);
    double *gdiff = (double *)malloc(sizeof(double) * m);
    for (int k = 0; k < M; ++k) {
        double c = 0.0;
        if (opts->model == 1) {
            ref_ifod_diffusivity(u_out, H, W, sigmas[0], lambda, gdiff, hrho);
            ref_ifod_dtensor(gdiff, H, W, Dall);
            memset(idx, 0, m);
        } else {
            if (opts->idx_inject) {
                memcpy(idx, opts->idx_inject + k * m, m);
            } else if (k == 0 || reselect) {
                ref_scale_select(u_out, H, W, ns, sigmas, mode, beta, c_param, idx, NULL, NULL, vmax, &c);
                if (opts->postprocess) {
                    double *ex = (double *)malloc(sizeof(double) * m);
                    double *ey = (double *)malloc(sizeof(double) * m);
                    uint8_t *pp = (uint8_t *)malloc(m);
                    ref_cross_direction(u_out, H, W, ns, sigmas, idx, ex, ey);
                    ref_postprocess(H, W, ns, sigmas, idx, vmax, ex, ey, opts->theta,
                                    (int)ceil(3.0 * sigmas[ns - 1]), pp);
                    memcpy(idx, pp, m);
                    free(ex); free(ey); free(pp);
                }
            }
            ref_tensor(u_out, H, W, idx, ns, sigmas, rho, hrho);
            ref_dtensor(hrho, H, W, lambda, mode, Dall);
        }
        ref_fed_cycle(u_out, Dall, H, W, ordered, n);
        if (idx_rec) memcpy(idx_rec + k * m, idx, m);
        if (c_rec) c_rec[k] = c;
        if (hrho_rec) memcpy(hrho_rec + 3 * k * m, hrho, sizeof(double) * 3 * m);
        if (u_rec) memcpy(u_rec + k * m, u_out, sizeof(double) * m);
    }
    free(vmax); free(gdiff);
    free(idx); free(hrho); free(Dall); free(ordered); free(perm);
    return n;
}
