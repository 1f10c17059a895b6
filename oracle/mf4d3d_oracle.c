/*
 * FP64 CPU oracle of the 3-D extension of the filter -- TEST INFRASTRUCTURE
 * ONLY (the rules of mf4d_oracle.c apply: it shares nothing with the GPU
 * library, and only the tests and the bench's CPU baseline may load it).
 *
 * The paper builds the filter in 2-D and names the 3-D extension as future
 * work (Sec. 5). Readings taken here, each the direct generalisation of the
 * 2-D definitions:
 *  - volumes are row-major [D][H][W] (x fastest, then y, then z), spacing 1;
 *    Gaussian blur, symmetric extension and central differences per axis as
 *    in 2-D; mixed derivatives by the 2-D cross stencil in each plane;
 *  - scale selection: Frangi's 3-D tube measure on sigma^2-normalised
 *    eigenvalues |n1| <= |n2| <= |n3|: R_A = |n2|/|n3|, R_B = |n1|/sqrt|n2 n3|,
 *    S = sqrt(n1^2+n2^2+n3^2), V = (1 - exp(-R_A^2/(2 a^2))) exp(-R_B^2/(2 b^2))
 *    (1 - exp(-S^2/(2 c^2))) with a = b = 1/2 and the image-wide
 *    c = max(S)/2; a bright tube (RIDGE) needs n2, n3 < 0, a dark one
 *    (VALLEY) n2, n3 > 0, BOTH tests no sign; V = 0 when n2 n3 = 0 or c = 0;
 *    the smallest scale index of maximal V;
 *  - the normalised integrated Hessian as Eq. (6) per component (6 of them);
 *  - the tensor: eigenpairs (nu_i, e_i) of H_rho; mu_i as Eq. (7) with the
 *    mode masks; eigentensors E_ii = e_i (x) e_i with mu_i, the symmetric
 *    E_ij = (e_i (x) e_j + e_j (x) e_i)/sqrt2 (i < j) with (mu_i + mu_j)/2
 *    and the antisymmetric ones with 0 -- the literal 9 x 9 D on
 *    (xx, xy, xz, yx, yy, yz, zx, zy, zz);
 *  - P = L^T D L with rows of L (the nine second-difference stencils, L_ij =
 *    L_ji) only at voxels whose 3x3x3 neighbourhood lies inside (natural
 *    boundary). ||L_ii||^2 <= 16 and ||L_ij||^2 <= 1, so with ||D|| <= 1 the
 *    largest eigenvalue of P is at most 3 * 16 + 6 * 1 = 54 and the explicit
 *    step is stable for tau <= 2/54 = 1/27 (the 2-D bound of 34 gives 1/17).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int ref_gauss_taps(double sigma, double *g);
int ref_gauss_radius(double sigma);
int ref_fed_schedule(int n, double tau_max, double *ordered, int *perm);

#define RIDGE3 0
#define VALLEY3 1

static int sym3(int i, int n)
{
    int p = 2 * n;
    i %= p;
    if (i < 0) i += p;
    return i < n ? i : p - 1 - i;
}

#define IX(z, y, x) (((size_t)(z) * H + (y)) * W + (x))

/* Separable Gaussian blur of a [D][H][W] volume, symmetric extension. */
void ref3_blur(const double *u, int D, int H, int W, double sigma, double *out)
{
    int r = ref_gauss_radius(sigma);
    double *g = (double *)malloc(sizeof(double) * (size_t)(2 * r + 1));
    ref_gauss_taps(sigma, g);
    size_t m = (size_t)D * H * W;
    double *a = (double *)malloc(sizeof(double) * m);
    double *b = (double *)malloc(sizeof(double) * m);
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < D; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double s = 0.0;
                for (int j = -r; j <= r; ++j) s += g[j + r] * u[IX(z, y, sym3(x + j, W))];
                a[IX(z, y, x)] = s;
            }
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < D; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double s = 0.0;
                for (int j = -r; j <= r; ++j) s += g[j + r] * a[IX(z, sym3(y + j, H), x)];
                b[IX(z, y, x)] = s;
            }
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < D; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                double s = 0.0;
                for (int j = -r; j <= r; ++j) s += g[j + r] * b[IX(sym3(z + j, D), y, x)];
                out[IX(z, y, x)] = s;
            }
    free(a); free(b); free(g);
}

/* Gradient and Hessian of a smoothed volume by central differences with the
 * symmetric extension. out: 9 planes g_x, g_y, g_z, h_xx, h_yy, h_zz, h_xy,
 * h_xz, h_yz; mixed terms use the cross stencil of Sec. 3.4 in their plane. */
void ref3_derivatives(const double *v, int D, int H, int W, double *out)
{
    size_t m = (size_t)D * H * W;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < D; ++z)
        for (int y = 0; y < H; ++y)
            for (int x = 0; x < W; ++x) {
                int xm = sym3(x - 1, W), xp = sym3(x + 1, W);
                int ym = sym3(y - 1, H), yp = sym3(y + 1, H);
                int zm = sym3(z - 1, D), zp = sym3(z + 1, D);
                size_t c = IX(z, y, x);
                out[c] = (v[IX(z, y, xp)] - v[IX(z, y, xm)]) / 2.0;
                out[m + c] = (v[IX(z, yp, x)] - v[IX(z, ym, x)]) / 2.0;
                out[2 * m + c] = (v[IX(zp, y, x)] - v[IX(zm, y, x)]) / 2.0;
                out[3 * m + c] = v[IX(z, y, xm)] - 2.0 * v[c] + v[IX(z, y, xp)];
                out[4 * m + c] = v[IX(z, ym, x)] - 2.0 * v[c] + v[IX(z, yp, x)];
                out[5 * m + c] = v[IX(zm, y, x)] - 2.0 * v[c] + v[IX(zp, y, x)];
                out[6 * m + c] = (v[IX(z, ym, xm)] + v[IX(z, yp, xp)] - v[IX(z, yp, xm)] - v[IX(z, ym, xp)]) / 4.0;
                out[7 * m + c] = (v[IX(zm, y, xm)] + v[IX(zp, y, xp)] - v[IX(zp, y, xm)] - v[IX(zm, y, xp)]) / 4.0;
                out[8 * m + c] = (v[IX(zm, ym, x)] + v[IX(zp, yp, x)] - v[IX(zp, ym, x)] - v[IX(zm, yp, x)]) / 4.0;
            }
}

/* Eigen-decomposition of a symmetric 3x3 matrix by cyclic Jacobi rotations
 * (run until the off-diagonal part is exactly zero or negligible against
 * the diagonal, at most 64 sweeps). Eigenvalues in descending order;
 * column k of V is the unit eigenvector of ev[k]. */
void ref3_eig(const double *A_in /* row-major 3x3 */, double *ev, double *V /* row-major 3x3 */)
{
    double A[3][3], Q[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[i][j] = A_in[3 * i + j];
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off == 0.0 || off <= 1e-36 * dia) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (A[p][q] == 0.0) continue;
                double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 3; ++k) {   /* A <- A J */
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {   /* A <- J^T A */
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {   /* Q <- Q J */
                    double qkp = Q[k][p], qkq = Q[k][q];
                    Q[k][p] = c * qkp - s * qkq;
                    Q[k][q] = s * qkp + c * qkq;
                }
            }
    }
    int ord[3] = {0, 1, 2};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (A[ord[j]][ord[j]] > A[ord[i]][ord[i]]) { int t = ord[i]; ord[i] = ord[j]; ord[j] = t; }
    for (int k = 0; k < 3; ++k) {
        ev[k] = A[ord[k]][ord[k]];
        for (int i = 0; i < 3; ++i) V[3 * i + k] = Q[i][ord[k]];
    }
}

/* Frangi 3-D tube measure of one voxel (reading in the header). h: h_xx,
 * h_yy, h_zz, h_xy, h_xz, h_yz of u_sigma. Returns V; writes S. */
double ref3_vesselness_px(const double *h, double sigma, int mode, double alpha, double beta, double c,
                          double *S_out)
{
    double s2 = sigma * sigma;
    double A[9] = {s2 * h[0], s2 * h[3], s2 * h[4], s2 * h[3], s2 * h[1], s2 * h[5], s2 * h[4], s2 * h[5], s2 * h[2]};
    double ev[3], V[9];
    ref3_eig(A, ev, V);
    /* sort by magnitude, ascending; equal magnitudes keep the descending order */
    double n[3] = {ev[0], ev[1], ev[2]};
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (fabs(n[j]) < fabs(n[i])) { double t = n[i]; n[i] = n[j]; n[j] = t; }
    double S = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    if (S_out) *S_out = S;
    if (c == 0.0 || n[1] * n[2] == 0.0) return 0.0;
    if (mode == RIDGE3 && (n[1] > 0.0 || n[2] > 0.0)) return 0.0;
    if (mode == VALLEY3 && (n[1] < 0.0 || n[2] < 0.0)) return 0.0;
    double RA = fabs(n[1]) / fabs(n[2]);
    double RB = fabs(n[0]) / sqrt(fabs(n[1] * n[2]));
    return (1.0 - exp(-RA * RA / (2.0 * alpha * alpha))) * exp(-RB * RB / (2.0 * beta * beta)) *
           (1.0 - exp(-S * S / (2.0 * c * c)));
}

/* Scale selection over the stack: c = max(S)/2 over all scales and voxels
 * (or c_param when positive), idx = smallest index of maximal V. Optional
 * V_all [ns][m]. */
void ref3_scale_select(const double *u, int D, int H, int W, int ns, const double *sigmas, int mode,
                       double alpha, double beta, double c_param, uint8_t *idx, double *V_all, double *c_out)
{
    size_t m = (size_t)D * H * W;
    double *us = (double *)malloc(sizeof(double) * m);
    double *der = (double *)malloc(sizeof(double) * 9 * m);
    double *hs = (double *)malloc(sizeof(double) * 6 * m * ns);
    double *Sv = (double *)malloc(sizeof(double) * m * ns);
    double smax = 0.0;
    for (int s = 0; s < ns; ++s) {
        ref3_blur(u, D, H, W, sigmas[s], us);
        ref3_derivatives(us, D, H, W, der);
        for (size_t p = 0; p < m; ++p)
            for (int k = 0; k < 6; ++k) hs[(s * m + p) * 6 + k] = der[(3 + k) * m + p];
        for (size_t p = 0; p < m; ++p) {
            ref3_vesselness_px(hs + (s * m + p) * 6, sigmas[s], mode, alpha, beta, 1.0, Sv + s * m + p);
            if (Sv[s * m + p] > smax) smax = Sv[s * m + p];
        }
    }
    double c = c_param > 0.0 ? c_param : 0.5 * smax;
    if (c_out) *c_out = c;
    for (size_t p = 0; p < m; ++p) {
        int best = 0;
        double bv = -1.0;
        for (int s = 0; s < ns; ++s) {
            double v = ref3_vesselness_px(hs + (s * m + p) * 6, sigmas[s], mode, alpha, beta, c, NULL);
            if (V_all) V_all[s * m + p] = v;
            if (v > bv) { bv = v; best = s; }
        }
        idx[p] = (uint8_t)best;
    }
    free(us); free(der); free(hs); free(Sv);
}

/* Normalised, integrated Hessian (Eq. (6) per component): N = H(u_sigma) /
 * sqrt(1 + |grad u_sigma|) at each voxel's scale, then G_rho * N. out: 6
 * planes (xx, yy, zz, xy, xz, yz). */
void ref3_tensor(const double *u, int D, int H, int W, const uint8_t *idx, int ns, const double *sigmas,
                 double rho, double *out)
{
    size_t m = (size_t)D * H * W;
    double *us = (double *)malloc(sizeof(double) * m);
    double *der = (double *)malloc(sizeof(double) * 9 * m);
    double *N = (double *)calloc(6 * m, sizeof(double));
    for (int s = 0; s < ns; ++s) {
        int used = 0;
        for (size_t p = 0; p < m && !used; ++p) used = idx[p] == s;
        if (!used) continue;
        ref3_blur(u, D, H, W, sigmas[s], us);
        ref3_derivatives(us, D, H, W, der);
        for (size_t p = 0; p < m; ++p) {
            if (idx[p] != s) continue;
            double gn = sqrt(der[p] * der[p] + der[m + p] * der[m + p] + der[2 * m + p] * der[2 * m + p]);
            double f = 1.0 / sqrt(1.0 + gn);
            for (int k = 0; k < 6; ++k) N[k * m + p] = der[(3 + k) * m + p] * f;
        }
    }
    for (int k = 0; k < 6; ++k) {
        if (rho > 0.0) ref3_blur(N + k * m, D, H, W, rho, out + k * m);
        else memcpy(out + k * m, N + k * m, sizeof(double) * m);
    }
    free(us); free(der); free(N);
}

/* The literal 9x9 tensor of one voxel from its H_rho (xx, yy, zz, xy, xz,
 * yz), on the vector order (xx, xy, xz, yx, yy, yz, zx, zy, zz). */
void ref3_dtensor_px(const double *h, double lambda, int mode, double *Dm /* 81 */, double *mu_out /* 3 */)
{
    double A[9] = {h[0], h[3], h[4], h[3], h[1], h[5], h[4], h[5], h[2]};
    double nu[3], V[9];
    ref3_eig(A, nu, V);
    double mu[3];
    for (int i = 0; i < 3; ++i) {
        mu[i] = 1.0 / (1.0 + nu[i] * nu[i] / (lambda * lambda));
        if (mode == RIDGE3 && nu[i] >= 0.0) mu[i] = 1.0;
        if (mode == VALLEY3 && nu[i] <= 0.0) mu[i] = 1.0;
    }
    if (mu_out) for (int i = 0; i < 3; ++i) mu_out[i] = mu[i];
    memset(Dm, 0, sizeof(double) * 81);
    const double rs2 = 1.0 / sqrt(2.0);
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j) {
            /* eigentensor vec: E[a][b] over a, b in {x, y, z} */
            double E[9];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) {
                    double ea_i = V[3 * a + i], eb_j = V[3 * b + j], ea_j = V[3 * a + j], eb_i = V[3 * b + i];
                    E[3 * a + b] = (i == j) ? ea_i * eb_i : rs2 * (ea_i * eb_j + ea_j * eb_i);
                }
            double w = (i == j) ? mu[i] : 0.5 * (mu[i] + mu[j]);
            for (int r = 0; r < 9; ++r)
                for (int q = 0; q < 9; ++q) Dm[9 * r + q] += w * E[r] * E[q];
        }
}

void ref3_dtensor(const double *hrho, int D, int H, int W, double lambda, int mode, double *Dall)
{
    size_t m = (size_t)D * H * W;
    #pragma omp parallel for schedule(static)
    for (size_t p = 0; p < m; ++p) {
        double h[6];
        for (int k = 0; k < 6; ++k) h[k] = hrho[k * m + p];
        ref3_dtensor_px(h, lambda, mode, Dall + 81 * p, NULL);
    }
}

/* r = L^T D L u with natural boundaries: t = D h at interior voxels, then
 * scattered back through the transposed stencils. */
void ref3_apply_P(const double *u, const double *Dall, int D, int H, int W, double *r)
{
    size_t m = (size_t)D * H * W;
    double *t = (double *)calloc(9 * m, sizeof(double));
    memset(r, 0, sizeof(double) * m);
    #pragma omp parallel for collapse(2) schedule(static)
    for (int z = 1; z < D - 1; ++z)
        for (int y = 1; y < H - 1; ++y)
            for (int x = 1; x < W - 1; ++x) {
#define U(zz, yy, xx) u[IX(zz, yy, xx)]
                double hxx = U(z, y, x - 1) - 2.0 * U(z, y, x) + U(z, y, x + 1);
                double hyy = U(z, y - 1, x) - 2.0 * U(z, y, x) + U(z, y + 1, x);
                double hzz = U(z - 1, y, x) - 2.0 * U(z, y, x) + U(z + 1, y, x);
                double hxy = (U(z, y - 1, x - 1) + U(z, y + 1, x + 1) - U(z, y + 1, x - 1) - U(z, y - 1, x + 1)) / 4.0;
                double hxz = (U(z - 1, y, x - 1) + U(z + 1, y, x + 1) - U(z + 1, y, x - 1) - U(z - 1, y, x + 1)) / 4.0;
                double hyz = (U(z - 1, y - 1, x) + U(z + 1, y + 1, x) - U(z + 1, y - 1, x) - U(z - 1, y + 1, x)) / 4.0;
#undef U
                double h[9] = {hxx, hxy, hxz, hxy, hyy, hyz, hxz, hyz, hzz};
                size_t p = IX(z, y, x);
                const double *Dm = Dall + 81 * p;
                for (int i = 0; i < 9; ++i) {
                    double s = 0.0;
                    for (int j = 0; j < 9; ++j) s += Dm[9 * i + j] * h[j];
                    t[9 * p + i] = s;
                }
            }
    /* rows three apart in z never touch the same output voxel */
    for (int phase = 0; phase < 3; ++phase) {
        #pragma omp parallel for schedule(static)
        for (int z = 1 + phase; z < D - 1; z += 3)
            for (int y = 1; y < H - 1; ++y)
                for (int x = 1; x < W - 1; ++x) {
                    const double *tp = t + 9 * IX(z, y, x);
#define R(zz, yy, xx) r[IX(zz, yy, xx)]
                    R(z, y, x - 1) += tp[0]; R(z, y, x) -= 2.0 * tp[0]; R(z, y, x + 1) += tp[0];
                    R(z, y - 1, x) += tp[4]; R(z, y, x) -= 2.0 * tp[4]; R(z, y + 1, x) += tp[4];
                    R(z - 1, y, x) += tp[8]; R(z, y, x) -= 2.0 * tp[8]; R(z + 1, y, x) += tp[8];
                    for (int k = 0; k < 2; ++k) {
                        double a = tp[k == 0 ? 1 : 3] / 4.0;   /* xy and yx */
                        R(z, y - 1, x - 1) += a; R(z, y + 1, x + 1) += a; R(z, y + 1, x - 1) -= a; R(z, y - 1, x + 1) -= a;
                        double b = tp[k == 0 ? 2 : 6] / 4.0;   /* xz and zx */
                        R(z - 1, y, x - 1) += b; R(z + 1, y, x + 1) += b; R(z + 1, y, x - 1) -= b; R(z - 1, y, x + 1) -= b;
                        double c = tp[k == 0 ? 5 : 7] / 4.0;   /* yz and zy */
                        R(z - 1, y - 1, x) += c; R(z + 1, y + 1, x) += c; R(z + 1, y - 1, x) -= c; R(z - 1, y + 1, x) -= c;
                    }
#undef R
                }
    }
    free(t);
}

void ref3_fed_cycle(double *u, const double *Dall, int D, int H, int W, const double *taus, int n)
{
    size_t m = (size_t)D * H * W;
    double *r = (double *)malloc(sizeof(double) * m);
    for (int i = 0; i < n; ++i) {
        ref3_apply_P(u, Dall, D, H, W, r);
        for (size_t p = 0; p < m; ++p) u[p] -= taus[i] * r[p];
    }
    free(r);
}

/* The 3-D filter: M cycles of selection, tensor and n FED substeps (the
 * kappa-ordered Eq. (23) steps for tau_max). idx_rec (nullable) [M][m],
 * c_rec (nullable) [M]. Returns 0. */
int ref3_filter(const double *u_in, double *u_out, int D, int H, int W, int ns, const double *sigmas, int mode,
                double lambda, double rho, double alpha, double beta, double c_param, int M, int n, double tau_max,
                uint8_t *idx_rec, double *c_rec)
{
    size_t m = (size_t)D * H * W;
    double *taus = (double *)malloc(sizeof(double) * n);
    int *perm = (int *)malloc(sizeof(int) * n);
    ref_fed_schedule(n, tau_max, taus, perm);
    memcpy(u_out, u_in, sizeof(double) * m);
    uint8_t *idx = (uint8_t *)malloc(m);
    double *hr = (double *)malloc(sizeof(double) * 6 * m);
    double *Dall = (double *)malloc(sizeof(double) * 81 * m);
    for (int k = 0; k < M; ++k) {
        double c = 0.0;
        ref3_scale_select(u_out, D, H, W, ns, sigmas, mode, alpha, beta, c_param, idx, NULL, &c);
        ref3_tensor(u_out, D, H, W, idx, ns, sigmas, rho, hr);
        ref3_dtensor(hr, D, H, W, lambda, mode, Dall);
        ref3_fed_cycle(u_out, Dall, D, H, W, taus, n);
        if (idx_rec) memcpy(idx_rec + k * m, idx, m);
        if (c_rec) c_rec[k] = c;
    }
    free(taus); free(perm); free(idx); free(hr); free(Dall);
    return 0;
}
