/*
 * Driver of the FP64 oracle for a sanitizer build -- TEST INFRASTRUCTURE
 * ONLY. tests/test_oracle_sanitize.py compiles it together with the oracle's
 * sources under AddressSanitizer and UndefinedBehaviorSanitizer and runs it.
 * It calls every entry point of the oracle on small seeded inputs, odd sizes
 * and the smallest shapes the filter accepts, so that an out-of-bounds
 * access, a use after free, a leak or an undefined operation anywhere in the
 * oracle ends the run with a report. It checks no values (the pin tests do).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct ref_opts {
    int model;
    int postprocess;
    double theta;
    const uint8_t *idx_inject;
} ref_opts;

int ref_filter(const double *u_in, double *u_out, int H, int W, int ns, const double *sigmas, int mode,
               double lambda, double rho, double beta, double c_param, int M, int n_substeps, double stop_time,
               double tau_max, int reselect, uint8_t *idx_rec, double *c_rec, double *hrho_rec, double *u_rec,
               const ref_opts *opts);
int ref3_filter(const double *u_in, double *u_out, int D, int H, int W, int ns, const double *sigmas, int mode,
                double lambda, double rho, double alpha, double beta, double c_param, int M, int n, double tau_max,
                uint8_t *idx_rec, double *c_rec);
void ref_crease_field(const double *u, int H, int W, double sigma_d, double *planes);
long ref_marching_creases(const double *planes, int H, int W, double strength, int mode, double *seg,
                          int8_t *type);
void ref_crease_match(const double *seg, const int8_t *type, int H, int W, const double *gt, const int *gt_type,
                      long n, double radius, double *dist_out, long *match_out);
int net_param_count(void);
double net_grad(const double *theta, const double *u, const uint8_t *label, int B, int H, int W, double w_conf,
                double *grad);
void net_forward_bf16(const double *theta, const double *u, int B, int H, int W, double *z);

static unsigned state = 12345u;
static double frand(void)
{
    state = state * 1664525u + 1013904223u;
    return (double)(state >> 8) / 16777216.0;
}

static void *xmalloc(size_t n)
{
    void *p = malloc(n ? n : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

static void filters_2d(int H, int W)
{
    const size_t m = (size_t)H * W;
    const double sig[3] = {1.0, 1.5, 2.2};
    const int M = 2;
    double *u = xmalloc(sizeof(double) * m), *out = xmalloc(sizeof(double) * m);
    uint8_t *idx = xmalloc((size_t)M * m);
    double *c = xmalloc(sizeof(double) * M), *hr = xmalloc(sizeof(double) * 3 * m * M);
    double *ur = xmalloc(sizeof(double) * m * M);
    for (size_t p = 0; p < m; ++p) u[p] = frand();
    for (int mode = 0; mode < 3; ++mode)
        ref_filter(u, out, H, W, 3, sig, mode, 0.005, 0.5, 0.5, -1.0, M, 5, 0.0, 0.05, 1, idx, c, hr, ur, NULL);
    ref_filter(u, out, H, W, 3, sig, 2, INFINITY, 0.0, 0.5, 0.2, M, 4, 0.0, 0.05, 0, NULL, NULL, NULL, NULL, NULL);
    ref_filter(u, out, H, W, 3, sig, 1, 0.005, 0.5, 0.5, -1.0, M, 0, 1.5, 0.05, 1, NULL, NULL, NULL, NULL, NULL);
    const ref_opts ifod = {1, 0, 0.0, NULL}, post = {0, 1, 0.2, NULL}, inject = {0, 0, 0.0, idx};
    ref_filter(u, out, H, W, 1, sig, 2, 0.005, 0.5, 0.5, -1.0, M, 5, 0.0, 0.05, 1, idx, c, hr, ur, &ifod);
    ref_filter(u, out, H, W, 3, sig, 0, 0.005, 0.5, 0.5, -1.0, M, 5, 0.0, 0.05, 1, idx, c, hr, ur, &post);
    ref_filter(u, out, H, W, 3, sig, 2, 0.005, 0.5, 0.5, -1.0, M, 5, 0.0, 0.05, 1, NULL, NULL, NULL, NULL,
               &inject);
    // creases of the filtered image and matching against a few segments
    double *planes = xmalloc(sizeof(double) * 6 * m);
    const size_t cells = (size_t)(H - 1) * (W - 1);
    double *seg = xmalloc(sizeof(double) * cells * 8);
    int8_t *type = xmalloc(cells * 2);
    ref_crease_field(out, H, W, 1.0, planes);
    for (int mode = 0; mode < 3; ++mode) ref_marching_creases(planes, H, W, 0.0, mode, seg, type);
    const long ng = 5;
    double gt[4 * 5];
    int gt_type[5];
    double dist[5];
    long match[5];
    for (long i = 0; i < ng; ++i) {
        for (int k = 0; k < 4; ++k) gt[4 * i + k] = frand() * (k % 2 ? H - 1 : W - 1);
        gt_type[i] = i % 2 ? -1 : 1;
    }
    ref_crease_match(seg, type, H, W, gt, gt_type, ng, 6.0, dist, match);
    free(u), free(out), free(idx), free(c), free(hr), free(ur), free(planes), free(seg), free(type);
}

static void filters_3d(int D, int H, int W)
{
    const size_t m = (size_t)D * H * W;
    const double sig[2] = {1.0, 1.5};
    const int M = 2;
    double *u = xmalloc(sizeof(double) * m), *out = xmalloc(sizeof(double) * m);
    uint8_t *idx = xmalloc((size_t)M * m);
    double c[2];
    for (size_t p = 0; p < m; ++p) u[p] = frand();
    for (int mode = 0; mode < 3; ++mode)
        ref3_filter(u, out, D, H, W, 2, sig, mode, 0.005, 0.5, 0.5, 0.5, -1.0, M, 3, 1.0 / 27.0, idx, c);
    free(u), free(out), free(idx);
}

static void network(int B, int H, int W)
{
    const size_t m = (size_t)B * H * W;
    const int np = net_param_count();
    double *th = xmalloc(sizeof(double) * np), *g = xmalloc(sizeof(double) * np);
    double *u = xmalloc(sizeof(double) * m), *z = xmalloc(sizeof(double) * m * 9);
    uint8_t *lab = xmalloc(m);
    for (int i = 0; i < np; ++i) th[i] = 0.2 * (frand() - 0.5);
    for (size_t p = 0; p < m; ++p) {
        u[p] = frand();
        lab[p] = (uint8_t)(frand() * 8.0);
    }
    net_grad(th, u, lab, B, H, W, 0.1, g);
    net_forward_bf16(th, u, B, H, W, z);
    free(th), free(g), free(u), free(z), free(lab);
}

int main(void)
{
    const int shapes[][2] = {{3, 3}, {3, 11}, {5, 7}, {17, 9}, {33, 40}};
    for (unsigned i = 0; i < sizeof shapes / sizeof shapes[0]; ++i) filters_2d(shapes[i][0], shapes[i][1]);
    const int vols[][3] = {{3, 3, 3}, {4, 5, 6}, {9, 8, 7}};
    for (unsigned i = 0; i < sizeof vols / sizeof vols[0]; ++i) filters_3d(vols[i][0], vols[i][1], vols[i][2]);
    network(2, 5, 7);
    network(1, 17, 16);
    printf("oracle sanitizer run: ok\n");
    return 0;
}
