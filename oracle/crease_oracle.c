/*
 * FP64 CPU oracle of crease extraction and its evaluation -- TEST
 * INFRASTRUCTURE ONLY (see mf4d_oracle.c for the rules; this file shares
 * nothing with the GPU library either).
 *
 * Sec. 3.6: creases are taken from the zero contour of the scalar field
 * d = det(g | Hg) of the filtered image by marching squares; Sec. 4: each
 * ground-truth segment is matched to the reconstructed segment of least
 * Hausdorff distance within a neighbourhood (6 px on synthetic data), and
 * the mean distance E and the detected share p are reported.
 *
 * Readings (the paper leaves these open):
 *  - g and H are the central differences of Sec. 3.4 applied to
 *    u_sigma = G_sigma * u (sigma = sigma_d, symmetric extension), as for
 *    the scale stack;
 *  - a corner is inside when d >= 0; the crossing on an edge from corner a
 *    to corner b is a + t (b - a) with t = d_a / (d_a - d_b); saddle cells
 *    (two opposite corners inside) are split by the sign of the mean of the
 *    four corners;
 *  - the zero set of d is a superset of the creases: it also holds the lines
 *    where the gradient along a crease vanishes, which cross the crease,
 *    and contours in flat regions. A segment is kept as a crease when, with
 *    H interpolated linearly along each crossed edge, both ends have the
 *    same type -- ridge where the eigenvalue of larger magnitude is
 *    negative, valley where it is positive (that eigenvalue's magnitude at
 *    least `strength`; none for equal eigenvalues) -- which the mode
 *    allows, and when the segment runs closer to the eigenvector of the
 *    weaker eigenvalue than to that of the stronger (at the mean of the two
 *    ends' Hessians), i.e. along the crease. The gradient's own direction
 *    is not used: the linear interpolation of d places a crossing a tenth
 *    of a pixel off the crest where the gradient along the crest is weak,
 *    and there the gradient points across it, while H and the contour's
 *    direction change slowly;
 *  - segments are stored per cell (x, y), corners (x, y), (x+1, y),
 *    (x+1, y+1), (x, y+1), in two slots sorted by their first edge (edges
 *    0 top, 1 right, 2 bottom, 3 left), ends ordered by edge;
 *  - a ground-truth segment G is matched by the directed Hausdorff distance
 *    from G to a reconstructed segment R, the largest distance of a point
 *    of G to R (attained at an end of G): the ground truth is a dense
 *    sampling of each centreline while the reconstruction has one piece per
 *    cell, so the two sets' pieces have unrelated lengths and positions
 *    along a crease, and the symmetric distance would charge a
 *    reconstruction lying on the crest for its extent along it; the
 *    distance reported for a matched ground-truth segment is that of its
 *    midpoint to its match.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

void ref_blur(const double *u, int H, int W, double sigma, double *out);
void ref_derivatives(const double *v, int H, int W, double *ux, double *uy,
                     double *uxx, double *uxy, double *uyy);

/* Planes [6][H][W]: g_x, g_y, h_xx, h_xy, h_yy of u_sigma and
 * d = det(g | Hg) = g_x (H g)_y - g_y (H g)_x. */
void ref_crease_field(const double *u, int H, int W, double sigma_d, double *planes)
{
    size_t m = (size_t)H * W;
    double *us = (double *)malloc(sizeof(double) * m);
    ref_blur(u, H, W, sigma_d, us);
    double *gx = planes, *gy = planes + m, *hxx = planes + 2 * m, *hxy = planes + 3 * m,
           *hyy = planes + 4 * m, *d = planes + 5 * m;
    ref_derivatives(us, H, W, gx, gy, hxx, hxy, hyy);
    for (size_t p = 0; p < m; ++p) {
        double hgx = hxx[p] * gx[p] + hxy[p] * gy[p];
        double hgy = hxy[p] * gx[p] + hyy[p] * gy[p];
        d[p] = gx[p] * hgy - gy[p] * hgx;
    }
    free(us);
}

/* Crease type of a point with Hessian (a, b, c): +1 ridge (stronger
 * eigenvalue negative), -1 valley (positive), 0 none (equal magnitudes or
 * below strength). The stronger eigenvalue is m + r for m > 0 and m - r for
 * m < 0, with m = (a + c) / 2 and r = sqrt(((a - c) / 2)^2 + b^2). */
static int crease_type(double a, double b, double c, double strength)
{
    double m = 0.5 * (a + c);
    double r = sqrt(0.25 * (a - c) * (a - c) + b * b);
    if (!(r > 0.0) || m == 0.0) return 0;
    if (fabs(m) + r < strength) return 0;
    return m < 0.0 ? 1 : -1;
}

/* Does direction v run closer to the weaker eigenvector of H = (a, b, c)
 * than to the stronger one? With q = v^T (H - m Id) v, (v.e1)^2 - (v.e2)^2
 * has the sign of q (e1 the eigenvector of m + r); the stronger one is e1
 * when m > 0 and e2 when m < 0. */
static int along_weak(double vx, double vy, double a, double b, double c)
{
    double m = 0.5 * (a + c);
    double q = 0.5 * (a - c) * (vx * vx - vy * vy) + 2.0 * b * vx * vy;
    return m > 0.0 ? q <= 0.0 : q >= 0.0;
}

/* Segment edge pairs per inside-pattern (bit k = corner k inside), for the
 * non-saddle cases; -1 = none. */
static void cell_edges(int pat, double centre, int *n, int e[2][2])
{
    *n = 0;
    switch (pat) {
    case 0: case 15: return;
    case 1: case 14: e[0][0] = 0; e[0][1] = 3; *n = 1; return;   /* corner 0 alone */
    case 2: case 13: e[0][0] = 0; e[0][1] = 1; *n = 1; return;   /* corner 1 alone */
    case 4: case 11: e[0][0] = 1; e[0][1] = 2; *n = 1; return;   /* corner 2 alone */
    case 8: case 7: e[0][0] = 2; e[0][1] = 3; *n = 1; return;    /* corner 3 alone */
    case 3: case 12: e[0][0] = 1; e[0][1] = 3; *n = 1; return;   /* corners 0, 1 vs 2, 3 */
    case 6: case 9: e[0][0] = 0; e[0][1] = 2; *n = 1; return;    /* corners 1, 2 vs 3, 0 */
    case 5:   /* corners 0 and 2 inside */
        if (centre >= 0.0) { e[0][0] = 0; e[0][1] = 1; e[1][0] = 2; e[1][1] = 3; }   /* cut 1 and 3 off */
        else { e[0][0] = 0; e[0][1] = 3; e[1][0] = 1; e[1][1] = 2; }                 /* cut 0 and 2 off */
        *n = 2;
        return;
    case 10:  /* corners 1 and 3 inside */
        if (centre >= 0.0) { e[0][0] = 0; e[0][1] = 3; e[1][0] = 1; e[1][1] = 2; }   /* cut 0 and 2 off */
        else { e[0][0] = 0; e[0][1] = 1; e[1][0] = 2; e[1][1] = 3; }                 /* cut 1 and 3 off */
        *n = 2;
        return;
    }
}

/* Marching squares on d with the crease test at both ends of each segment.
 * seg: [H-1][W-1][2][4] (x0, y0, x1, y1); type: [H-1][W-1][2], 0 = empty.
 * mode: 0 ridges, 1 valleys, 2 both. Returns the number of segments. */
long ref_marching_creases(const double *planes, int H, int W, double strength, int mode,
                          double *seg, int8_t *type)
{
    size_t m = (size_t)H * W;
    const double *hxx = planes + 2 * m, *hxy = planes + 3 * m, *hyy = planes + 4 * m, *d = planes + 5 * m;
    long count = 0;
    /* corner k of cell (x, y) and the corners (a, b) of edge e */
    const int cx[4] = {0, 1, 1, 0}, cy[4] = {0, 0, 1, 1};
    const int ea[4] = {0, 1, 2, 3}, eb[4] = {1, 2, 3, 0};
    for (int y = 0; y + 1 < H; ++y) {
        for (int x = 0; x + 1 < W; ++x) {
            size_t cell = (size_t)y * (W - 1) + x;
            double *s = seg + 8 * cell;
            int8_t *t = type + 2 * cell;
            memset(s, 0, sizeof(double) * 8);
            t[0] = t[1] = 0;
            size_t pc[4];
            double dc[4];
            int pat = 0;
            for (int k = 0; k < 4; ++k) {
                pc[k] = (size_t)(y + cy[k]) * W + (x + cx[k]);
                dc[k] = d[pc[k]];
                if (dc[k] >= 0.0) pat |= 1 << k;
            }
            double centre = 0.25 * (dc[0] + dc[1] + dc[2] + dc[3]);
            int ns, e[2][2];
            cell_edges(pat, centre, &ns, e);
            int slot = 0;
            for (int q = 0; q < ns; ++q) {
                double px[2], py[2], ha[2], hb[2], hc[2];
                int ty[2];
                for (int j = 0; j < 2; ++j) {
                    int ed = e[q][j], a = ea[ed], b = eb[ed];
                    double tt = dc[a] / (dc[a] - dc[b]);
                    px[j] = (double)(x + cx[a]) + tt * (double)(cx[b] - cx[a]);
                    py[j] = (double)(y + cy[a]) + tt * (double)(cy[b] - cy[a]);
                    size_t pa = pc[a], pb = pc[b];
                    ha[j] = hxx[pa] + tt * (hxx[pb] - hxx[pa]);
                    hb[j] = hxy[pa] + tt * (hxy[pb] - hxy[pa]);
                    hc[j] = hyy[pa] + tt * (hyy[pb] - hyy[pa]);
                    ty[j] = crease_type(ha[j], hb[j], hc[j], strength);
                }
                if (ty[0] == 0 || ty[0] != ty[1]) continue;
                if (!along_weak(px[1] - px[0], py[1] - py[0], 0.5 * (ha[0] + ha[1]), 0.5 * (hb[0] + hb[1]),
                                0.5 * (hc[0] + hc[1])))
                    continue;
                if (mode == 0 && ty[0] != 1) continue;
                if (mode == 1 && ty[0] != -1) continue;
                s[4 * slot + 0] = px[0];
                s[4 * slot + 1] = py[0];
                s[4 * slot + 2] = px[1];
                s[4 * slot + 3] = py[1];
                t[slot] = (int8_t)ty[0];
                ++slot;
                ++count;
            }
        }
    }
    return count;
}

static double point_segment(double px, double py, double ax, double ay, double bx, double by)
{
    double vx = bx - ax, vy = by - ay;
    double l2 = vx * vx + vy * vy;
    double t = 0.0;
    if (l2 > 0.0) {
        t = ((px - ax) * vx + (py - ay) * vy) / l2;
        if (t < 0.0) t = 0.0;
        if (t > 1.0) t = 1.0;
    }
    double dx = px - (ax + t * vx), dy = py - (ay + t * vy);
    return sqrt(dx * dx + dy * dy);
}

/* Directed Hausdorff distance from segment A = (a0, a1) to segment
 * B = (b0, b1): the largest distance of a point of A to B, attained at an
 * end of A (the distance to a segment is convex along a line). */
double ref_segment_hausdorff(const double *A, const double *B)
{
    double h = point_segment(A[0], A[1], B[0], B[1], B[2], B[3]);
    double v = point_segment(A[2], A[3], B[0], B[1], B[2], B[3]);
    return v > h ? v : h;
}

/* For each ground-truth segment gt[i] (x0, y0, x1, y1) of type gt_type[i]:
 * among the reconstructed segments of that type with directed Hausdorff
 * distance (from gt[i]) <= radius, the one of least distance (ties: the first cell in row-major
 * order, then slot 0); dist_out[i] = distance of gt[i]'s midpoint to it and
 * match_out[i] = 2 * cell + slot, or -1 / -1 when there is none. Only cells
 * that can hold such a segment are visited (a segment within that distance
 * passes within radius of gt[i]'s ends, so it meets gt[i]'s bounding box
 * grown by radius, and the cell of a segment holds all its points). */
void ref_crease_match(const double *seg, const int8_t *type, int H, int W, const double *gt,
                      const int *gt_type, long n, double radius, double *dist_out, long *match_out)
{
    #pragma omp parallel for schedule(dynamic, 64)
    for (long i = 0; i < n; ++i) {
        const double *G = gt + 4 * i;
        double lox = fmin(G[0], G[2]) - radius, hix = fmax(G[0], G[2]) + radius;
        double loy = fmin(G[1], G[3]) - radius, hiy = fmax(G[1], G[3]) + radius;
        int x0 = (int)floor(lox) - 1, x1 = (int)ceil(hix) + 1;
        int y0 = (int)floor(loy) - 1, y1 = (int)ceil(hiy) + 1;
        if (x0 < 0) x0 = 0;
        if (y0 < 0) y0 = 0;
        if (x1 > W - 2) x1 = W - 2;
        if (y1 > H - 2) y1 = H - 2;
        double best = INFINITY;
        long bm = -1;
        for (int y = y0; y <= y1; ++y)
            for (int x = x0; x <= x1; ++x)
                for (int sl = 0; sl < 2; ++sl) {
                    size_t c = (size_t)y * (W - 1) + x;
                    if (type[2 * c + sl] != gt_type[i]) continue;
                    double h = ref_segment_hausdorff(G, seg + 8 * c + 4 * sl);
                    if (h <= radius && h < best) { best = h; bm = (long)(2 * c + sl); }
                }
        match_out[i] = bm;
        if (bm < 0) { dist_out[i] = -1.0; continue; }
        const double *R = seg + 4 * bm;
        dist_out[i] = point_segment(0.5 * (G[0] + G[2]), 0.5 * (G[1] + G[3]), R[0], R[1], R[2], R[3]);
    }
}
