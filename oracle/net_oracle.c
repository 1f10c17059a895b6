/*
 * FP64 CPU oracle of the learned scale surrogate -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain-loop reference of the 5-layer 3x3 convolutional network that
 * predicts, per pixel, the index of the selected Gaussian scale (8 logits)
 * and a confidence logit, with its training loss and the gradients of that
 * loss. It is what the GPU's MFMA forward and backward kernels are checked
 * against; it is itself pinned by central finite differences in the tests.
 * It shares no code with the GPU library.
 *
 * Network: layers l = 0..4, 3x3 convolutions with zero padding,
 *   a_{l+1} = relu(conv(a_l, W_l) + b_l) for l < 4, z = conv(a_4, W_4) + b_4,
 *   channels 1 -> 32 -> 32 -> 32 -> 32 -> 9. W_l is [cout][cin][3][3].
 * Loss (mean over pixels): softmax cross-entropy of z[0..7] against the
 *   label, plus w_conf times the binary cross-entropy of sigmoid(z[8])
 *   against t = (argmax z[0..7] == label); t is a constant of the loss.
 * Layout: activations [B][C][H][W], double.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static const int NET_C[6] = {1, 32, 32, 32, 32, 9};

int net_param_count(void)
{
    int n = 0;
    for (int l = 0; l < 5; ++l) n += NET_C[l + 1] * NET_C[l] * 9 + NET_C[l + 1];
    return n;
}

/* parameter vector: for each layer W_l (cout*cin*9) then b_l (cout) */
static const double *layer_w(const double *theta, int l)
{
    const double *p = theta;
    for (int k = 0; k < l; ++k) p += NET_C[k + 1] * NET_C[k] * 9 + NET_C[k + 1];
    return p;
}

static void conv3x3(const double *in, int B, int cin, int H, int W, const double *w, const double *b, int cout,
                    double *out)
{
    /* OpenMP only splits the independent output planes */
    #pragma omp parallel for collapse(2) schedule(static)
    for (int n = 0; n < B; ++n)
        for (int co = 0; co < cout; ++co)
            for (int y = 0; y < H; ++y)
                for (int x = 0; x < W; ++x) {
                    double s = b[co];
                    for (int ci = 0; ci < cin; ++ci)
                        for (int dy = -1; dy <= 1; ++dy)
                            for (int dx = -1; dx <= 1; ++dx) {
                                const int yy = y + dy, xx = x + dx;
                                if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                                s += w[((co * cin + ci) * 3 + dy + 1) * 3 + dx + 1] *
                                     in[((size_t)(n * cin + ci) * H + yy) * W + xx];
                            }
                    out[((size_t)(n * cout + co) * H + y) * W + x] = s;
                }
}

/* Forward pass. acts (nullable) receives a_1..a_4 ([4][B][32][H][W]);
 * z receives the output [B][9][H][W]. */
void net_forward(const double *theta, const double *u, int B, int H, int W, double *acts, double *z)
{
    size_t m = (size_t)B * H * W;
    double *a = (double *)malloc(sizeof(double) * m * 32);
    double *t = (double *)malloc(sizeof(double) * m * 32);
    memcpy(a, u, sizeof(double) * m);
    for (int l = 0; l < 5; ++l) {
        const double *w = layer_w(theta, l);
        const double *b = w + NET_C[l + 1] * NET_C[l] * 9;
        conv3x3(a, B, NET_C[l], H, W, w, b, NET_C[l + 1], l < 4 ? t : z);
        if (l < 4) {
            for (size_t i = 0; i < m * 32; ++i) t[i] = t[i] > 0.0 ? t[i] : 0.0;
            if (acts) memcpy(acts + (size_t)l * m * 32, t, sizeof(double) * m * 32);
            double *s = a;
            a = t;
            t = s;
        }
    }
    free(a);
    free(t);
}

/* Loss of the forward output z against labels; dz (nullable) receives
 * dLoss/dz. Returns the loss. */
double net_loss(const double *z, const uint8_t *label, int B, int H, int W, double w_conf, double *dz)
{
    const size_t hw = (size_t)H * W, m = (size_t)B * hw;
    double loss = 0.0;
    for (int n = 0; n < B; ++n)
        for (size_t p = 0; p < hw; ++p) {
            double zz[9];
            for (int k = 0; k < 9; ++k) zz[k] = z[(n * 9 + k) * hw + p];
            double mx = zz[0];
            int am = 0;
            for (int k = 1; k < 8; ++k)
                if (zz[k] > mx) { mx = zz[k]; am = k; }
            double se = 0.0;
            for (int k = 0; k < 8; ++k) se += exp(zz[k] - mx);
            const int y = label[n * hw + p];
            loss += -(zz[y] - mx - log(se));
            const double tgt = (am == y) ? 1.0 : 0.0;
            const double c = 1.0 / (1.0 + exp(-zz[8]));
            /* BCE with logits, stable form */
            loss += w_conf * (fmax(zz[8], 0.0) - zz[8] * tgt + log1p(exp(-fabs(zz[8]))));
            if (dz) {
                for (int k = 0; k < 8; ++k)
                    dz[(n * 9 + k) * hw + p] = (exp(zz[k] - mx) / se - (k == y ? 1.0 : 0.0)) / (double)m;
                dz[(n * 9 + 8) * hw + p] = w_conf * (c - tgt) / (double)m;
            }
        }
    return loss / (double)m;
}

/* Gradient of the loss with respect to theta (by the chain rule through the
 * layers in reverse order). Returns the loss. */
double net_grad(const double *theta, const double *u, const uint8_t *label, int B, int H, int W, double w_conf,
                double *grad)
{
    const size_t m = (size_t)B * H * W;
    double *acts = (double *)malloc(sizeof(double) * 4 * m * 32);
    double *z = (double *)malloc(sizeof(double) * m * 9);
    double *d = (double *)malloc(sizeof(double) * m * 32);
    double *dn = (double *)malloc(sizeof(double) * m * 32);
    net_forward(theta, u, B, H, W, acts, z);
    const double loss = net_loss(z, label, B, H, W, w_conf, d);
    memset(grad, 0, sizeof(double) * net_param_count());
    for (int l = 4; l >= 0; --l) {
        const int cin = NET_C[l], cout = NET_C[l + 1];
        const double *in = l == 0 ? u : acts + (size_t)(l - 1) * m * 32;
        const double *w = layer_w(theta, l);
        double *gw = grad + (layer_w(theta, l) - theta);
        double *gb = gw + cout * cin * 9;
        /* d holds dLoss/d(pre-activation output of layer l), [B][cout][H][W] */
        for (int n = 0; n < B; ++n)
            for (int co = 0; co < cout; ++co)
                for (int y = 0; y < H; ++y)
                    for (int x = 0; x < W; ++x) {
                        const double g = d[((size_t)(n * cout + co) * H + y) * W + x];
                        gb[co] += g;
                        for (int ci = 0; ci < cin; ++ci)
                            for (int dy = -1; dy <= 1; ++dy)
                                for (int dx = -1; dx <= 1; ++dx) {
                                    const int yy = y + dy, xx = x + dx;
                                    if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                                    gw[((co * cin + ci) * 3 + dy + 1) * 3 + dx + 1] +=
                                        g * in[((size_t)(n * cin + ci) * H + yy) * W + xx];
                                }
                    }
        if (l == 0) break;
        /* input gradient, then the relu of the layer below */
        memset(dn, 0, sizeof(double) * m * cin);
        for (int n = 0; n < B; ++n)
            for (int co = 0; co < cout; ++co)
                for (int y = 0; y < H; ++y)
                    for (int x = 0; x < W; ++x) {
                        const double g = d[((size_t)(n * cout + co) * H + y) * W + x];
                        for (int ci = 0; ci < cin; ++ci)
                            for (int dy = -1; dy <= 1; ++dy)
                                for (int dx = -1; dx <= 1; ++dx) {
                                    const int yy = y + dy, xx = x + dx;
                                    if (yy < 0 || yy >= H || xx < 0 || xx >= W) continue;
                                    dn[((size_t)(n * cin + ci) * H + yy) * W + xx] +=
                                        g * w[((co * cin + ci) * 3 + dy + 1) * 3 + dx + 1];
                                }
                    }
        for (size_t i = 0; i < m * cin; ++i) d[i] = in[i] > 0.0 ? dn[i] : 0.0;
    }
    free(acts);
    free(z);
    free(d);
    free(dn);
    return loss;
}

/* The network as the library defines it for inference (BF16 weights, inputs
 * and activations): the input, the weights and every layer's activation
 * (relu of the layer's output rounded to float) are rounded to BF16, round to
 * nearest even; sums are taken in double, the biases are used as given and
 * the logits are not rounded. z receives [B][9][H][W]. */
static double bf16_of(double v)
{
    float f = (float)v;
    uint32_t b;
    memcpy(&b, &f, sizeof b);
    b += 0x7fffu + ((b >> 16) & 1u);
    b &= 0xffff0000u;
    memcpy(&f, &b, sizeof f);
    return (double)f;
}

void net_forward_bf16(const double *theta, const double *u, int B, int H, int W, double *z)
{
    size_t m = (size_t)B * H * W;
    int np = net_param_count();
    double *th = (double *)malloc(sizeof(double) * (size_t)np);
    memcpy(th, theta, sizeof(double) * (size_t)np);
    for (int l = 0; l < 5; ++l) {   /* weights to BF16, biases kept */
        double *w = th + (layer_w(theta, l) - theta);
        for (int i = 0; i < NET_C[l + 1] * NET_C[l] * 9; ++i) w[i] = bf16_of(w[i]);
    }
    double *a = (double *)malloc(sizeof(double) * m * 32);
    double *t = (double *)malloc(sizeof(double) * m * 32);
    for (size_t i = 0; i < m; ++i) a[i] = bf16_of(u[i]);
    for (int l = 0; l < 5; ++l) {
        const double *w = th + (layer_w(theta, l) - theta);
        const double *b = w + NET_C[l + 1] * NET_C[l] * 9;
        conv3x3(a, B, NET_C[l], H, W, w, b, NET_C[l + 1], l < 4 ? t : z);
        if (l < 4) {
            for (size_t i = 0; i < m * 32; ++i) t[i] = bf16_of(t[i] > 0.0 ? t[i] : 0.0);
            double *s = a;
            a = t;
            t = s;
        }
    }
    free(a);
    free(t);
    free(th);
}
