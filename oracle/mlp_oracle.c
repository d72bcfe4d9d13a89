/*
 * mlp_oracle.c -- plain FP64 CPU reference of the pair-scoring network of the
 * learned form, and of its loss gradient.  TEST INFRASTRUCTURE ONLY: used by
 * the tests to check the GPU training kernels; shares no code with them.
 *
 * Network: x (4) -> h1 = relu(W1 x + b1) (64) -> h2 = relu(W2 h1 + b2) (64)
 *          -> z = w3 . h2 + b3 (a logit).
 * Loss over a batch of n samples with labels y in {0,1} and positive weight p:
 *   L = (1/n) sum_s [ p y_s softplus(-z_s) + (1 - y_s) softplus(z_s) ]
 * (binary cross-entropy with logits).  Parameter vector layout (4545 values):
 *   W1[64][4], b1[64], W2[64][64], b2[64], w3[64], b3.
 * Backward pass written out from the chain rule; relu'(0) is taken as 0.
 */
#include <math.h>
#include <string.h>

enum { H = 64, IN = 4 };
enum { OFF_W1 = 0, OFF_B1 = OFF_W1 + H * IN, OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + H * H,
       OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + H, NPARAM = OFF_B3 + 1 };

int mo_nparam(void) { return NPARAM; }

static double softplus(double v) { return v > 0 ? v + log1p(exp(-v)) : log1p(exp(v)); }
static double sigmoid(double v) { return v >= 0 ? 1.0 / (1.0 + exp(-v)) : exp(v) / (1.0 + exp(v)); }

/* logits of n samples */
void mo_forward(const double *P, const double *X, int n, double *z)
{
    double h1[H], h2[H];
    for (int s = 0; s < n; ++s) {
        const double *x = X + (size_t)s * IN;
        for (int k = 0; k < H; ++k) {
            double a = P[OFF_B1 + k];
            for (int c = 0; c < IN; ++c) a += P[OFF_W1 + k * IN + c] * x[c];
            h1[k] = a > 0 ? a : 0;
        }
        for (int k = 0; k < H; ++k) {
            double a = P[OFF_B2 + k];
            for (int m = 0; m < H; ++m) a += P[OFF_W2 + k * H + m] * h1[m];
            h2[k] = a > 0 ? a : 0;
        }
        double o = P[OFF_B3];
        for (int k = 0; k < H; ++k) o += P[OFF_W3 + k] * h2[k];
        z[s] = o;
    }
}

/* loss and its gradient with respect to every parameter */
double mo_loss_grad(const double *P, const double *X, const unsigned char *y, int n, double pos_w, double *G)
{
    double h1[H], h2[H], a1[H], a2[H], d2[H], d1[H];
    memset(G, 0, sizeof(double) * NPARAM);
    double L = 0.0;
    for (int s = 0; s < n; ++s) {
        const double *x = X + (size_t)s * IN;
        for (int k = 0; k < H; ++k) {
            double a = P[OFF_B1 + k];
            for (int c = 0; c < IN; ++c) a += P[OFF_W1 + k * IN + c] * x[c];
            a1[k] = a;
            h1[k] = a > 0 ? a : 0;
        }
        for (int k = 0; k < H; ++k) {
            double a = P[OFF_B2 + k];
            for (int m = 0; m < H; ++m) a += P[OFF_W2 + k * H + m] * h1[m];
            a2[k] = a;
            h2[k] = a > 0 ? a : 0;
        }
        double z = P[OFF_B3];
        for (int k = 0; k < H; ++k) z += P[OFF_W3 + k] * h2[k];
        const double ys = y[s] ? 1.0 : 0.0;
        L += pos_w * ys * softplus(-z) + (1.0 - ys) * softplus(z);
        /* dL/dz = -p y sigmoid(-z) + (1 - y) sigmoid(z) */
        const double dz = (-pos_w * ys * sigmoid(-z) + (1.0 - ys) * sigmoid(z)) / n;
        G[OFF_B3] += dz;
        for (int k = 0; k < H; ++k) {
            G[OFF_W3 + k] += dz * h2[k];
            d2[k] = a2[k] > 0 ? dz * P[OFF_W3 + k] : 0.0;
        }
        for (int m = 0; m < H; ++m) d1[m] = 0.0;
        for (int k = 0; k < H; ++k) {
            G[OFF_B2 + k] += d2[k];
            for (int m = 0; m < H; ++m) {
                G[OFF_W2 + k * H + m] += d2[k] * h1[m];
                d1[m] += d2[k] * P[OFF_W2 + k * H + m];
            }
        }
        for (int m = 0; m < H; ++m) {
            const double g = a1[m] > 0 ? d1[m] : 0.0;
            G[OFF_B1 + m] += g;
            for (int c = 0; c < IN; ++c) G[OFF_W1 + m * IN + c] += g * x[c];
        }
    }
    return L / n;
}
