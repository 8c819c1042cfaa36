/*
 * kepler_guess_oracle.c -- plain FP64 CPU oracle of the learned starting
 * value for the universal-variable Kepler solve, its training loss, the
 * loss gradient by backpropagation, and the Adam update.
 *
 * TEST INFRASTRUCTURE ONLY, under the same rules as qsym_oracle.c: the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it;
 * the product path never calls it and shares no code with it.
 *
 * The paper solves Kepler's equation in universal variables (Appendix A)
 * from a fixed start; a learned start is not part of the paper.  What is
 * fixed here is therefore a definition of our own, stated once:
 *
 * Features of a body at (x0, v0) advanced by dt about mu (dt != 0):
 *   r0 = |x0|, s = sign(dt), T = sqrt(mu) |dt| / r0^1.5   (step in units of
 *   the local dynamical time), alpha = 2/r0 - |v0|^2/mu (Appendix A)
 *     f0 = ln r0
 *     f1 = s (x0 . v0) / sqrt(mu r0)
 *     f2 = alpha r0
 *     f3 = ln T
 *   The sign s enters through f1 because Kepler's equation is odd under
 *   (x, x0.v0, dt) -> (-x, -x0.v0, -dt), so a backward step is the forward
 *   step of the time-reversed orbit with the root negated.
 * First-order root x_p = sqrt(mu) dt / r0.  Target of a solved root x:
 *     y = ln(x / x_p) / T
 *   (the deviation from x_p grows with the step, so dividing by T keeps the
 *   target bounded and makes a fixed network error shrink with the step).
 * Network on standardised features i_k = (f_k - m_k) / s_k, tanh units:
 *     h1 = tanh(W1 i + b1)      W1: 32 x 4
 *     h2 = tanh(W2 h1 + b2)     W2: 32 x 32
 *     o  = W3 . h2 + b3         W3: 32
 * Guess: x_g = x_p exp(T (o s_y + m_y)).
 * Parameter vector (1249 values, then 10 scalers):
 *   W1 row-major at 0 (row = first-layer unit), b1 at 128, W2 row-major at
 *   160 (row = second-layer unit, column = first-layer unit), b2 at 1184,
 *   W3 at 1216, b3 at 1248; scalers at 1249: m_0..m_3, s_0..s_3, m_y, s_y.
 * Loss over n samples: L = (1/n) sum (o - (y - m_y)/s_y)^2.
 * Adam: Kingma & Ba (2015), Algorithm 1 (bias-corrected moment estimates).
 *
 * Parity pins (CPU tests): the gradient against central finite differences
 * of the loss; the network wiring against closed forms with sparse weights;
 * the features' scale invariance and time-reversal symmetry; the guess as
 * the exact inverse of the target; Adam against its closed form under a
 * constant gradient; the scalers against an arithmetic sequence.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define G_H 32
#define G_NPARAM 1249
#define G_W1 0
#define G_B1 128
#define G_W2 160
#define G_B2 1184
#define G_W3 1216
#define G_B3 1248

int orc_kepler_root(double mu, const double *x0, const double *v0, double dt, int32_t mode,
                    double x_start, int32_t use_start, double *x_out, int32_t *iters);

/* Features, first-order root and scaled step of one body; returns 1 (and
 * leaves the outputs untouched) when dt == 0. */
int orc_guess_features(double mu, const double *x0, const double *v0, double dt, double *f,
                       double *xp, double *T)
{
    if (dt == 0.0) return 1;
    double r0 = sqrt(x0[0] * x0[0] + x0[1] * x0[1] + x0[2] * x0[2]);
    double vv = v0[0] * v0[0] + v0[1] * v0[1] + v0[2] * v0[2];
    double rv = x0[0] * v0[0] + x0[1] * v0[1] + x0[2] * v0[2];
    double s = dt > 0.0 ? 1.0 : -1.0;
    double alpha = 2.0 / r0 - vv / mu;
    double tt = sqrt(mu) * fabs(dt) / (r0 * sqrt(r0));
    f[0] = log(r0);
    f[1] = s * rv / sqrt(mu * r0);
    f[2] = alpha * r0;
    f[3] = log(tt);
    *xp = sqrt(mu) * dt / r0;
    *T = tt;
    return 0;
}

/* Network output on standardised inputs; h1, h2 (32 each) receive the
 * hidden activations when not NULL. */
double orc_guess_net(const double *w, const double *in, double *h1o, double *h2o)
{
    double h1[G_H], h2[G_H];
    for (int k = 0; k < G_H; ++k) {
        double a = w[G_B1 + k];
        for (int c = 0; c < 4; ++c) a += w[G_W1 + 4 * k + c] * in[c];
        h1[k] = tanh(a);
    }
    double o = w[G_B3];
    for (int k = 0; k < G_H; ++k) {
        double a = w[G_B2 + k];
        for (int c = 0; c < G_H; ++c) a += w[G_W2 + G_H * k + c] * h1[c];
        h2[k] = tanh(a);
        o += w[G_W3 + k] * h2[k];
    }
    if (h1o) memcpy(h1o, h1, sizeof h1);
    if (h2o) memcpy(h2o, h2, sizeof h2);
    return o;
}

static void standardise(const double *w, const double *f, double *in)
{
    const double *sc = w + G_NPARAM;
    for (int c = 0; c < 4; ++c) in[c] = (f[c] - sc[c]) / sc[4 + c];
}

/* Learned starting value of the universal anomaly (w holds 1249 parameters
 * and 10 scalers); 0 for dt == 0. */
double orc_guess(const double *w, double mu, const double *x0, const double *v0, double dt)
{
    double f[4], in[4], xp, T;
    if (orc_guess_features(mu, x0, v0, dt, f, &xp, &T)) return 0.0;
    standardise(w, f, in);
    double o = orc_guess_net(w, in, NULL, NULL);
    const double *sc = w + G_NPARAM;
    return xp * exp(T * (o * sc[9] + sc[8]));
}

/* Target y = ln(x / x_p) / T of a solved root x. */
double orc_guess_target(double mu, const double *x0, const double *v0, double dt, double x)
{
    double f[4], xp, T;
    if (orc_guess_features(mu, x0, v0, dt, f, &xp, &T)) return 0.0;
    return log(x / xp) / T;
}

/* Features [n][4] and targets [n] of n solved bodies (q, v as [n][3]). */
void orc_guess_dataset(int64_t n, double mu, const double *q, const double *v,
                       const double *dt, const double *x, double *f, double *y)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double xp, T;
        orc_guess_features(mu, q + 3 * i, v + 3 * i, dt[i], f + 4 * i, &xp, &T);
        y[i] = log(x[i] / xp) / T;
    }
}

/* Means and population standard deviations of the four feature columns and
 * of the target; a zero deviation is replaced by 1. */
void orc_guess_scalers(int64_t n, const double *f, const double *y, double *sc)
{
    for (int c = 0; c < 5; ++c) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += c < 4 ? f[4 * i + c] : y[i];
        double mean = s / (double)n, q = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            double d = (c < 4 ? f[4 * i + c] : y[i]) - mean;
            q += d * d;
        }
        double sd = sqrt(q / (double)n);
        if (c < 4) {
            sc[c] = mean;
            sc[4 + c] = sd > 0.0 ? sd : 1.0;
        } else {
            sc[8] = mean;
            sc[9] = sd > 0.0 ? sd : 1.0;
        }
    }
}

/* Loss L = (1/n) sum (o - (y - m_y)/s_y)^2 over n samples of raw features
 * f [n][4] and raw targets y [n], and (when grad is not NULL) dL/dw for the
 * 1249 parameters by backpropagation through the two tanh layers. */
double orc_guess_loss_grad(const double *w, int64_t n, const double *f, const double *y,
                           double *grad)
{
    const double *sc = w + G_NPARAM;
    double loss = 0.0;
    if (grad) memset(grad, 0, sizeof(double) * G_NPARAM);
    for (int64_t i = 0; i < n; ++i) {
        double in[4], h1[G_H], h2[G_H];
        standardise(w, f + 4 * i, in);
        double o = orc_guess_net(w, in, h1, h2);
        double e = o - (y[i] - sc[8]) / sc[9];
        loss += e * e;
        if (!grad) continue;
        double d = 2.0 * e / (double)n; /* dL/do */
        grad[G_B3] += d;
        double d2[G_H];
        for (int k = 0; k < G_H; ++k) {
            grad[G_W3 + k] += d * h2[k];
            d2[k] = d * w[G_W3 + k] * (1.0 - h2[k] * h2[k]);
            grad[G_B2 + k] += d2[k];
            for (int c = 0; c < G_H; ++c) grad[G_W2 + G_H * k + c] += d2[k] * h1[c];
        }
        for (int c = 0; c < G_H; ++c) {
            double back = 0.0;
            for (int k = 0; k < G_H; ++k) back += w[G_W2 + G_H * k + c] * d2[k];
            double d1 = back * (1.0 - h1[c] * h1[c]);
            grad[G_B1 + c] += d1;
            for (int j = 0; j < 4; ++j) grad[G_W1 + 4 * c + j] += d1 * in[j];
        }
    }
    return loss / (double)n;
}

/* One Adam update of n parameters at step t >= 1 (Kingma & Ba, Alg. 1). */
void orc_adam(int64_t n, double *w, const double *g, double *m, double *v, int64_t t,
              double lr, double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        w[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* Roots of n bodies with per-body steps (Appendix A solve); x_start [n]
 * (mode 2) may be NULL.  Returns the number of solves that hit the cap. */
int64_t orc_kepler_roots(int64_t n, double mu, const double *q, const double *v,
                         const double *dt, int32_t mode, const double *x_start, double *x,
                         int32_t *iters)
{
    int64_t fails = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : fails)
    for (int64_t i = 0; i < n; ++i)
        fails += orc_kepler_root(mu, q + 3 * i, v + 3 * i, dt[i], mode,
                                 x_start ? x_start[i] : 0.0, x_start != NULL, x + i, iters + i);
    return fails;
}
