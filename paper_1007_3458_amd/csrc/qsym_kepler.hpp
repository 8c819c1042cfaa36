// qsym_kepler.hpp -- universal-variable Kepler solve of one body (Appendix A
// of Moore & Quillen, arXiv:1007.3458) and the learned starting value of its
// Newton iteration, as device functions shared by the step kernels and the
// stand-alone solve/training kernels.
#pragma once
#include "qsym_common.hpp"

namespace qsym {

// ------------------------------------------------------------------------
// Appendix A: Stumpff functions
// ------------------------------------------------------------------------
__device__ __forceinline__ void stumpff(double y, double &C, double &S)
{
    if (fabs(y) < 1.0) {
        // C = sum_k (-y)^k/(2k+2)!, S = sum_k (-y)^k/(2k+3)!, Horner, k <= 13
        constexpr double c[14] = {
            1.0 / 2.0, 1.0 / 24.0, 1.0 / 720.0, 1.0 / 40320.0, 1.0 / 3628800.0,
            1.0 / 479001600.0, 1.0 / 87178291200.0, 1.0 / 20922789888000.0,
            1.0 / 6402373705728000.0, 1.0 / 2432902008176640000.0,
            1.0 / 1.1240007277776077e21, 1.0 / 6.204484017332394e23,
            1.0 / 4.0329146112660565e26, 1.0 / 3.0488834461171387e29};
        constexpr double s[14] = {
            1.0 / 6.0, 1.0 / 120.0, 1.0 / 5040.0, 1.0 / 362880.0, 1.0 / 39916800.0,
            1.0 / 6227020800.0, 1.0 / 1307674368000.0, 1.0 / 355687428096000.0,
            1.0 / 121645100408832000.0, 1.0 / 5.109094217170944e19,
            1.0 / 2.585201673888498e22, 1.0 / 1.5511210043330986e25,
            1.0 / 1.0888869450418352e28, 1.0 / 8.841761993739702e30};
        const double w = -y;
        double cc = c[13], ss = s[13];
#pragma unroll
        for (int k = 12; k >= 0; --k) {
            cc = fma(w, cc, c[k]);
            ss = fma(w, ss, s[k]);
        }
        C = cc;
        S = ss;
    } else if (y > 0.0) {
        const double sy = sqrt(y);
        C = (1.0 - cos(sy)) / y;
        S = (sy - sin(sy)) / (y * sy);
    } else {
        const double sy = sqrt(-y);
        C = (cosh(sy) - 1.0) / (-y);
        S = (sinh(sy) - sy) / ((-y) * sy);
    }
}

constexpr int kKeplerCap = 30;
constexpr double kKeplerTol = 1e-14;

// iterate to |dx| <= 1e-14 |x| (Laguerre n = 5, or Newton); returns 1 when
// converged, adds the iterations to *count
__device__ int kepler_iterate(double smu, double r0, double rv, double alpha, double dt,
                              int laguerre, double &x, int &count)
{
    const double b = 1.0 - r0 * alpha;
    // loop invariants, and the universal Kepler equation and its
    // derivatives as fused multiply-adds (one division per iteration)
    const double q = rv / smu, sdt = smu * dt;
    for (int it = 1; it <= kKeplerCap; ++it) {
        const double x2 = x * x;
        const double z = alpha * x2;
        double C, S;
        stumpff(z, C, S);
        const double zs = fma(-z, S, 1.0);   // 1 - z S
        const double F = fma(q * x2, C, fma(b * x2 * x, S, fma(r0, x, -sdt)));
        const double Fp = fma(q * x, zs, fma(b * x2, C, r0));
        double dx;
        if (laguerre) {
            const double Fpp = fma(q, fma(-z, C, 1.0), b * x * zs);
            const double nl = 5.0;
            const double rad =
                sqrt(fabs(fma((nl - 1.0) * (nl - 1.0) * Fp, Fp, -nl * (nl - 1.0) * F * Fpp)));
            dx = nl * F / (Fp + (Fp >= 0.0 ? rad : -rad));
        } else {
            dx = F / Fp;
        }
        x = x - dx;
        if (fabs(dx) <= kKeplerTol * fabs(x)) {
            count += it;
            return 1;
        }
    }
    count += kKeplerCap;
    return 0;
}

// ------------------------------------------------------------------------
// Learned starting value of the universal anomaly (not in the paper, which
// starts its iteration from a fixed value).  With r0 = |x0|, s = sign(dt),
// T = sqrt(mu)|dt| / r0^1.5 and alpha = 2/r0 - v0^2/mu, the features are
//   f0 = ln r0, f1 = s (x0.v0) / sqrt(mu r0), f2 = alpha r0, f3 = ln T
// (Kepler's equation is odd under (x, x0.v0, dt) -> (-x, -x0.v0, -dt), so
// the sign of the step rides on f1).  A 4-32-32-1 tanh network on the
// standardised features gives o; the start is
//   x_g = x_p exp(T (o s_y + m_y)),   x_p = sqrt(mu) dt / r0,
// i.e. the network predicts ln(x / x_p) / T, bounded for small steps.
// Weights (FP32): W1[32][4] at 0 (row = first-layer unit), b1 at 128,
// W2[32][32] at 160 (row = second-layer unit), b2 at 1184, W3 at 1216,
// b3 at 1248, then the scalers m_0..m_3, s_0..s_3, m_y, s_y at 1249.
// ------------------------------------------------------------------------
constexpr int kGW1 = 0, kGB1 = 128, kGW2 = 160, kGB2 = 1184, kGW3 = 1216, kGB3 = 1248;
constexpr int kGuessParams = 1249;
constexpr int kGuessWeights = kGuessParams + 10;

// tanh|a| = (1 - e^{-2|a|}) / (1 + e^{-2|a|}) with the hardware base-2
// exponential and reciprocal, sign restored; absolute error a few 1e-8.
__device__ __forceinline__ float tanh_fast(float a)
{
    const float t = __builtin_amdgcn_exp2f(-2.8853900817779268f * fabsf(a));  // 2/ln 2
    return copysignf((1.0f - t) * __builtin_amdgcn_rcpf(1.0f + t), a);
}

// features (FP32) and the scaled step T of one body (dt != 0)
__device__ __forceinline__ void guess_features(double smu, double r0, double rv, double alpha,
                                               double dt, float f[4], float &T)
{
    const float r0f = (float)r0;
    const float sr = sqrtf(r0f);
    T = (float)(smu * fabs(dt)) / (r0f * sr);
    f[0] = __logf(r0f);
    f[1] = (float)(dt > 0.0 ? rv : -rv) / ((float)smu * sr);
    f[2] = (float)(alpha * r0);
    f[3] = __logf(T);
}

// network output on standardised inputs (weights read uniformly by every
// lane, so they stream through the scalar cache)
__device__ __forceinline__ float guess_net(const float *__restrict__ w, const float in[4])
{
    float h1[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        float a = w[kGB1 + k];
#pragma unroll
        for (int c = 0; c < 4; ++c) a = fmaf(w[kGW1 + 4 * k + c], in[c], a);
        h1[k] = tanh_fast(a);
    }
    float o = w[kGB3];
#pragma unroll 2
    for (int k = 0; k < 32; ++k) {
        float a = w[kGB2 + k];
#pragma unroll
        for (int c = 0; c < 32; ++c) a = fmaf(w[kGW2 + 32 * k + c], h1[c], a);
        o = fmaf(w[kGW3 + k], tanh_fast(a), o);
    }
    return o;
}

__device__ __forceinline__ void guess_standardise(const float *__restrict__ w, const float f[4],
                                                  float in[4])
{
    const float *sc = w + kGuessParams;
#pragma unroll
    for (int c = 0; c < 4; ++c) in[c] = (f[c] - sc[c]) / sc[4 + c];
}

// learned start; not finite when the weights or the features are unusable
__device__ __forceinline__ double guess_start(const float *__restrict__ w, double smu, double r0,
                                              double rv, double alpha, double dt)
{
    float f[4], in[4], T;
    guess_features(smu, r0, rv, alpha, dt, f, T);
    guess_standardise(w, f, in);
    const float o = guess_net(w, in);
    const float *sc = w + kGuessParams;
    const float y = fmaf(o, sc[9], sc[8]);
    return (smu * dt / r0) * (double)__expf(T * y);
}

// A proposed start is used only when its ratio rho to the first-order guess
// lies where the root's must: dx/dt = sqrt(mu)/r along the orbit, so
// rho = r0 <1/r> is bounded by r0/r_max and r0/q (pericentre q = h^2/(mu(1+e)),
// apocentre r_max = h^2/(mu(1-e)) for a bound orbit, e^2 = 1 - alpha h^2/mu).
// Outside that range a start cannot be near the root, and far outside it
// the Stumpff functions of a huge argument can stop Newton at a wrong value.
__device__ __forceinline__ bool start_admissible(double mu, double r0, double rv, double alpha,
                                                 double rho)
{
    if (!(rho > 0.0) || !isfinite(rho)) return false;
    const double h2 = mu * r0 * (2.0 - alpha * r0) - rv * rv;  // |x0 x v0|^2
    if (!(h2 > 0.0)) return true;
    const double e2 = 1.0 - alpha * h2 / mu;
    const double e = e2 > 0.0 ? sqrt(e2) : 0.0;
    if (rho > r0 * mu * (1.0 + e) / h2) return false;
    if (alpha > 0.0 && e < 1.0 && rho < r0 * mu * (1.0 - e) / h2) return false;
    return true;
}

// ------------------------------------------------------------------------
// Root of Kepler's equation in universal variables.
//   mode 0: Laguerre (n = 5) from x = r0; on reaching the cap, once more
//           from the first-order guess sqrt(mu) dt / r0
//   mode 1: Newton from the first-order guess
//   mode 2: Newton from the learned start when it is admissible, else
//           from the first-order guess
// Modes 1 and 2 fall back to Laguerre from the first-order guess when Newton
// reaches the cap.  Returns 1 when converged; adds iterations to count and
// sets restart when the first start reached the cap.
// ------------------------------------------------------------------------
__device__ __forceinline__ int kepler_root(double smu, double r0, double rv, double alpha,
                                           double dt, int mode, const float *w, double &x,
                                           int &count, int &restart)
{
    const double guess = smu * dt / r0;
    int ok;
    restart = 0;
    if (mode == 0) {
        x = r0;
        ok = kepler_iterate(smu, r0, rv, alpha, dt, 1, x, count);
        if (!ok) {
            restart = 1;
            x = guess;
            ok = kepler_iterate(smu, r0, rv, alpha, dt, 1, x, count);
        }
    } else {
        x = guess;
        if (mode == 2) {
            const double g = guess_start(w, smu, r0, rv, alpha, dt);
            if (start_admissible(smu * smu, r0, rv, alpha, g / guess)) x = g;
        }
        ok = kepler_iterate(smu, r0, rv, alpha, dt, 0, x, count);
        if (!ok) {
            restart = 1;
            x = guess;
            ok = kepler_iterate(smu, r0, rv, alpha, dt, 1, x, count);
        }
    }
    return ok;
}

// Advance one body by dt about mu (Appendix A f and g functions); returns
// iterations, sets fail when every start reached the cap and restart when
// the first one did.
__device__ __forceinline__ int kepler_advance(double mu, int mode, const float *w, double dt,
                                              double &x, double &y, double &z, double &vx,
                                              double &vy, double &vz, int &fail, int &restart)
{
    fail = 0;
    restart = 0;
    if (dt == 0.0) return 0;
    const double r0 = sqrt(x * x + y * y + z * z);
    const double vv = vx * vx + vy * vy + vz * vz;
    const double rv = x * vx + y * vy + z * vz;
    const double smu = sqrt(mu);
    const double alpha = 2.0 / r0 - vv / mu;
    int count = 0;
    double xu;
    fail = !kepler_root(smu, r0, rv, alpha, dt, mode, w, xu, count, restart);
    const double zz = alpha * xu * xu;
    double C, S;
    stumpff(zz, C, S);
    const double f = 1.0 - xu * xu * C / r0;
    const double g = dt - xu * xu * xu * S / smu;
    const double nx = f * x + g * vx, ny = f * y + g * vy, nz = f * z + g * vz;
    const double r = sqrt(nx * nx + ny * ny + nz * nz);
    const double fd = smu * xu * (zz * S - 1.0) / (r * r0);
    const double gd = 1.0 - xu * xu * C / r;
    const double nvx = fd * x + gd * vx, nvy = fd * y + gd * vy, nvz = fd * z + gd * vz;
    x = nx;
    y = ny;
    z = nz;
    vx = nvx;
    vy = nvy;
    vz = nvz;
    return count;
}

}  // namespace qsym
