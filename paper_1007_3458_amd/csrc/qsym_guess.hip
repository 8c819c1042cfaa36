// qsym_guess.hip -- stand-alone Kepler solves and the training of the learned
// starting value of the Newton iteration (features, scalers, gradient of the
// loss by backpropagation, Adam) for MI355X / gfx950.
//
// The network and its features are defined in qsym_kepler.hpp.  Training
// samples are stored column-major in FP32: rows 0..3 of `feat` hold the
// features f0..f3 and row 4 the target y = ln(x / x_p) / T, each row `ld`
// floats apart.  The loss over n samples is (1/n) sum (o - (y - m_y)/s_y)^2.
#include "qsym.h"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>

#include "qsym_kepler.hpp"

using namespace qsym;

namespace {

constexpr int kGRow = 140;                  // floats per sample row in LDS (12 banks mod 32)
constexpr int kGPart = kGuessParams + 1;    // gradient sums + loss sum of one wave
constexpr int kGMaxParts = 4096;            // waves of one gradient launch
constexpr int kGMomBlocks = 1024;           // blocks of the moments reduction
constexpr int kGMaxEpochs = 4096;

struct State6 {
    const double *x, *y, *z, *vx, *vy, *vz;
};

__device__ __forceinline__ void body_terms(const State6 &s, long long i, double &r0, double &rv,
                                           double &vv)
{
    const double x = s.x[i], y = s.y[i], z = s.z[i], vx = s.vx[i], vy = s.vy[i], vz = s.vz[i];
    r0 = sqrt(x * x + y * y + z * z);
    vv = vx * vx + vy * vy + vz * vz;
    rv = x * vx + y * vy + z * vz;
}

// universal anomaly of each body for its own step (Appendix A solve);
// iters < 0 marks a solve that reached the cap from every start
__global__ __launch_bounds__(256) void k_kepler_solve(double mu, long long n, State6 s,
                                                      const double *__restrict__ dt, int mode,
                                                      const float *__restrict__ w,
                                                      double *__restrict__ xo, int *__restrict__ it)
{
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= n) return;
    const double h = dt[i];
    if (h == 0.0) {
        xo[i] = 0.0;
        if (it) it[i] = 0;
        return;
    }
    double r0, rv, vv;
    body_terms(s, i, r0, rv, vv);
    const double smu = sqrt(mu);
    const double alpha = 2.0 / r0 - vv / mu;
    int count = 0, restart;
    double x;
    const int ok = kepler_root(smu, r0, rv, alpha, h, mode, w, x, count, restart);
    xo[i] = x;
    if (it) it[i] = ok ? count : -count;
}

// learned start alone (0 for a zero step)
__global__ __launch_bounds__(256) void k_kepler_guess(double mu, long long n, State6 s,
                                                      const double *__restrict__ dt,
                                                      const float *__restrict__ w,
                                                      double *__restrict__ xo)
{
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= n) return;
    const double h = dt[i];
    if (h == 0.0) {
        xo[i] = 0.0;
        return;
    }
    double r0, rv, vv;
    body_terms(s, i, r0, rv, vv);
    const double smu = sqrt(mu);
    xo[i] = guess_start(w, smu, r0, rv, 2.0 / r0 - vv / mu, h);
}

// features (and targets when xr is given) of n solved bodies; *bad counts
// samples that cannot be used (zero step, non-finite feature or target)
__global__ __launch_bounds__(256) void k_guess_prepare(double mu, long long n, State6 s,
                                                       const double *__restrict__ dt,
                                                       const double *__restrict__ xr,
                                                       float *__restrict__ feat, long long ld,
                                                       unsigned long long *bad)
{
    const long long i = blockIdx.x * 256LL + threadIdx.x;
    if (i >= n) return;
    const double h = dt[i];
    double r0, rv, vv;
    body_terms(s, i, r0, rv, vv);
    const double smu = sqrt(mu);
    float f[4] = {NAN, NAN, NAN, NAN}, T = NAN;
    float y = 0.0f;
    bool ok = h != 0.0;
    if (ok) {
        guess_features(smu, r0, rv, 2.0 / r0 - vv / mu, h, f, T);
        if (xr) {
            const double Td = smu * fabs(h) / (r0 * sqrt(r0));
            y = (float)(log(xr[i] / (smu * h / r0)) / Td);
            ok = isfinite(y);
        }
        for (int c = 0; c < 4; ++c) ok = ok && isfinite(f[c]);
    }
    for (int c = 0; c < 4; ++c) feat[c * ld + i] = f[c];
    feat[4 * ld + i] = y;
    if (!ok) atomicAdd(bad, 1ULL);
}

// per-block FP64 sums of each of the 5 rows and of their squares
__global__ __launch_bounds__(256) void k_guess_moments(long long n, const float *__restrict__ feat,
                                                       long long ld, double *__restrict__ part)
{
    __shared__ double red[10][256];
    double a[10] = {};
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += 256LL * gridDim.x)
        for (int c = 0; c < 5; ++c) {
            const double v = feat[c * ld + i];
            a[c] += v;
            a[5 + c] += v * v;
        }
    for (int c = 0; c < 10; ++c) red[c][threadIdx.x] = a[c];
    __syncthreads();
    for (int st = 128; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st)
            for (int c = 0; c < 10; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x < 10) part[blockIdx.x * 10 + threadIdx.x] = red[threadIdx.x][0];
}

// means and population deviations into the scaler slots of w (a deviation
// of 0 or a non-finite one becomes 1)
__global__ void k_guess_scalers(const double *__restrict__ part, int nb, long long n,
                                float *__restrict__ w)
{
    const int c = threadIdx.x;
    if (c >= 5) return;
    double s = 0.0, q = 0.0;
    for (int b = 0; b < nb; ++b) {
        s += part[b * 10 + c];
        q += part[b * 10 + 5 + c];
    }
    const double mean = s / (double)n;
    double var = q / (double)n - mean * mean;
    double sd = var > 0.0 ? sqrt(var) : 0.0;
    if (!(sd > 0.0) || !isfinite(sd)) sd = 1.0;
    float *sc = w + kGuessParams;
    if (c < 4) {
        sc[c] = (float)mean;
        sc[4 + c] = (float)sd;
    } else {
        sc[8] = (float)mean;
        sc[9] = (float)sd;
    }
}

// Loss gradient sums over n samples, one wave per 64-sample tile (tiles
// strided over the grid).  Each lane runs one sample forward and back; the
// per-sample factors go to LDS and the wave then forms the sums over its
// tile: the 32 x 32 second-layer block as a 4 x 4 register tile per lane,
// the first layer, biases and output weights per first-layer/second-layer
// unit.  part[wave] receives sum e dO/dw (e = o - target; the factor 2/n is
// applied by the update) and sum e^2.
__global__ __launch_bounds__(64) void k_guess_grad(const float *__restrict__ w,
                                                   const float *__restrict__ feat, long long ld,
                                                   long long n, float *__restrict__ part)
{
    __shared__ __align__(16) float rows[64 * kGRow];
    const int l = threadIdx.x;
    const int k0 = 4 * (l >> 3), c0 = 4 * (l & 7), u = l & 31;
    const float *sc = w + kGuessParams;
    float acc[4][4] = {};
    float gb1 = 0.f, gb2 = 0.f, gw3 = 0.f, gb3 = 0.f, lsum = 0.f;
    float gw1[4] = {0.f, 0.f, 0.f, 0.f};
    for (long long tile = blockIdx.x; tile * 64 < n; tile += gridDim.x) {
        const long long s = tile * 64 + l;
        const bool valid = s < n;
        float in[4], yt = 0.f;
#pragma unroll
        for (int c = 0; c < 4; ++c) in[c] = valid ? (feat[c * ld + s] - sc[c]) / sc[4 + c] : 0.f;
        if (valid) yt = (feat[4 * ld + s] - sc[8]) / sc[9];
        float h1[32], h2[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            float a = w[kGB1 + k];
#pragma unroll
            for (int c = 0; c < 4; ++c) a = fmaf(w[kGW1 + 4 * k + c], in[c], a);
            h1[k] = tanh_fast(a);
        }
        float o = w[kGB3];
#pragma unroll
        for (int k = 0; k < 32; ++k) {
            float a = w[kGB2 + k];
#pragma unroll
            for (int c = 0; c < 32; ++c) a = fmaf(w[kGW2 + 32 * k + c], h1[c], a);
            h2[k] = tanh_fast(a);
            o = fmaf(w[kGW3 + k], h2[k], o);
        }
        const float e = valid ? o - yt : 0.f;
        float *row = rows + l * kGRow;
        float d2[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) d2[k] = e * w[kGW3 + k] * (1.f - h2[k] * h2[k]);
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            *(float4 *)(row + 4 * q) = make_float4(h1[4 * q], h1[4 * q + 1], h1[4 * q + 2], h1[4 * q + 3]);
            *(float4 *)(row + 32 + 4 * q) =
                make_float4(d2[4 * q], d2[4 * q + 1], d2[4 * q + 2], d2[4 * q + 3]);
            *(float4 *)(row + 96 + 4 * q) =
                make_float4(h2[4 * q], h2[4 * q + 1], h2[4 * q + 2], h2[4 * q + 3]);
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            float d1[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = 4 * q + j;
                float b = 0.f;
#pragma unroll
                for (int k = 0; k < 32; ++k) b = fmaf(w[kGW2 + 32 * k + c], d2[k], b);
                d1[j] = b * (1.f - h1[c] * h1[c]);
            }
            *(float4 *)(row + 64 + 4 * q) = make_float4(d1[0], d1[1], d1[2], d1[3]);
        }
        *(float4 *)(row + 128) = make_float4(in[0], in[1], in[2], in[3]);
        row[132] = e;
        row[133] = e * e;
        __syncthreads();
#pragma unroll 4
        for (int t = 0; t < 64; ++t) {
            const float *rt = rows + t * kGRow;
            const float4 dv = *(const float4 *)(rt + 32 + k0);
            const float4 hv = *(const float4 *)(rt + c0);
            const float dk[4] = {dv.x, dv.y, dv.z, dv.w};
            const float hc[4] = {hv.x, hv.y, hv.z, hv.w};
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(dk[i], hc[j], acc[i][j]);
            const float d1u = rt[64 + u], d2u = rt[32 + u], h2u = rt[96 + u];
            const float4 iv = *(const float4 *)(rt + 128);
            const float et = rt[132];
            gb1 += d1u;
            gb2 += d2u;
            gw3 = fmaf(et, h2u, gw3);
            gw1[0] = fmaf(d1u, iv.x, gw1[0]);
            gw1[1] = fmaf(d1u, iv.y, gw1[1]);
            gw1[2] = fmaf(d1u, iv.z, gw1[2]);
            gw1[3] = fmaf(d1u, iv.w, gw1[3]);
            gb3 += et;
            lsum += rt[133];
        }
        __syncthreads();
    }
    float *p = part + (long long)blockIdx.x * kGPart;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) p[kGW2 + 32 * (k0 + i) + c0 + j] = acc[i][j];
    if (l < 32) {
        p[kGB1 + l] = gb1;
        p[kGB2 + l] = gb2;
        p[kGW3 + l] = gw3;
        for (int j = 0; j < 4; ++j) p[kGW1 + 4 * l + j] = gw1[j];
    }
    if (l == 0) {
        p[kGB3] = gb3;
        p[kGuessParams] = lsum;
    }
}

// g_p = gscale * sum over nparts rows of gsrc (row stride `stride`), in a
// fixed order; optional gradient output, loss accumulation (thread 1249,
// only when loss_acc is given) and Adam update (Kingma & Ba, Alg. 1, with
// c1 = 1 - b1^t, c2 = 1 - b2^t)
struct UpdateArgs {
    const float *gsrc;
    int nparts;
    long long stride;
    double gscale, lscale;
    float *gout;
    double *loss_acc;
    float *w, *m, *v;
    double lr, b1, b2, eps, c1, c2;
    int adam;
};

__global__ __launch_bounds__(256) void k_guess_update(UpdateArgs a)
{
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p > kGuessParams) return;
    if (p == kGuessParams && !a.loss_acc) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int q = 0;
    for (; q + 4 <= a.nparts; q += 4) {
        s0 += (double)a.gsrc[(q + 0) * a.stride + p];
        s1 += (double)a.gsrc[(q + 1) * a.stride + p];
        s2 += (double)a.gsrc[(q + 2) * a.stride + p];
        s3 += (double)a.gsrc[(q + 3) * a.stride + p];
    }
    for (; q < a.nparts; ++q) s0 += (double)a.gsrc[q * a.stride + p];
    const double s = (s0 + s1) + (s2 + s3);
    if (p == kGuessParams) {
        *a.loss_acc += s * a.lscale;
        return;
    }
    const double g = s * a.gscale;
    if (a.gout) a.gout[p] = (float)g;
    if (a.adam) {
        const double mm = a.b1 * (double)a.m[p] + (1.0 - a.b1) * g;
        const double vv = a.b2 * (double)a.v[p] + (1.0 - a.b2) * g * g;
        a.m[p] = (float)mm;
        a.v[p] = (float)vv;
        const double mh = mm / a.c1, vh = vv / a.c2;
        a.w[p] = (float)((double)a.w[p] - a.lr * mh / (sqrt(vh) + a.eps));
    }
}

__global__ void k_zero_f64(double *p, int n)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

State6 state6(const double *st, long long n)
{
    return State6{st, st + n, st + 2 * n, st + 3 * n, st + 4 * n, st + 5 * n};
}

unsigned grid_of(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

struct qsym_guess_trainer {
    hipStream_t stream = nullptr;
    long long max_batch = 0;
    int max_parts = 0;
    char *mem = nullptr;
    float *part = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;
    double *loss = nullptr, *mom = nullptr, *curve = nullptr;
    unsigned long long *bad = nullptr;
    long long t = 0;
    std::string err;
};

namespace {

int tfail(qsym_guess_trainer *tr, int code, const std::string &msg)
{
    if (tr) tr->err = msg;
    return code;
}

#define TCHK(tr, call)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return tfail((tr), QSYM_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

int launch_grad(qsym_guess_trainer *tr, const float *w, const float *feat, long long ld,
                long long n, int &nparts)
{
    nparts = (int)std::min<long long>((n + 63) / 64, tr->max_parts);
    hipLaunchKernelGGL(k_guess_grad, dim3(nparts), dim3(64), 0, tr->stream, w, feat, ld, n,
                       tr->part);
    TCHK(tr, hipGetLastError());
    return QSYM_OK;
}

int launch_update(qsym_guess_trainer *tr, const UpdateArgs &a)
{
    hipLaunchKernelGGL(k_guess_update, dim3(grid_of(kGuessParams + 1, 256)), dim3(256), 0,
                       tr->stream, a);
    TCHK(tr, hipGetLastError());
    return QSYM_OK;
}

bool bad_state_args(long long n, const void *st, const void *dt) { return n < 0 || (n > 0 && (!st || !dt)); }

}  // namespace

// ------------------------------------------------------------------------
// Scratch of the allocation-free loss gradient (qsym_guess_grad_static):
// the per-wave partial sums of up to kStaticParts waves (64 samples each)
// and the loss accumulator, in one file-scope device array.  Every device
// the library runs on holds its own copy until the process ends; host code
// reaches it only through the address hipGetSymbolAddress gives on that
// device (the array's name is a host-side stand-in).
// ------------------------------------------------------------------------
constexpr int kStaticParts = QSYM_GUESS_STATIC_MAX / 64;
constexpr size_t kStaticPartBytes = (size_t)kStaticParts * kGPart * sizeof(float);
constexpr size_t kStaticScratchBytes = kStaticPartBytes + 256;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

void qsym_noctx_error(const char *msg);

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of this device's scratch, looked up once per device (with
// that device current) and kept
int static_scratch(void **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        qsym_noctx_error("guess_grad_static: no current HIP device");
        return QSYM_EHIP;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            qsym_noctx_error((std::string("guess_grad_static: hipGetSymbolAddress: ") +
                              hipGetErrorString(e)).c_str());
            return QSYM_EHIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return QSYM_OK;
}

}  // namespace

extern "C" {

int qsym_kepler_solve(double mu, int64_t n, const double *state, const double *dt, int32_t mode,
                      const float *weights, double *x_out, int32_t *iters, void *stream)
{
    if (!(mu > 0) || bad_state_args(n, state, dt) || mode < 0 || mode > 2 ||
        (mode == 2 && !weights) || (n > 0 && !x_out))
        return QSYM_EINVAL;
    if (n == 0) return QSYM_OK;
    hipLaunchKernelGGL(k_kepler_solve, dim3(grid_of(n, 256)), dim3(256), 0, (hipStream_t)stream, mu,
                       (long long)n, state6(state, n), dt, (int)mode, weights, x_out, (int *)iters);
    return hipGetLastError() == hipSuccess ? QSYM_OK : QSYM_EHIP;
}

int qsym_kepler_guess(double mu, int64_t n, const double *state, const double *dt,
                      const float *weights, double *x_out, void *stream)
{
    if (!(mu > 0) || bad_state_args(n, state, dt) || (n > 0 && (!weights || !x_out)))
        return QSYM_EINVAL;
    if (n == 0) return QSYM_OK;
    hipLaunchKernelGGL(k_kepler_guess, dim3(grid_of(n, 256)), dim3(256), 0, (hipStream_t)stream, mu,
                       (long long)n, state6(state, n), dt, weights, x_out);
    return hipGetLastError() == hipSuccess ? QSYM_OK : QSYM_EHIP;
}

int qsym_guess_trainer_create(int64_t max_batch, void *stream, qsym_guess_trainer **out)
{
    if (!out || max_batch < 1) return QSYM_EINVAL;
    *out = nullptr;
    auto *tr = new qsym_guess_trainer();
    tr->stream = (hipStream_t)stream;
    tr->max_batch = max_batch;
    tr->max_parts = (int)std::min<long long>((max_batch + 63) / 64, kGMaxParts);
    const size_t b_part = (size_t)tr->max_parts * kGPart * sizeof(float);
    const size_t b_vec = 1280 * sizeof(float);
    const size_t b_mom = (size_t)kGMomBlocks * 10 * sizeof(double);
    const size_t b_curve = kGMaxEpochs * sizeof(double);
    const size_t total = b_part + 3 * b_vec + 256 + b_mom + b_curve + 256;
    if (hipMalloc((void **)&tr->mem, total) != hipSuccess) {
        delete tr;
        return QSYM_ENOMEM;
    }
    char *p = tr->mem;
    tr->part = (float *)p; p += b_part;
    tr->g = (float *)p; p += b_vec;
    tr->m = (float *)p; p += b_vec;
    tr->v = (float *)p; p += b_vec;
    tr->loss = (double *)p; p += 256;
    tr->mom = (double *)p; p += b_mom;
    tr->curve = (double *)p; p += b_curve;
    tr->bad = (unsigned long long *)p;
    if (hipMemsetAsync(tr->mem, 0, total, tr->stream) != hipSuccess ||
        hipStreamSynchronize(tr->stream) != hipSuccess) {
        hipFree(tr->mem);
        delete tr;
        return QSYM_EHIP;
    }
    *out = tr;
    return QSYM_OK;
}

void qsym_guess_trainer_destroy(qsym_guess_trainer *tr)
{
    if (!tr) return;
    hipStreamSynchronize(tr->stream);
    hipFree(tr->mem);
    delete tr;
}

const char *qsym_guess_trainer_error(const qsym_guess_trainer *tr) { return tr ? tr->err.c_str() : ""; }

int qsym_guess_reset(qsym_guess_trainer *tr)
{
    if (!tr) return QSYM_EINVAL;
    TCHK(tr, hipMemsetAsync(tr->m, 0, 2 * 1280 * sizeof(float), tr->stream));
    tr->t = 0;
    return QSYM_OK;
}

int qsym_guess_prepare(qsym_guess_trainer *tr, double mu, int64_t n, const double *state,
                       const double *dt, const double *x_root, float *feat, int64_t ld)
{
    if (!tr) return QSYM_EINVAL;
    if (!(mu > 0) || bad_state_args(n, state, dt) || (n > 0 && !feat) || ld < n)
        return tfail(tr, QSYM_EINVAL, "guess_prepare: bad arguments (mu > 0, ld >= n)");
    if (n == 0) return QSYM_OK;
    TCHK(tr, hipMemsetAsync(tr->bad, 0, sizeof(unsigned long long), tr->stream));
    hipLaunchKernelGGL(k_guess_prepare, dim3(grid_of(n, 256)), dim3(256), 0, tr->stream, mu,
                       (long long)n, state6(state, n), dt, x_root, feat, (long long)ld, tr->bad);
    TCHK(tr, hipGetLastError());
    unsigned long long bad = 0;
    TCHK(tr, hipMemcpyAsync(&bad, tr->bad, sizeof bad, hipMemcpyDeviceToHost, tr->stream));
    TCHK(tr, hipStreamSynchronize(tr->stream));
    if (bad)
        return tfail(tr, QSYM_EINVAL,
                     std::to_string(bad) + " samples unusable (zero step or non-finite feature/target)");
    return QSYM_OK;
}

int qsym_guess_fit_scalers(qsym_guess_trainer *tr, const float *feat, int64_t ld, int64_t n,
                           float *weights)
{
    if (!tr) return QSYM_EINVAL;
    if (n < 1 || ld < n || !feat || !weights)
        return tfail(tr, QSYM_EINVAL, "guess_fit_scalers: need n >= 1, ld >= n");
    const int nb = (int)std::min<long long>((n + 255) / 256, kGMomBlocks);
    hipLaunchKernelGGL(k_guess_moments, dim3(nb), dim3(256), 0, tr->stream, (long long)n, feat,
                       (long long)ld, tr->mom);
    TCHK(tr, hipGetLastError());
    hipLaunchKernelGGL(k_guess_scalers, dim3(1), dim3(64), 0, tr->stream, tr->mom, nb,
                       (long long)n, weights);
    TCHK(tr, hipGetLastError());
    return QSYM_OK;
}

int qsym_guess_grad(qsym_guess_trainer *tr, const float *weights, const float *feat, int64_t ld,
                    int64_t n, float *grad, double *loss)
{
    if (!tr) return QSYM_EINVAL;
    if (n < 1 || n > tr->max_batch || ld < n || !weights || !feat || !grad)
        return tfail(tr, QSYM_EINVAL, "guess_grad: need 1 <= n <= max_batch, ld >= n");
    int nparts;
    if (int rc = launch_grad(tr, weights, feat, ld, n, nparts)) return rc;
    hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(256), 0, tr->stream, tr->loss, 1);
    UpdateArgs a{};
    a.gsrc = tr->part;
    a.nparts = nparts;
    a.stride = kGPart;
    a.gscale = 2.0 / (double)n;
    a.lscale = 1.0 / (double)n;
    a.gout = grad;
    a.loss_acc = tr->loss;
    if (int rc = launch_update(tr, a)) return rc;
    if (loss) {
        TCHK(tr, hipMemcpyAsync(loss, tr->loss, sizeof(double), hipMemcpyDeviceToHost, tr->stream));
        TCHK(tr, hipStreamSynchronize(tr->stream));
    }
    return QSYM_OK;
}

int qsym_guess_grad_static(const float *weights, const float *feat, int64_t ld, int64_t n,
                           float *grad, double *loss, void *stream)
{
    if (n < 1 || n > QSYM_GUESS_STATIC_MAX || ld < n || !weights || !feat || !grad) {
        qsym_noctx_error("guess_grad_static: need 1 <= n <= QSYM_GUESS_STATIC_MAX (16384), "
                         "ld >= n and non-null weights, feat, grad");
        return QSYM_EINVAL;
    }
    void *base = nullptr;
    if (int rc = static_scratch(&base)) return rc;
    float *part = (float *)base;
    double *lacc = (double *)((char *)base + kStaticPartBytes);
    hipStream_t st = (hipStream_t)stream;
    // the same launches as qsym_guess_grad: one wave per 64 samples (every
    // partial row is written whole), the loss accumulator cleared by a kernel
    const int nparts = (int)((n + 63) / 64);
    hipLaunchKernelGGL(k_guess_grad, dim3(nparts), dim3(64), 0, st, weights, feat, (long long)ld,
                       (long long)n, part);
    if (hipGetLastError() != hipSuccess) return QSYM_EHIP;
    hipLaunchKernelGGL(k_zero_f64, dim3(1), dim3(256), 0, st, lacc, 1);
    if (hipGetLastError() != hipSuccess) return QSYM_EHIP;
    UpdateArgs a{};
    a.gsrc = part;
    a.nparts = nparts;
    a.stride = kGPart;
    a.gscale = 2.0 / (double)n;
    a.lscale = 1.0 / (double)n;
    a.gout = grad;
    a.loss_acc = lacc;
    hipLaunchKernelGGL(k_guess_update, dim3(grid_of(kGuessParams + 1, 256)), dim3(256), 0, st, a);
    if (hipGetLastError() != hipSuccess) return QSYM_EHIP;
    if (loss) {
        if (hipMemcpyAsync(loss, lacc, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return QSYM_EHIP;
    }
    return QSYM_OK;
}

int qsym_guess_adam(qsym_guess_trainer *tr, float *weights, const float *grad, double lr,
                    double b1, double b2, double eps)
{
    if (!tr) return QSYM_EINVAL;
    if (!weights || !grad || !(lr >= 0) || !(b1 >= 0 && b1 < 1) || !(b2 >= 0 && b2 < 1) || !(eps >= 0))
        return tfail(tr, QSYM_EINVAL, "guess_adam: bad arguments");
    tr->t += 1;
    UpdateArgs a{};
    a.gsrc = grad;
    a.nparts = 1;
    a.stride = 0;
    a.gscale = 1.0;
    a.w = weights;
    a.m = tr->m;
    a.v = tr->v;
    a.lr = lr;
    a.b1 = b1;
    a.b2 = b2;
    a.eps = eps;
    a.c1 = 1.0 - std::pow(b1, (double)tr->t);
    a.c2 = 1.0 - std::pow(b2, (double)tr->t);
    a.adam = 1;
    return launch_update(tr, a);
}

int qsym_guess_train(qsym_guess_trainer *tr, float *weights, const float *feat, int64_t ld,
                     int64_t n, int64_t batch, int32_t epochs, double lr, double lr_final,
                     double *curve)
{
    if (!tr) return QSYM_EINVAL;
    if (!weights || !feat || n < 1 || ld < n || batch < 1 || batch > tr->max_batch || epochs < 1 ||
        epochs > kGMaxEpochs || !(lr > 0) || !(lr_final >= 0))
        return tfail(tr, QSYM_EINVAL,
                     "guess_train: need n >= 1, ld >= n, 1 <= batch <= max_batch, 1 <= epochs <= 4096, lr > 0");
    hipLaunchKernelGGL(k_zero_f64, dim3(grid_of(epochs, 256)), dim3(256), 0, tr->stream, tr->curve,
                       (int)epochs);
    TCHK(tr, hipGetLastError());
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    for (int e = 0; e < epochs; ++e) {
        // cosine decay from lr to lr_final over the epochs
        const double lre = lr_final + (lr - lr_final) * 0.5 * (1.0 + std::cos(kPi * e / epochs));
        for (long long b0 = 0; b0 < n; b0 += batch) {
            const long long nb = std::min<long long>(batch, n - b0);
            int nparts;
            if (int rc = launch_grad(tr, weights, feat + b0, ld, nb, nparts)) return rc;
            tr->t += 1;
            UpdateArgs a{};
            a.gsrc = tr->part;
            a.nparts = nparts;
            a.stride = kGPart;
            a.gscale = 2.0 / (double)nb;
            a.lscale = 1.0 / (double)n;
            a.loss_acc = tr->curve + e;
            a.w = weights;
            a.m = tr->m;
            a.v = tr->v;
            a.lr = lre;
            a.b1 = b1;
            a.b2 = b2;
            a.eps = eps;
            a.c1 = 1.0 - std::pow(b1, (double)tr->t);
            a.c2 = 1.0 - std::pow(b2, (double)tr->t);
            a.adam = 1;
            if (int rc = launch_update(tr, a)) return rc;
        }
    }
    if (curve)
        TCHK(tr, hipMemcpyAsync(curve, tr->curve, sizeof(double) * epochs, hipMemcpyDeviceToHost,
                                tr->stream));
    TCHK(tr, hipStreamSynchronize(tr->stream));
    return QSYM_OK;
}

}  // extern "C"
