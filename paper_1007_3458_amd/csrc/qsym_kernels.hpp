// qsym_kernels.hpp -- HIP kernels of the democratic-heliocentric hybrid step
// (Moore & Quillen, arXiv:1007.3458) for MI355X / gfx950.
//
// The translation unit is compiled with -ffp-contract=off: every fused
// multiply-add below is written out with fma() where it is wanted (pair
// sums), and the decision paths (per-body semi-major axis, fine encounter
// test, r_crit) use plain IEEE +, -, *, /, sqrt in a fixed order.
#pragma once
#include "qsym_common.hpp"
#include "qsym_kepler.hpp"

namespace qsym {

// ------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------
__device__ __forceinline__ double dnorm3(double a, double b, double c)
{
    return sqrt(a * a + b * b + c * c);
}

// Workgroup-wide sum of one double per thread in a fixed tree order (the
// same bits in every workgroup that reduces the same inputs).
template <int BS>
__device__ __forceinline__ double block_sum(double v, double *lds)
{
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
#pragma unroll
    for (int s = BS / 2; s > 0; s >>= 1) {
        if (t < s) lds[t] = lds[t] + lds[t + s];
        __syncthreads();
    }
    double r = lds[0];
    __syncthreads();
    return r;
}

// Momentum partials: one per Kepler-pass chunk of kChunkK = 64 bodies (a
// wave's worth), the sum over the chunk by an xor butterfly within the wave
// (both partners add the same two values, so every lane ends with the same
// bits).  A workgroup over a kChunk-body chunk writes the partials of its
// four quarters, wave w the one of quarter w: the same bits as a
// workgroup over that quarter alone.
__device__ __forceinline__ void wave_sum3(double v[3])
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double p0 = __shfl_xor(v[0], o, 64);
        const double p1 = __shfl_xor(v[1], o, 64);
        const double p2 = __shfl_xor(v[2], o, 64);
        v[0] += p0;
        v[1] += p1;
        v[2] += p2;
    }
}

// partials of the quarters of O(N) chunk bc (workgroup of kChunk threads,
// thread t holds body bc.y + t or zeros)
__device__ __forceinline__ void chunk_momentum(const Dev &d, int4 bc, double p[3])
{
    static_assert(kChunk == 4 * kChunkK && kChunkK == 64, "a chunk is four Kepler-pass chunks");
    wave_sum3(p);
    const int t = threadIdx.x, w = t >> 6;
    const int s = bc.x;
    const int q = d.sys_k0[s] + (bc.y - d.sys_off[s]) / kChunkK + w;
    if ((t & 63) == 0 && w * kChunkK < bc.z && q < d.sys_k0[s + 1])
        for (int k = 0; k < 3; ++k) d.pm[3 * q + k] = p[k];
}

// LDS written by some lanes of a wave and read by others: the wave's LDS
// operations complete in order, so a fence and a wave barrier suffice
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void latch(unsigned long long *ctr, unsigned long long bits)
{
    atomicOr(&ctr[C_STATUS], bits);
}

// Workgroup records for the load-balance figure (profiling only; rec is
// null otherwise): three words per workgroup of the launch (cleared before
// the launch): 1 + the compute unit (XCC id << 8 | SE, SH and CU ids of
// HW_ID) and the 100 MHz real-time clock at the workgroup's start, written
// by thread 0 when it starts, and its end, the latest of its waves' ends
// (an atomic maximum per wave, so no barrier is added).  A workgroup that
// returns early leaves its end at zero.
__device__ __forceinline__ void wg_start(unsigned long long *rec)
{
    if (rec == nullptr || threadIdx.x != 0) return;
    // s_getreg operands: register id | offset << 6 | (bits - 1) << 11
    const unsigned hw = __builtin_amdgcn_s_getreg(4 | (31 << 11));    // HW_ID
    const unsigned xcc = __builtin_amdgcn_s_getreg(20 | (3 << 11));   // XCC_ID[3:0]
    unsigned long long *r = rec + 3ull * blockIdx.x;
    r[0] = 1ull + ((xcc << 8) | ((hw >> 8) & 0xffu));
    r[1] = __builtin_amdgcn_s_memrealtime();
}

__device__ __forceinline__ void wg_finish(unsigned long long *rec)
{
    if (rec == nullptr || (threadIdx.x & 63) != 0) return;
    atomicMax(rec + 3ull * blockIdx.x + 2, (unsigned long long)__builtin_amdgcn_s_memrealtime());
}

// Momentum of system s summed from its chunk partials in a fixed order:
// each wave on its own (lane-strided sums, then a butterfly whose lane-0
// result every lane takes), so no workgroup barrier and the same bits in
// every wave of every workgroup.
__device__ void system_momentum(const Dev &d, int s, double P[3])
{
    const int c0 = d.sys_k0[s], c1 = d.sys_k0[s + 1];
    const int lane = threadIdx.x & 63;
    double a[3] = {0.0, 0.0, 0.0};
    // four partials requested before any is added (the same order), so
    // their loads overlap
    int c = c0 + lane;
    for (; c + 192 < c1; c += 256) {
        double v[4][3];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < 3; ++k) v[u][k] = d.pm[3 * (c + 64 * u) + k];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int k = 0; k < 3; ++k) a[k] += v[u][k];
    }
    for (; c < c1; c += 64) {
        a[0] += d.pm[3 * c];
        a[1] += d.pm[3 * c + 1];
        a[2] += d.pm[3 * c + 2];
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        a[0] += __shfl_xor(a[0], o, 64);
        a[1] += __shfl_xor(a[1], o, 64);
        a[2] += __shfl_xor(a[2], o, 64);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const long long b = __double_as_longlong(a[k]);
        const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
        const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
        P[k] = __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    }
}

// ------------------------------------------------------------------------
// E_Dft (Sec. 2): per-chunk momentum partials sum_i m_i v_i
// ------------------------------------------------------------------------
__global__ __launch_bounds__(kChunk) void k_momentum(Dev d)
{
    const int4 bc = d.bchunk[blockIdx.x];
    const int t = threadIdx.x;
    const int i = bc.y + t;
    double p[3] = {0.0, 0.0, 0.0};
    if (t < bc.z) {
        const double mi = d.m[i];
        p[0] = mi * d.vx[i];
        p[1] = mi * d.vy[i];
        p[2] = mi * d.vz[i];
    }
    chunk_momentum(d, bc, p);
}

// ------------------------------------------------------------------------
// E_Dft(dt): Q_i += dt * P / m0 (Sec. 2, H_Dft), optionally followed by the
// per-body quantities of the encounter search (Sec. 2.4) at the drifted
// state: a_i (osculating semi-major axis, r_i when unbound), the Hill-radius
// term ch_i = h_i (mutual) or h_i a_i (sum) and the escape speed
// cv_i = sqrt(2 mu / r_i).  The first workgroup resets the per-step
// counters.
// ------------------------------------------------------------------------
struct DriftArgs {
    Dev d;
    double dt, G, tau_crude, aE, cs;
    int prepass, hill_mode, reset, count_step;
    int sweep_stats;   // grid crude sweep next: per-chunk sums of (a, h or h a, ve), clear its table
    int backup;        // first drift of a hybrid step: keep the state at the step's start
    int restore;       // last drift of a hybrid step: put it back when the step could not be done
    int fused;         // the previous step's last drift (dt, counted) before this step's first
};

__global__ __launch_bounds__(kChunk) void k_drift(DriftArgs a)
{
    __shared__ double lds[kChunk];
    const Dev &d = a.d;
    const int4 bc = d.bchunk[blockIdx.x];
    const int s = bc.x;
    // the status is only raised by other kernels, so every workgroup reads
    // the same word here
    const bool frozen = (a.backup || a.restore) && (d.ctr[C_STATUS] & S_FREEZE);
    const long long S = (long long)(d.y - d.x);   // stride of the state arrays
    if (a.restore && frozen) {
        // the step could not hold its encounter pairs: the state goes back to
        // the step's start, with its momentum partials (as k_momentum)
        const int t = threadIdx.x, i = bc.y + t;
        double p[3] = {0.0, 0.0, 0.0};
        if (t < bc.z) {
            const double *bk = d.bk;
            d.x[i] = bk[i];
            d.y[i] = bk[S + i];
            d.z[i] = bk[2 * S + i];
            d.vx[i] = bk[3 * S + i];
            d.vy[i] = bk[4 * S + i];
            d.vz[i] = bk[5 * S + i];
            const double mi = d.m[i];
            p[0] = mi * d.vx[i];
            p[1] = mi * d.vy[i];
            p[2] = mi * d.vz[i];
        }
        chunk_momentum(d, bc, p);
        if (blockIdx.x == 0 && t == 0) d.ctr[C_OVERFLOW] += 1;
        return;
    }
    double P[3];
    system_momentum(d, s, P);
    if (a.reset && blockIdx.x == 0 && threadIdx.x == 0) {
        d.ctr[C_CAND] = 0;
        d.ctr[C_ENC] = 0;
        d.ctr[C_NSETS] = 0;
        d.ctr[C_MAXSET] = 0;
        d.ctr[C_SUB] = 0;
        d.ctr[C_NU] = 0;
        d.ctr[C_NSMALL] = 0;
        d.ctr[C_NBIG] = 0;
        d.ctr[C_NGRID] = 0;
        d.ctr[C_NLARGE] = 0;
        d.gbar[0] = 0u;
        d.gbar[1] = 0u;
        d.gbar[2] = 0u;
    }
    if (a.count_step && blockIdx.x == 0 && threadIdx.x == 0) d.ctr[C_STEPS] += 1;
    if (a.reset && threadIdx.x == 0 && (int)blockIdx.x == d.sys_c0[s]) d.sys_ecnt[s] = 0;
    const int t = threadIdx.x;
    const bool ok = t < bc.z;
    const int i = bc.y + t;
    const double m0 = d.sys_m0[s];
    double sw[3] = {0.0, 0.0, 0.0};
    if (ok) {
        double x = d.x[i], y = d.y[i], z = d.z[i];
        if (a.fused) {
            // the previous step's last E_Dft(dt): the same addition a launch
            // of its own would make (a drift leaves P unchanged, so the same
            // P serves both)
            x = x + a.dt * (P[0] / m0);
            y = y + a.dt * (P[1] / m0);
            z = z + a.dt * (P[2] / m0);
        }
        if (a.backup && !frozen) {
            // the state at this step's start
            d.bk[i] = x;
            d.bk[S + i] = y;
            d.bk[2 * S + i] = z;
            d.bk[3 * S + i] = d.vx[i];
            d.bk[4 * S + i] = d.vy[i];
            d.bk[5 * S + i] = d.vz[i];
        }
        x = x + a.dt * (P[0] / m0);
        y = y + a.dt * (P[1] / m0);
        z = z + a.dt * (P[2] / m0);
        d.x[i] = x;
        d.y[i] = y;
        d.z[i] = z;
        if (a.prepass) {
            const double mu = a.G * m0;
            const double vx = d.vx[i], vy = d.vy[i], vz = d.vz[i];
            const double r = sqrt(x * x + y * y + z * z);
            const double inva = 2.0 / r - (vx * vx + vy * vy + vz * vz) / mu;
            const double A = (inva > 0.0) ? 1.0 / inva : r;
            const double ve = sqrt(2.0 * mu / r);
            const double ch = (a.hill_mode == 0) ? d.h[i] : d.h[i] * A;
            d.A[i] = A;
            d.ch[i] = ch;
            d.cv[i] = ve;
            sw[0] = A;
            sw[1] = ch;
            sw[2] = ve;
        }
    }
    if (a.sweep_stats) {
        // the grid sweep's statistics: chunk sums in a fixed order
        for (int k = 0; k < 3; ++k) {
            const double v = block_sum<kChunk>(sw[k], lds);
            if (t == 0) d.sw_part[3 * blockIdx.x + k] = v;
        }
        for (int k = blockIdx.x * kChunk + t; k < d.sw_nb; k += gridDim.x * kChunk) d.sw_cnt[k] = 0;
    }
}

// ------------------------------------------------------------------------
// E_Int (Sec. 2, H_Int): all-pairs kick, i in registers, j tiles through
// LDS; the crude encounter sweep of Sec. 2.4 is fused into the j loop of
// the first kick for the unordered pairs i < j.  Each workgroup writes the
// partial acceleration of its i-bodies over its j-chunk; the partials are
// reduced in chunk order by k_apply_* (deterministic).
//
// FP64 pair term (PREC 0): r^-3 from the hardware reciprocal square root
// (about 24 correct bits) refined by the binomial series of (1-e)^(-3/2)
// with e = 1 - r^2 y0^2:  m r^-3 = m y0^3 (1 + e (3/2 + 15/8 e)), which is
// exact to FP64 rounding since |e| < 2^-22.  r^2 is floored at 1e-200 so a
// body's own pair (and coincident bodies) contributes exactly zero.
//
// FP32 pair term (PREC 1): see pair32.
//
// Crude sweep: per j-tile the maxima of (h or h a, a, ve) bound the exact
// threshold of every pair of the tile from above, so the pair loop only
// compares r^2 with one per-i bound (one compare per pair); the few pairs
// under it take the exact test of the definition.
// ------------------------------------------------------------------------
struct KickArgs {
    Dev d;
    const KickItem *items;   // work items of this kick's launch shape
    double G;
    long long cap;     // candidate capacity
    int nitems;
    int remap;         // XCD-aware workgroup order
    int hill_mode;     // crude test form
    double aE, cs, tau_abs;
    double r2seed;     // 1e-200, passed at run time so it stays a register operand
    double c158, c32;  // 15/8 and 3/2 of the r^-3 correction, likewise register operands
    unsigned long long *rec = nullptr;   // workgroup records (profiling), else null
};

// workgroup b of a grid of g (multiple of 8) runs on XCD b % 8; give each
// XCD a contiguous run of items so that its L2 sees few j-chunks
__device__ __forceinline__ int xcd_item(int b, int g)
{
    const int per = g >> 3;
    return (b & 7) * per + (b >> 3);
}

// a double moved between lanes by the DPP pattern CTRL (both halves, every
// row and bank enabled)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double readlane_f64(double v, int lane)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// maximum over the wave (fmax: NaN only where every lane has NaN): the row
// maxima through four DPP levels (quad_perm [1,0,3,2] and [2,3,0,1],
// row_half_mirror, row_mirror), then the four rows read into scalar
// registers; every lane gets the same value
__device__ __forceinline__ double wave_max(double v)
{
    v = fmax(v, dpp_f64<0xB1>(v));
    v = fmax(v, dpp_f64<0x4E>(v));
    v = fmax(v, dpp_f64<0x141>(v));
    v = fmax(v, dpp_f64<0x140>(v));
    return fmax(fmax(readlane_f64(v, 0), readlane_f64(v, 16)),
                fmax(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// Crude sweep, exact form (Sec. 2.4 reading): evaluated only for the pairs
// that passed the per-tile bound; same operands and operation order as the
// definition:  |Q_j-Q_i|^2 < (c_s (R_up + |tau| (ve_i + ve_j)))^2.
// X, Y, Z: the positions the sweep runs at (the kick's, or their snapshot).
__device__ __forceinline__ bool crude_pass(const Dev &d, const double *X, const double *Y,
                                           const double *Z, int hill_mode, double aE, double cs,
                                           double tau_abs, int i, int j)
{
    const double dx = X[j] - X[i];
    const double dy = Y[j] - Y[i];
    const double dz = Z[j] - Z[i];
    const double r2 = dx * dx + dy * dy + dz * dz;
    double Rup;
    if (hill_mode == 0)
        Rup = aE * (d.h[i] + d.h[j]) * (d.A[i] + d.A[j]) / 2.0;
    else
        Rup = aE * (d.h[i] * d.A[i] + d.h[j] * d.A[j]);
    const double lim = cs * (Rup + tau_abs * (d.cv[i] + d.cv[j]));
    return r2 < lim * lim;
}

__device__ __forceinline__ void crude_exact(const KickArgs &ka, int i, int j)
{
    const Dev &d = ka.d;
    if (j <= i) return;
    if (crude_pass(d, d.x, d.y, d.z, ka.hill_mode, ka.aE, ka.cs, ka.tau_abs, i, j)) {
        const unsigned long long slot = atomicAdd(&d.ctr[C_CAND], 1ull);
        if ((long long)slot < ka.cap) d.cand[slot] = make_int2(i, j);
    }
}

// FP64 pair term (see the header comment of the kick).  r^2 carries a
// 1e-200 seed (so the own pair gives 0 * finite = 0 and r^2 >= 1e-184 is
// unchanged); the correction is the factor w = 1 + e (3/2 + 15/8 e), so the
// term costs 17 VALU instructions: 3 add, 9 fma, 4 mul, 1 rsq.
__device__ __forceinline__ void pair64(const double4 &pj, double xi, double yi, double zi,
                                       double seed, double c158, double c32, double &ax,
                                       double &ay, double &az, double &r2)
{
    const double dx = pj.x - xi, dy = pj.y - yi, dz = pj.z - zi;
    r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, seed)));
    const double y0 = __builtin_amdgcn_rsq(r2);
    const double y2 = y0 * y0;
    const double e = fma(-r2, y2, 1.0);
    // r^-3 = y0^3 (1 - e)^(-3/2) = y0^3 (1 + 3/2 e + 15/8 e^2 + O(e^3)), |e| ~ 1e-7
    const double w = fma(e, fma(e, c158, c32), 1.0);
    const double ms = (y2 * y0) * (pj.w * w);
    ax = fma(ms, dx, ax);
    ay = fma(ms, dy, ay);
    az = fma(ms, dz, az);
}

// FP32 pair term on an FP64 separation: the differences and r^2 stay FP64
// (an FP64 add or fma costs the same issue slot as an FP32 one on this
// chip, and r^2 in FP64 needs one conversion instead of three), only r^-3
// is formed in FP32 from the hardware rsq (no refinement); it is widened
// once and multiplied by the FP64 G m (the product of a float and a
// double loses nothing a float product would keep, and saves the mass's
// narrowing), and the sum is accumulated in FP64.  The 1e-24 seed keeps
// the own pair finite (r^-3 = 1e36 < FLT_MAX) and changes no physical pair.
__device__ __forceinline__ void pair32(const double4 &pj, double xi, double yi, double zi,
                                       double &ax, double &ay, double &az, double &r2)
{
    const double dx = pj.x - xi, dy = pj.y - yi, dz = pj.z - zi;
    r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, 1e-24)));
    const float y = __builtin_amdgcn_rsqf((float)r2);
    const double ms = pj.w * (double)(y * y * y);
    ax = fma(ms, dx, ax);
    ay = fma(ms, dy, ay);
    az = fma(ms, dz, az);
}

// padding of a partial j-tile: far away (r^2 ~ 3e36, finite in FP32) and massless, so it
// adds nothing and never passes the crude bound
constexpr double kFar = 1e18;

// pairs under the tile bound are queued in LDS (lane, i slot, j offset)
// and given the exact test after the tile, so the pair loop has no call
constexpr int kCrudeQ = 512;

template <int BS, int IPL, int MODE>
__device__ __forceinline__ void crude_drain(const KickArgs &ka, int i0, int ni, int jt, int jend,
                                            const int *ii, unsigned *qbuf, unsigned *qn)
{
    const unsigned n = *qn;
    const int tid = threadIdx.x;
    if (n <= (unsigned)kCrudeQ) {
        for (unsigned e = tid; e < n; e += BS) {
            const unsigned v = qbuf[e];
            const int lt = (int)(v >> 16), u = (int)((v >> 8) & 0xffu), jj = (int)(v & 0xffu);
            if (lt + u * BS < ni) crude_exact(ka, i0 + lt + u * BS, jt + jj);
        }
    } else {
        // queue overflow (a dense tile): exact test of every pair of the tile
        const int je = min(jt + BS, jend);
#pragma unroll
        for (int u = 0; u < IPL; ++u)
            if (tid + u * BS < ni)
                for (int j = jt; j < je; ++j) crude_exact(ka, ii[u], j);
    }
}

template <int BS, int IPL, int MODE, int PREC>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(1, 4))) void k_kick(KickArgs ka)
{
    const Dev &d = ka.d;
    const int tid = threadIdx.x;
    int b = blockIdx.x;
    if (ka.remap) b = xcd_item(b, gridDim.x);
    if (b >= ka.nitems) return;
    if (d.ctr[C_STATUS] & S_FREEZE) return;   // a step left undone: nothing to compute
    const KickItem it = ka.items[b];
    constexpr int NW = BS / 64;

    __shared__ double4 sj[BS];
    __shared__ double smax[3][NW];
    __shared__ unsigned qbuf[MODE ? kCrudeQ : 1];
    __shared__ unsigned qn;

    double xi[IPL], yi[IPL], zi[IPL];
    double ax[IPL], ay[IPL], az[IPL];
    double hi[IPL], Ai[IPL], vi[IPL];
    int ii[IPL];
#pragma unroll
    for (int u = 0; u < IPL; ++u) {
        const int i = it.i0 + tid + u * BS;
        const bool ok = (tid + u * BS) < it.ni;
        xi[u] = ok ? d.x[i] : 0.0;
        yi[u] = ok ? d.y[i] : 0.0;
        zi[u] = ok ? d.z[i] : 0.0;
        ax[u] = ay[u] = az[u] = 0.0;
        if (MODE) {
            hi[u] = ok ? d.ch[i] : 0.0;
            Ai[u] = ok ? d.A[i] : 0.0;
            vi[u] = ok ? d.cv[i] : 0.0;
        }
        ii[u] = ok ? i : 0x7fffffff;
    }
    if (MODE && tid == 0) qn = 0u;
    const int jend = it.j0 + it.nj;
    const double G = ka.G;
    const double seed = ka.r2seed, c158 = ka.c158, c32 = ka.c32;
    int qtile = -1;   // tile whose queue is pending
    for (int jt = it.j0; jt < jend; jt += BS) {
        const int j = jt + tid;
        const bool okj = j < jend;
        __syncthreads();
        if constexpr (MODE != 0) {
            if (qtile >= 0) {
                if (qn) crude_drain<BS, IPL, MODE>(ka, it.i0, it.ni, qtile, it.j0 + it.nj, ii, qbuf, &qn);
                __syncthreads();
                if (tid == 0) qn = 0u;
                qtile = -1;
            }
        }
        sj[tid] = okj ? make_double4(d.x[j], d.y[j], d.z[j], G * d.m[j])
                      : make_double4(kFar, kFar, kFar, 0.0);
        const int last_j = min(jt + BS, jend) - 1;
        const bool pred = MODE && (last_j > it.i0);
        // j-slots of this tile, rounded up to the unroll factor (the
        // padding slots are massless and far away)
        const int ntj = (last_j - jt + 1 + 3) & ~3;
        if (MODE && pred) {
            // tile maxima of the crude-sweep terms (all non-negative)
            double t0 = okj ? d.ch[j] : 0.0, t1 = okj ? d.A[j] : 0.0, t2 = okj ? d.cv[j] : 0.0;
            t0 = wave_max(t0);
            t1 = wave_max(t1);
            t2 = wave_max(t2);
            if ((tid & 63) == 0) {
                smax[0][tid >> 6] = t0;
                smax[1][tid >> 6] = t1;
                smax[2][tid >> 6] = t2;
            }
        }
        __syncthreads();
        if constexpr (MODE != 0) {
            if (pred) {
                double HT = smax[0][0], AT = smax[1][0], VT = smax[2][0];
#pragma unroll
                for (int w = 1; w < NW; ++w) {
                    HT = fmax(HT, smax[0][w]);
                    AT = fmax(AT, smax[1][w]);
                    VT = fmax(VT, smax[2][w]);
                }
                // per-(i, tile) upper bound of the crude threshold: every
                // operation is monotone in the j-terms, so th >= the exact
                // limit of every j in the tile; the factor covers the
                // different rounding of r^2 in the pair loop
                double th2[IPL];
#pragma unroll
                for (int u = 0; u < IPL; ++u) {
                    double Rb;
                    if (MODE == 1)
                        Rb = ka.aE * (hi[u] + HT) * (Ai[u] + AT) / 2.0;
                    else
                        Rb = ka.aE * (hi[u] + HT);
                    const double th = ka.cs * (Rb + ka.tau_abs * (vi[u] + VT));
                    th2[u] = th * th * 1.000000000001;
                }
#pragma unroll 4
                for (int jj = 0; jj < ntj; ++jj) {
                    const double4 pj = sj[jj];
#pragma unroll
                    for (int u = 0; u < IPL; ++u) {
                        double r2;
                        if constexpr (PREC == 0)
                            pair64(pj, xi[u], yi[u], zi[u], seed, c158, c32, ax[u], ay[u], az[u], r2);
                        else
                            pair32(pj, xi[u], yi[u], zi[u], ax[u], ay[u], az[u], r2);
                        if (r2 < th2[u]) {
                            const unsigned k = atomicAdd(&qn, 1u);
                            if (k < (unsigned)kCrudeQ)
                                qbuf[k] = ((unsigned)tid << 16) | ((unsigned)u << 8) | (unsigned)jj;
                        }
                    }
                }
                qtile = jt;
                continue;
            }
        }
        if constexpr (PREC == 0) {
#pragma unroll 4
            for (int jj = 0; jj < ntj; ++jj) {
                const double4 pj = sj[jj];
#pragma unroll
                for (int u = 0; u < IPL; ++u) {
                    double r2;
                    pair64(pj, xi[u], yi[u], zi[u], seed, c158, c32, ax[u], ay[u], az[u], r2);
                }
            }
        } else {
#pragma unroll 4
            for (int jj = 0; jj < ntj; ++jj) {
                const double4 pj = sj[jj];
#pragma unroll
                for (int u = 0; u < IPL; ++u) {
                    double r2;
                    pair32(pj, xi[u], yi[u], zi[u], ax[u], ay[u], az[u], r2);
                }
            }
        }
    }
    if constexpr (MODE != 0) {
        __syncthreads();
        if (qtile >= 0 && qn)
            crude_drain<BS, IPL, MODE>(ka, it.i0, it.ni, qtile, it.j0 + it.nj, ii, qbuf, &qn);
    }
    const int s = it.sys;
    const int ns = d.sys_off[s + 1] - d.sys_off[s];
    const long long base = d.sys_poff[s] + (long long)it.chunk * 3 * ns;
#pragma unroll
    for (int u = 0; u < IPL; ++u) {
        if (tid + u * BS < it.ni) {
            const int il = it.i0 + tid + u * BS - d.sys_off[s];
            d.acc[base + il] = ax[u];
            d.acc[base + ns + il] = ay[u];
            d.acc[base + 2 * ns + il] = az[u];
        }
    }
}

// ------------------------------------------------------------------------
// Symmetric kick (Newton's third law): each unordered pair once.  A work
// item is a chunk of j-bodies [j0, j0 + nj) and a range of i-blocks
// [i0, i0 + ni) (blocks of BS * IPL bodies, IPL = 1 or 2 per thread).  An
// i-block starting at ib meets only the part j >= ib of the chunk.  Each
// wave owns 64 IPL i (IPL per lane, in groups of 64) and meets the j-tile in
// sub-tiles of 64: in step k lane l pairs its i with sub-tile entry
// (l + k) mod 64, so the 64 lanes touch 64 different j and the reaction on
// each j travels with it in three registers that move one lane down after
// every step (both i of a lane add to it); after 64 steps
// every lane holds the whole reaction on "its" j again.  For each lane
// group a sub-tile that starts before the group's i is skipped, the one
// that starts at it keeps only the pairs l < (l + k) mod 64, so every pair
// i < j of the system is met exactly once over all items.  The force on i
// goes to its i-side slot
// `chunk` (as written by k_kick); the reactions of the waves are added in
// wave order and then to the item's own j-side slot `slot` (the item's
// first i-block stores, later ones add).  Each slot entry is only ever
// touched by one thread of one item: no atomics, a fixed order.  Per pair:
// one pair term for both forces (21 VALU instructions, one rsq) and 6/IPL
// instructions of lane rotation (DPP), against 2 x 17 for the two ordered
// pairs of k_kick.  The sub-tile sits twice in a row in LDS, so
// entry l + k needs no wrap-around and every read takes its offset from
// the instruction.
// ------------------------------------------------------------------------

// lane l receives v of lane (l + 1) mod 64: DPP wave_rol:1 (control 0x134;
// its lane layout checked on the device: lane l reads lane l + 1, lane 63
// lane 0)
__device__ __forceinline__ double lane_rotate1(double v) { return dpp_f64<0x134>(v); }

// FP64 pair of the symmetric kick: force on i into (ax, ay, az), reaction
// on j into (fx, fy, fz); keep = false drops the pair
__device__ __forceinline__ void pair_sym64(double xj, double yj, double zj, double gmj, double xi,
                                           double yi, double zi, double gmi, double seed,
                                           double c158, double c32, bool keep, double &ax,
                                           double &ay, double &az, double &fx, double &fy,
                                           double &fz, double &r2)
{
    const double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, seed)));
    const double y0 = __builtin_amdgcn_rsq(r2);
    const double y2 = y0 * y0;
    const double e = fma(-r2, y2, 1.0);
    const double w = fma(e, fma(e, c158, c32), 1.0);
    double r3 = (y2 * y0) * w;
    if (!keep) r3 = 0.0;
    const double msj = gmj * r3, msi = gmi * r3;
    ax = fma(msj, dx, ax);
    ay = fma(msj, dy, ay);
    az = fma(msj, dz, az);
    fx = fma(-msi, dx, fx);
    fy = fma(-msi, dy, fy);
    fz = fma(-msi, dz, fz);
}

// FP32 form: r^-3 from the FP32 rsq on the FP64 r^2, widened once and
// multiplied by the FP64 G m of either body (as pair32)
__device__ __forceinline__ void pair_sym32(double xj, double yj, double zj, double gmj, double xi,
                                           double yi, double zi, double gmi, bool keep, double &ax,
                                           double &ay, double &az, double &fx, double &fy,
                                           double &fz, double &r2)
{
    const double dx = xj - xi, dy = yj - yi, dz = zj - zi;
    r2 = fma(dz, dz, fma(dy, dy, fma(dx, dx, 1e-24)));
    const float y = __builtin_amdgcn_rsqf((float)r2);
    const double r3 = keep ? (double)(y * y * y) : 0.0;
    const double msj = gmj * r3, msi = gmi * r3;
    ax = fma(msj, dx, ax);
    ay = fma(msj, dy, ay);
    az = fma(msj, dz, az);
    fx = fma(-msi, dx, fx);
    fy = fma(-msi, dy, fy);
    fz = fma(-msi, dz, fz);
}

// How one lane group of 64 i meets a sub-tile of 64 j: all pairs (the
// sub-tile lies past the group), the pairs l < (l + k) mod 64 (the sub-tile
// is the group itself), or none (the sub-tile lies before it).
enum { SYM_FULL = 0, SYM_DIAG = 1, SYM_SKIP = 2 };

// 64 rotation steps of one wave over one sub-tile; lane group u (i_u =
// u-th i of the lane) meets it as M0 (u = 0) / M1 (u = 1).  sxy, szm
// point at the doubled sub-tile ((x, y) and (z, G m) rows of 128).
// Crude-sweep hits are queued as body pairs (ib + lt, jsub + j offset) in
// qi, qj.
template <int MODE, int PREC, int IPL, int M0, int M1>
__device__ __forceinline__ void sym_subtile(const double2 *sxy, const double2 *szm, int lane,
                                            const double *xi, const double *yi,
                                            const double *zi, const double *gmi,
                                            const double *th2, const int *lt,
                                            double seed, double c158, double c32, double *ax,
                                            double *ay, double *az, double &fx, double &fy,
                                            double &fz, int *qi, int *qj, unsigned *qn, int ib,
                                            int jsub)
{
    // the crude test's queue pushes split the loop body into blocks, and a
    // deep unroll then keeps too many values live: unroll less with it
    constexpr int UNR = MODE != 0 ? 2 : 8;
    // with the crude test each rotation step is a block of its own (its
    // branch), so the crude kicks read the next step's j while this one
    // runs (a scheduling barrier keeps the reads there; entry lane + 64
    // still lies in the doubled sub-tile); the plain kick's unrolled body
    // overlaps them by itself
    double2 nxy = sxy[lane], nzm = szm[lane];
#pragma unroll UNR
    for (int k = 0; k < 64; ++k) {
        double xj, yj, zj, gmj;
        if constexpr (MODE != 0) {
            xj = nxy.x; yj = nxy.y; zj = nzm.x; gmj = nzm.y;
            nxy = sxy[lane + k + 1];
            nzm = szm[lane + k + 1];
            __builtin_amdgcn_sched_barrier(0);
        } else {
            const double2 pxy = sxy[lane + k], pzm = szm[lane + k];
            xj = pxy.x; yj = pxy.y; zj = pzm.x; gmj = pzm.y;
        }
        bool hit[IPL];
#pragma unroll
        for (int u = 0; u < IPL; ++u) {
            const int M = u == 0 ? M0 : M1;
            hit[u] = false;
            if (M == SYM_SKIP) continue;
            const bool keep = M == SYM_DIAG ? (k > 0 && lane + k < 64) : true;
            double r2;
            if constexpr (PREC == 0)
                pair_sym64(xj, yj, zj, gmj, xi[u], yi[u], zi[u], gmi[u], seed, c158, c32, keep,
                           ax[u], ay[u], az[u], fx, fy, fz, r2);
            else
                pair_sym32(xj, yj, zj, gmj, xi[u], yi[u], zi[u], gmi[u], keep, ax[u], ay[u], az[u],
                           fx, fy, fz, r2);
            if constexpr (MODE != 0) hit[u] = keep && r2 < th2[u];
        }
        if constexpr (MODE != 0) {
            // one branch per rotation step for the lane's IPL pairs
            bool any = hit[0];
#pragma unroll
            for (int u = 1; u < IPL; ++u) any = any || hit[u];
            if (any) {
                unsigned cnt = 0u;
#pragma unroll
                for (int u = 0; u < IPL; ++u) cnt += hit[u] ? 1u : 0u;
                unsigned q = atomicAdd(qn, cnt);
#pragma unroll
                for (int u = 0; u < IPL; ++u) {
                    if (hit[u]) {
                        if (q < (unsigned)kCrudeQ) {
                            qi[q] = ib + lt[u];
                            qj[q] = jsub + ((lane + k) & 63);
                        }
                        ++q;
                    }
                }
            }
        }
        fx = lane_rotate1(fx);
        fy = lane_rotate1(fy);
        fz = lane_rotate1(fz);
    }
}

// The queued pairs of the item so far (absolute body indices, n <=
// kCrudeQ): the exact crude test of the definition, the passing pairs
// gathered in LDS and appended to the candidate list with one atomic for
// the workgroup (a counter every workgroup hits once per flush, not once per
// candidate).  Called by the whole workgroup.
template <int BS>
__device__ void sym_flush(const KickArgs &ka, const int *qi, const int *qj, unsigned n, int2 *cl,
                          unsigned *cn, int *cbase)
{
    const Dev &d = ka.d;
    const int tid = threadIdx.x;
    for (unsigned e = tid; e < n; e += BS) {
        const int i = qi[e], j = qj[e];
        if (j > i && crude_pass(d, d.x, d.y, d.z, ka.hill_mode, ka.aE, ka.cs, ka.tau_abs, i, j)) {
            const unsigned k = atomicAdd(cn, 1u);
            cl[k] = make_int2(i, j);
        }
    }
    __syncthreads();
    const unsigned c = *cn;
    if (c) {
        if (tid == 0) *cbase = (int)atomicAdd(&d.ctr[C_CAND], (unsigned long long)c);
        __syncthreads();
        const long long b0 = *cbase;
        for (unsigned k = tid; k < c; k += BS)
            if (b0 + k < ka.cap) d.cand[b0 + k] = cl[k];
    }
}

// a tile whose hits overflowed the queue: the exact test of every pair of
// the tile with j > i (appended one by one; rare)
template <int BS, int IPL>
__device__ void sym_tile_exact(const KickArgs &ka, int jt, int jend, const int *iu, const bool *oku)
{
    const int je = min(jt + BS, jend);
#pragma unroll
    for (int u = 0; u < IPL; ++u)
        if (oku[u])
            for (int j = jt; j < je; ++j) crude_exact(ka, iu[u], j);
}

// REC: the variant that writes workgroup records (profiling with records;
// a separate instantiation, so the kernel timed otherwise carries no trace
// of them: any extra live value changes this kernel's register
// allocation).  Its occupancy is held at the plain variant's (waves per
// SIMD: 4 for the plain kick and the 128-thread, one-i crude kick, 3 for
// the other crude kicks), so that its records show the timed kernel's
// balance.
template <int BS, int IPL, int MODE, int PREC>
constexpr int kick_rec_waves()
{
    return MODE == 0 ? 4 : (IPL == 1 && BS == 128 ? 4 : 3);
}

template <int BS, int IPL, int MODE, int PREC, bool REC = false>
__global__ __launch_bounds__(BS)
__attribute__((amdgpu_waves_per_eu(REC ? kick_rec_waves<BS, IPL, MODE, PREC>() : 1, 4))) void k_kick_sym(
    KickArgs ka)
{
    static_assert(IPL == 1 || IPL == 2, "one or two i per lane");
    const Dev &d = ka.d;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if constexpr (REC) wg_start(ka.rec);
    int b = blockIdx.x;
    if (ka.remap) b = xcd_item(b, gridDim.x);
    if (b >= ka.nitems) return;
    if (d.ctr[C_STATUS] & S_FREEZE) return;   // a step left undone: nothing to compute
    const KickItem it = ka.items[b];
    constexpr int NW = BS / 64;
    constexpr int BI = BS * IPL;

    // the j-tile, each sub-tile of 64 stored twice in a row (128 entries)
    // (x, y) and (z, G m) of a j side by side: one 16-byte read each per
    // rotation step, at offsets from one address per unrolled group
    __shared__ double2 txy[NW][128], tzm[NW][128];
    __shared__ double wpart[NW][3][BS];
    __shared__ double smax[3][NW];
    // crude sweep: pairs under the tile bound, queued over the tiles of the
    // item (flushed when half full and at the item's end), and the pairs
    // passing the exact test before their one append
    __shared__ int qi[MODE ? kCrudeQ : 1], qj[MODE ? kCrudeQ : 1];
    __shared__ int2 cl[MODE ? kCrudeQ : 1];
    __shared__ unsigned qn, cn;
    __shared__ int cbase;

    const int s = it.sys;
    const int so = d.sys_off[s];
    const int ns = d.sys_off[s + 1] - so;
    const long long base = d.sys_poff[s];
    const int jend = it.j0 + it.nj;
    // the item's reaction slot; entry j is owned by thread (j - j0) % BS.
    // The first i-block stores every entry from max(j0, i0) on without
    // reading it; only the entries before (no i of the item precedes them)
    // are cleared here.
    double *rj = d.acc + base + (long long)it.slot * 3 * ns - so;
    const int jfirst = max(it.j0, it.i0);
    for (int k = tid; k < jfirst - it.j0; k += BS) {
        rj[it.j0 + k] = 0.0;
        rj[ns + it.j0 + k] = 0.0;
        rj[2 * ns + it.j0 + k] = 0.0;
    }
    if (MODE && tid == 0) {
        qn = 0u;
        cn = 0u;
    }
    unsigned qstart = 0;   // queue entries left by earlier tiles of the item (uniform)
    const double G = ka.G;
    const double seed = ka.r2seed, c158 = ka.c158;
    // 3/2 in a vector register: the correction's inner fma would otherwise
    // take two scalar operands and cost a move per pair
    double c32;
    asm volatile("v_mov_b64 %0, %1" : "=v"(c32) : "s"(ka.c32));
    for (int ib = it.i0; ib < it.i0 + it.ni; ib += BI) {
        const bool first_ib = ib == it.i0;
        const int nib = min(BI, it.i0 + it.ni - ib);
        // lane group u of wave w holds i = ib + 64 (IPL w + u) + lane
        double xi[IPL], yi[IPL], zi[IPL], gmi[IPL], hi[IPL], Ai[IPL], vi[IPL];
        double ax[IPL], ay[IPL], az[IPL], th2[IPL];
        int iu[IPL], lt[IPL];
        bool oku[IPL];
#pragma unroll
        for (int u = 0; u < IPL; ++u) {
            lt[u] = 64 * (IPL * wv + u) + lane;
            iu[u] = ib + lt[u];
            oku[u] = lt[u] < nib;
            const int i = iu[u];
            xi[u] = oku[u] ? d.x[i] : kFar;
            yi[u] = oku[u] ? d.y[i] : kFar;
            zi[u] = oku[u] ? d.z[i] : kFar;
            gmi[u] = oku[u] ? G * d.m[i] : 0.0;
            hi[u] = Ai[u] = vi[u] = 0.0;
            if (MODE && oku[u]) {
                hi[u] = d.ch[i];
                Ai[u] = d.A[i];
                vi[u] = d.cv[i];
            }
            ax[u] = ay[u] = az[u] = 0.0;
            th2[u] = -1.0;
        }
        const int iw = ib + 64 * IPL * wv;   // first i of this wave
        const bool wave_i = 64 * IPL * wv < nib;
        for (int jt = max(it.j0, ib); jt < jend; jt += BS) {
            const int j = jt + tid;
            const bool okj = j < jend;
            __syncthreads();   // the previous tile's LDS reads and queue are done
            {
                const double xj = okj ? d.x[j] : kFar, yj = okj ? d.y[j] : kFar;
                const double zj = okj ? d.z[j] : kFar, mj = okj ? G * d.m[j] : 0.0;
                txy[wv][lane] = txy[wv][lane + 64] = make_double2(xj, yj);
                tzm[wv][lane] = tzm[wv][lane + 64] = make_double2(zj, mj);
            }
            // this thread's reaction entry, read early (latency hidden by the
            // pairs); the item's first i-block starts it from zero
            double racc[3] = {0.0, 0.0, 0.0};
            if (okj && !first_ib) {
                racc[0] = rj[j];
                racc[1] = rj[ns + j];
                racc[2] = rj[2 * ns + j];
            }
            if constexpr (MODE != 0) {
                double t0 = okj ? d.ch[j] : 0.0, t1 = okj ? d.A[j] : 0.0, t2 = okj ? d.cv[j] : 0.0;
                t0 = wave_max(t0);
                t1 = wave_max(t1);
                t2 = wave_max(t2);
                if (lane == 0) {
                    smax[0][wv] = t0;
                    smax[1][wv] = t1;
                    smax[2][wv] = t2;
                }
            }
            __syncthreads();
            if constexpr (MODE != 0) {
                double HT = smax[0][0], AT = smax[1][0], VT = smax[2][0];
#pragma unroll
                for (int w2 = 1; w2 < NW; ++w2) {
                    HT = fmax(HT, smax[0][w2]);
                    AT = fmax(AT, smax[1][w2]);
                    VT = fmax(VT, smax[2][w2]);
                }
                // per-(i, tile) upper bound of the crude threshold (as in k_kick)
#pragma unroll
                for (int u = 0; u < IPL; ++u) {
                    double Rb;
                    if (MODE == 1)
                        Rb = ka.aE * (hi[u] + HT) * (Ai[u] + AT) / 2.0;
                    else
                        Rb = ka.aE * (hi[u] + HT);
                    const double th = ka.cs * (Rb + ka.tau_abs * (vi[u] + VT));
                    th2[u] = oku[u] ? th * th * 1.000000000001 : -1.0;
                }
            }
#pragma unroll 1
            for (int sub = 0; sub < NW; ++sub) {
                const int jw = jt + 64 * sub;
                double fx = 0.0, fy = 0.0, fz = 0.0;
                const int rel = jw - iw;   // a multiple of 64
                const double2 *pxy = &txy[sub][0], *pzm = &tzm[sub][0];
                // whole waves past the i-block's end or sub-tiles past the
                // chunk's end have no pairs (uniform per wave)
                if (!wave_i || jw >= jend || rel < 0) {
                    // nothing to add
                } else if (rel >= 64 * IPL) {
                    sym_subtile<MODE, PREC, IPL, SYM_FULL, SYM_FULL>(
                        pxy, pzm, lane, xi, yi, zi, gmi, th2, lt, seed, c158, c32, ax, ay,
                        az, fx, fy, fz, qi, qj, &qn, ib, jt + 64 * sub);
                } else if (IPL == 2 && rel == 64) {
                    sym_subtile<MODE, PREC, IPL, SYM_FULL, SYM_DIAG>(
                        pxy, pzm, lane, xi, yi, zi, gmi, th2, lt, seed, c158, c32, ax, ay,
                        az, fx, fy, fz, qi, qj, &qn, ib, jt + 64 * sub);
                } else {   // rel == 0
                    sym_subtile<MODE, PREC, IPL, SYM_DIAG, SYM_SKIP>(
                        pxy, pzm, lane, xi, yi, zi, gmi, th2, lt, seed, c158, c32, ax, ay,
                        az, fx, fy, fz, qi, qj, &qn, ib, jt + 64 * sub);
                }
                wpart[wv][0][64 * sub + lane] = fx;
                wpart[wv][1][64 * sub + lane] = fy;
                wpart[wv][2][64 * sub + lane] = fz;
            }
            __syncthreads();
            // the tile's reactions, waves in order, onto the slot
            if (okj) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    double sum = wpart[0][c][tid];
#pragma unroll
                    for (int w2 = 1; w2 < NW; ++w2) sum += wpart[w2][c][tid];
                    rj[c * ns + j] = racc[c] + sum;
                }
            }
            if constexpr (MODE != 0) {
                // qn is final (the barrier above follows every push)
                const unsigned nq = qn;
                unsigned keep = nq;
                if (nq > (unsigned)kCrudeQ) {
                    // this tile's pushes overflowed: drop them, test the tile
                    sym_tile_exact<BS, IPL>(ka, jt, jend, iu, oku);
                    keep = qstart;
                }
                const bool last = ib + BI >= it.i0 + it.ni && jt + BS >= jend;
                if (keep > (unsigned)kCrudeQ / 2 || (last && keep > 0)) {
                    sym_flush<BS>(ka, qi, qj, keep, cl, &cn, &cbase);
                    keep = 0;
                }
                __syncthreads();   // every thread has read qn and cn
                if (tid == 0) {
                    qn = keep;
                    cn = 0u;
                }
                qstart = keep;
            }
        }
        // forces on this i-block: i-side slot `chunk`
        const long long pb = base + (long long)it.chunk * 3 * ns;
#pragma unroll
        for (int u = 0; u < IPL; ++u) {
            if (oku[u]) {
                const int il = iu[u] - so;
                d.acc[pb + il] = ax[u];
                d.acc[pb + ns + il] = ay[u];
                d.acc[pb + 2 * ns + il] = az[u];
            }
        }
    }
    if constexpr (MODE != 0) {
        // the last tile flushes the queue; an item whose last i-block met
        // no tile would leave pairs here
        if (qstart > 0) sym_flush<BS>(ka, qi, qj, qstart, cl, &cn, &cbase);
    }
    if constexpr (REC) wg_finish(ka.rec);
}

// sum of the kick partials of body i (local index il of system s)
// Kick partials of body il of system s.  Full-matrix kick (K.z == 0): the
// K.x j-chunk slots.  Symmetric kick (K = {S, JC, RB}): i-side slots of the
// chunks from il's own chunk cx on (the chunks it meets as an i), then the
// j-side slots of its chunk, one per i-range of RB bodies below the chunk's
// end.  Always summed in slot order.
// share `part` of P of the partial-sum slots of local body il: the body's
// slots (its i-side chunks, then for the symmetric kick the j-side
// i-ranges that reach it) in list order, every P-th from the part-th
// slots q = part, part + P, ... < qe of the list whose entry q is slot
// q0 + q below qs and slot base + (q - qs) from qs on, added in list order.
// Four slots are requested before any is added, so the loads' latencies
// overlap (a loop that adds each value as it arrives waits once per slot).
__device__ __forceinline__ void sum_slot_list(const double *p, long long ns, int part, int P,
                                              int qe, int qs, long long q0, long long base,
                                              double &ax, double &ay, double &az)
{
    int q = part;
    for (; q + 3 * P < qe; q += 4 * P) {
        double vx[4], vy[4], vz[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int qq = q + u * P;
            const long long sl = qq < qs ? q0 + qq : base + (qq - qs);
            vx[u] = p[(3 * sl) * ns];
            vy[u] = p[(3 * sl + 1) * ns];
            vz[u] = p[(3 * sl + 2) * ns];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            ax += vx[u];
            ay += vy[u];
            az += vz[u];
        }
    }
    for (; q < qe; q += P) {
        const long long sl = q < qs ? q0 + q : base + (q - qs);
        ax += p[(3 * sl) * ns];
        ay += p[(3 * sl + 1) * ns];
        az += p[(3 * sl + 2) * ns];
    }
}

__device__ __forceinline__ void sum_partials(const Dev &d, const int4 *sysK, int s, int il,
                                             int part, int P, double a[3])
{
    const int ns = d.sys_off[s + 1] - d.sys_off[s];
    const int4 K = sysK[s];
    const double *p = d.acc + d.sys_poff[s] + il;
    double ax = 0.0, ay = 0.0, az = 0.0;
    if (K.w == 2) {
        // balanced rows (K = {KX, BI, row table, 2}): the i-side slots of
        // the items of il's row, then the reaction slots of the rows up to
        // and including its own
        const int r = il / K.y;
        const int kr = d.krow[K.z + r];
        sum_slot_list(p, ns, part, P, kr + r + 1, kr, 0, K.x, ax, ay, az);
    } else {
        int c0 = 0, c1 = K.x, r1 = 0;
        if (K.z > 0) {
            const int cx = il / K.y;
            c0 = cx;
            r1 = (min((cx + 1) * K.y, ns) + K.z - 1) / K.z;
        }
        const int ni = c1 - c0;
        sum_slot_list(p, ns, part, P, ni + r1, ni, c0, K.x, ax, ay, az);
    }
    a[0] = ax;
    a[1] = ay;
    a[2] = az;
}

// ------------------------------------------------------------------------
// First kick applied (v += dt a), state snapshot (q0, v0), then E_Kep(tau)
// of every body (Sec. 2.3 steps 2-3).  mode < 0 skips the kick part,
// kick_only skips the Kepler part (operator-level entry points).
// ------------------------------------------------------------------------
struct ApplyArgs {
    Dev d;
    const int4 *chunks; // body chunks of this launch (one per workgroup)
    const int4 *sysK;  // partial-slot layout of the kick being applied
    double dt_kick, dt_kep, G;
    int do_kick, do_kep, snapshot, kepler_mode, momentum;
};

template <int BS, int P>
__global__ __launch_bounds__(BS * P) void k_apply_kepler(ApplyArgs a)
{
    // P threads per body share the reduction of its partial-sum slots (one
    // body's serial sum over tens of slots is bound by memory latency): the
    // p-th thread group of BS sums every P-th slot from the p-th for the
    // chunk's consecutive bodies, and the P shares are added in order.  The
    // per-body steps then run on the first BS threads.
    static_assert(BS == 64, "the chunk's bodies are one wave (the statistics are wave sums)");
    __shared__ double share[P > 1 ? P : 1][3][BS];
    __shared__ int bad;
    const Dev &d = a.d;
    const int4 bc = a.chunks[blockIdx.x];
    const int s = bc.x;
    const int t = threadIdx.x;
    if (t == 0) bad = 0;
    double sh[3] = {0.0, 0.0, 0.0};
    if (P > 1 && a.do_kick) {
        const int bt = t % BS, part = t / BS;
        if (bt < bc.z) sum_partials(d, a.sysK, s, bc.y + bt - d.sys_off[s], part, P, sh);
        share[part][0][bt] = sh[0];
        share[part][1][bt] = sh[1];
        share[part][2][bt] = sh[2];
    }
    __syncthreads();
    double mom[3] = {0.0, 0.0, 0.0};
    int kit = -1, krs = 0;   // this body's Kepler iterations and restart
    if (t < BS && t < bc.z) {
        const int i = bc.y + t;
        double x = d.x[i], y = d.y[i], z = d.z[i];
        double vx = d.vx[i], vy = d.vy[i], vz = d.vz[i];
        if (a.do_kick) {
            double acc[3];
            if constexpr (P > 1) {
                for (int c = 0; c < 3; ++c) {
                    acc[c] = share[0][c][t];
                    for (int q = 1; q < P; ++q) acc[c] += share[q][c][t];
                }
            } else {
                sum_partials(d, a.sysK, s, i - d.sys_off[s], 0, 1, acc);
            }
            vx += a.dt_kick * acc[0];
            vy += a.dt_kick * acc[1];
            vz += a.dt_kick * acc[2];
        }
        if (a.snapshot) {
            d.x0[i] = x;
            d.y0[i] = y;
            d.z0[i] = z;
            d.vx0[i] = vx;
            d.vy0[i] = vy;
            d.vz0[i] = vz;
        }
        if (a.do_kep) {
            int fail, restart;
            kit = kepler_advance(a.G * d.sys_m0[s], a.kepler_mode, d.guess, a.dt_kep, x, y, z, vx,
                                 vy, vz, fail, restart);
            krs = restart;
            if (fail) atomicOr(&bad, (int)S_KEPLER);
        }
        if (!(isfinite(x) && isfinite(y) && isfinite(z) && isfinite(vx) && isfinite(vy) &&
              isfinite(vz)))
            atomicOr(&bad, (int)S_NONFINITE);
        d.x[i] = x;
        d.y[i] = y;
        d.z[i] = z;
        d.vx[i] = vx;
        d.vy[i] = vy;
        d.vz[i] = vz;
        const double mi = d.m[i];
        mom[0] = mi * vx;
        mom[1] = mi * vy;
        mom[2] = mi * vz;
    }
    if (a.momentum) {
        // the chunk's bodies are on the first wave (BS = kChunkK)
        static_assert(BS == kChunkK, "one momentum partial per Kepler-pass chunk");
        if (t < 64) {
            wave_sum3(mom);
            if (t == 0)
                for (int k = 0; k < 3; ++k) d.pm[3 * blockIdx.x + k] = mom[k];
        }
    }
    if (a.do_kep && t < 64) {
        // the chunk's iteration statistics by ballots over its wave (one
        // per iteration count present, counted upward until every body is
        // counted), instead of 64 lanes' atomics on one LDS word each
        unsigned long long *ks = d.kstat + (size_t)(blockIdx.x & (kStatStripes - 1)) * kStatStride;
        unsigned long long rem = __ballot(kit >= 0);
        unsigned long long sum = 0, top = 0;
        for (int b = 0; rem != 0ull; ++b) {
            const unsigned long long m = __ballot(kit == b);
            if (m) {
                const unsigned long long c = (unsigned long long)__popcll(m);
                if (t == 0) atomicAdd(&ks[b < kHist ? b : kHist - 1], c);
                sum += c * (unsigned long long)b;
                top = (unsigned long long)b;
                rem &= ~m;
            }
        }
        const unsigned long long nrs = (unsigned long long)__popcll(__ballot(krs != 0));
        if (t == 0) {
            atomicAdd(&ks[kHist], sum);
            atomicMax(&ks[kHist + 1], top);
            if (nrs) atomicAdd(&ks[kHist + 2], nrs);
        }
    }
    __syncthreads();
    if (t == 0 && bad) latch(d.ctr, (unsigned long long)bad);
}

// ------------------------------------------------------------------------
// Sec. 2.4 fine sweep: cubic Hermite interpolant of D(s) = |dq(s)|^2 over
// the step from (q0, v0) and (q1, v1), its minimum over [0, 1] compared
// with a_E x mutual Hill radius (cube-free form) or a_E x (sum of Hill
// radii).  Fixed IEEE operation order, no contraction.
// ------------------------------------------------------------------------
__device__ __forceinline__ double cubic_at(double c0, double c1, double c2, double c3, double s)
{
    return c0 + s * (c1 + s * (c2 + s * c3));
}

__device__ int fine_pair(int hill_mode, double aE, double m0, double tau, double mi, double mj,
                         double hi, double hj, double Ai, double Aj, const double a0[3],
                         const double b0[3], const double a1[3], const double b1[3], double &lhs,
                         double &rhs)
{
    const double D0 = a0[0] * a0[0] + a0[1] * a0[1] + a0[2] * a0[2];
    const double D1 = a1[0] * a1[0] + a1[1] * a1[1] + a1[2] * a1[2];
    const double d0 = 2.0 * tau * (a0[0] * b0[0] + a0[1] * b0[1] + a0[2] * b0[2]);
    const double d1 = 2.0 * tau * (a1[0] * b1[0] + a1[1] * b1[1] + a1[2] * b1[2]);
    const double c0 = D0, c1 = d0;
    const double c2 = 3.0 * (D1 - D0) - 2.0 * d0 - d1;
    const double c3 = 2.0 * (D0 - D1) + d0 + d1;
    double Dm = (D0 < D1) ? D0 : D1;
    const double disc = c2 * c2 - 3.0 * c3 * c1;
    if (disc >= 0.0) {
        const double sq = sqrt(disc);
        const double qq = -(c2 + (c2 >= 0.0 ? sq : -sq));
        if (c3 != 0.0) {
            const double sr = qq / (3.0 * c3);
            if (sr > 0.0 && sr < 1.0) {
                const double D = cubic_at(c0, c1, c2, c3, sr);
                if (D < Dm) Dm = D;
            }
        }
        if (qq != 0.0) {
            const double sr = c1 / qq;
            if (sr > 0.0 && sr < 1.0) {
                const double D = cubic_at(c0, c1, c2, c3, sr);
                if (D < Dm) Dm = D;
            }
        }
    }
    if (Dm < 0.0) Dm = 0.0;
    if (hill_mode == 0) {
        const double T = aE * (Ai + Aj) / 2.0;
        const double M = (mi + mj) / (3.0 * m0);
        const double T2 = T * T;
        lhs = Dm * Dm * Dm;
        rhs = T2 * T2 * T2 * M * M;
    } else {
        const double R = aE * (hi * Ai + hj * Aj);
        lhs = Dm;
        rhs = R * R;
    }
    return lhs < rhs;
}

struct FineArgs {
    Dev d;
    double tau, aE, cs, tau_abs;
    long long cap;
    int hill_mode;
    int n_eitems;   // all-pairs tiles (the energy items) for the overflow sweep
};

// fine test of candidate (i, j), i < j, appended to its system's segment
// when it is an encounter (the count is kept even past the segment's end;
// k_sets adds the systems' counts into C_ENC).  The lanes of a wave that
// append to the same system as its first appending lane share one atomic
// (a counter hit once per pair serialises in its L2 channel).
__device__ __forceinline__ void fine_one(const FineArgs &a, int i, int j)
{
    const Dev &d = a.d;
    const double a0[3] = {d.x0[j] - d.x0[i], d.y0[j] - d.y0[i], d.z0[j] - d.z0[i]};
    const double b0[3] = {d.vx0[j] - d.vx0[i], d.vy0[j] - d.vy0[i], d.vz0[j] - d.vz0[i]};
    const double a1[3] = {d.x[j] - d.x[i], d.y[j] - d.y[i], d.z[j] - d.z[i]};
    const double b1[3] = {d.vx[j] - d.vx[i], d.vy[j] - d.vy[i], d.vz[j] - d.vz[i]};
    double lhs, rhs;
    const int s = d.body_sys[i];
    const int f = fine_pair(a.hill_mode, a.aE, d.sys_m0[s], a.tau, d.m[i], d.m[j], d.h[i], d.h[j],
                            d.A[i], d.A[j], a0, b0, a1, b1, lhs, rhs);
    const unsigned long long m = __ballot(f);
    if (!m) return;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)m) - 1;
    const int sl = __shfl(s, leader, 64);
    const unsigned long long same = __ballot(f && s == sl);
    int base = 0;
    if (lane == leader) base = atomicAdd(&d.sys_ecnt[sl], __popcll(same));
    base = __shfl(base, leader, 64);
    if (!f) return;
    const int slot = s == sl ? base + __popcll(same & __lanemask_lt()) : atomicAdd(&d.sys_ecnt[s], 1);
    if (slot < d.sys_eoff[s + 1] - d.sys_eoff[s]) d.enc[d.sys_eoff[s] + slot] = make_int2(i, j);
}

// The candidates of the crude sweep, or, when more candidates were found
// than the list holds, every pair i < j of every system: the crude test of
// the definition at the snapshot positions (the first kick's positions, so
// the same decisions the sweep took) and the fine test for those passing.
// Either way no encounter is lost; the second way costs one all-pairs pass
// and is counted in C_FALLBACK.
__global__ __launch_bounds__(256) void k_fine(FineArgs a)
{
    const Dev &d = a.d;
    if (d.ctr[C_STATUS] & S_FREEZE) return;
    const unsigned long long cnt = d.ctr[C_CAND];
    if ((long long)cnt <= a.cap) {
        const long long n = (long long)cnt;
        for (long long k = blockIdx.x * 256ll + threadIdx.x; k < n; k += (long long)gridDim.x * 256) {
            const int2 p = d.cand[k];
            fine_one(a, p.x, p.y);
        }
        return;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) d.ctr[C_FALLBACK] += 1;
    for (int it = blockIdx.x; it < a.n_eitems; it += gridDim.x) {
        const KickItem e = d.eitems[it];
        if ((int)threadIdx.x >= e.ni) continue;
        const int i = e.i0 + threadIdx.x;
        const int jhi = e.j0 + e.nj;
        for (int j = max(e.j0, i + 1); j < jhi; ++j)
            if (crude_pass(d, d.x0, d.y0, d.z0, a.hill_mode, a.aE, a.cs, a.tau_abs, i, j))
                fine_one(a, i, j);
    }
}

// stateless fine sweep on caller arrays (SoA [3][n])
__global__ __launch_bounds__(256) void k_fine_standalone(
    int hill_mode, double aE, double m0, double tau, long long n, const double *m, const double *h,
    const double *A, const double *q0, const double *v0, const double *q1, const double *v1,
    long long np, const int *pairs, int *flags, double *lhs_out, double *rhs_out)
{
    const long long k = blockIdx.x * 256ll + threadIdx.x;
    if (k >= np) return;
    const int i = pairs[2 * k], j = pairs[2 * k + 1];
    double a0[3], b0[3], a1[3], b1[3];
    for (int c = 0; c < 3; ++c) {
        a0[c] = q0[c * n + j] - q0[c * n + i];
        b0[c] = v0[c * n + j] - v0[c * n + i];
        a1[c] = q1[c * n + j] - q1[c * n + i];
        b1[c] = v1[c * n + j] - v1[c * n + i];
    }
    double lhs, rhs;
    flags[k] = fine_pair(hill_mode, aE, m0, tau, m[i], m[j], h[i], h[j], A[i], A[j], a0, b0, a1,
                         b1, lhs, rhs);
    if (lhs_out) lhs_out[k] = lhs;
    if (rhs_out) rhs_out[k] = rhs;
}

// ------------------------------------------------------------------------
// Sec. 2.3 step 4 / Sec. 2.4: canonical encounter list, division into
// non-intersecting sets (connected components; a set is labelled by its
// smallest body index, members ascending), r_crit = a_H max h_i a_i.
// One workgroup; everything in LDS (<= kCapE pairs).
// ------------------------------------------------------------------------
// Ascending bitonic sort of the 32-bit keys v[0..n2) by one workgroup of
// kSetsThreads threads, n2 = R * kSetsThreads a power of two.  Thread t keeps
// the R keys at positions t*R .. t*R+R-1 in registers: compare-exchanges
// between keys of one thread run in registers, between lanes of one wave
// through cross-lane shuffles, and only partners in different waves (distance
// >= 64 R) go through LDS with workgroup barriers.  Same network, and so the
// same result, as the textbook LDS bitonic sort.
template <int R>
__device__ void bitonic_regs(unsigned *v, int n2)
{
    const int t = threadIdx.x;
    unsigned e[R];
#pragma unroll
    for (int r = 0; r < R; ++r) e[r] = v[t * R + r];
    for (int k = 2; k <= n2; k <<= 1) {
        int jx = k >> 1;
        for (; jx >= 64 * R; jx >>= 1) {
            __syncthreads();
#pragma unroll
            for (int r = 0; r < R; ++r) v[t * R + r] = e[r];
            __syncthreads();
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = t * R + r;
                const unsigned p = v[i ^ jx];
                const bool keep_min = ((i & jx) == 0) == ((i & k) == 0);
                e[r] = keep_min ? min(e[r], p) : max(e[r], p);
            }
        }
        for (; jx >= R; jx >>= 1) {
            const int lm = jx / R;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = t * R + r;
                const unsigned p = (unsigned)__shfl_xor((int)e[r], lm, 64);
                const bool keep_min = ((i & jx) == 0) == ((i & k) == 0);
                e[r] = keep_min ? min(e[r], p) : max(e[r], p);
            }
        }
#pragma unroll
        for (int jj = R / 2; jj > 0; jj >>= 1) {
            if (jj >= k) continue;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                if (r & jj) continue;
                const unsigned x = e[r], y = e[r | jj];
                const bool asc = ((t * R + r) & k) == 0;
                e[r] = asc ? min(x, y) : max(x, y);
                e[r | jj] = asc ? max(x, y) : min(x, y);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) v[t * R + r] = e[r];
    __syncthreads();
}

// v[0..n2), n2 a power of two in [kSetsThreads, 32 kSetsThreads]
__device__ void block_sort_u32(unsigned *v, int n2)
{
    // the same n2 on every lane: scalar loop bounds and a scalar switch
    n2 = __builtin_amdgcn_readfirstlane(n2);
    switch (n2 / kSetsThreads) {
    case 1: bitonic_regs<1>(v, n2); break;
    case 2: bitonic_regs<2>(v, n2); break;
    case 4: bitonic_regs<4>(v, n2); break;
    case 8: bitonic_regs<8>(v, n2); break;
    case 16: bitonic_regs<16>(v, n2); break;
    default: bitonic_regs<32>(v, n2); break;
    }
}

// inclusive scan over the wave by DPP moves (VALU operations, no LDS round
// trips): row_shr 1, 2, 4, 8 within each row of 16 (a lane with no source
// adds 0), then row_bcast 15 carries row 0's total into row 1 and row 2's
// into row 3, and row_bcast 31 the total of rows 0-1 into rows 2 and 3
__device__ __forceinline__ int wave_incl_scan(int v)
{
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, false);   // row_shr:1
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, false);   // row_shr:2
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, false);   // row_shr:4
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, false);   // row_shr:8
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);   // row_bcast:15, rows 1, 3
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);   // row_bcast:31, rows 2, 3
    return v;
}

// exclusive scan of v[0..n) in place by one workgroup (thread-contiguous
// runs, wave scans, one scan of the wave totals); returns the total.
// tmp needs blockDim/64 + 1 entries.
__device__ int block_scan_excl(int *v, int n, int *tmp)
{
    const int T = blockDim.x;
    const int nw = T >> 6;
    const int per = (n + T - 1) / T;
    const int t = threadIdx.x;
    int s = 0;
    for (int k = 0; k < per; ++k) {
        const int i = t * per + k;
        if (i < n) s += v[i];
    }
    const int incl = wave_incl_scan(s);
    if ((t & 63) == 63) tmp[t >> 6] = incl;
    __syncthreads();
    if (t < 64) {
        const int w = (t < nw) ? tmp[t] : 0;
        const int wi = wave_incl_scan(w);
        if (t < nw) tmp[t] = wi - w;
        if (t == nw - 1) tmp[nw] = wi;
    }
    __syncthreads();
    int run = tmp[t >> 6] + incl - s;
    for (int k = 0; k < per; ++k) {
        const int i = t * per + k;
        if (i < n) {
            const int c = v[i];
            v[i] = run;
            run += c;
        }
    }
    const int total = tmp[nw];
    __syncthreads();
    return total;
}

struct SetsArgs {
    Dev d;
    double aH;
    double planet_mass;   // > 0: whole-system rule on (see k_sets)
};

template <int T>
__device__ void sets_global(const SetsArgs &a, int sys, int *tmp, int &base_set, int &base_mem,
                            int &s_whole);

// the largest set of the workgroup's sets onto the step's counter: a wave
// maximum first, so one atomic per wave goes to the counter's word, not one
// per thread that met a set
__device__ __forceinline__ void note_max_set(unsigned long long *ctr, unsigned big)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) big = max(big, (unsigned)__shfl_xor((int)big, o, 64));
    if ((threadIdx.x & 63) == 0 && big) atomicMax(ctr, (unsigned long long)big);
}

// binary search of v in the ascending u[0..n)
__device__ __forceinline__ int lower_rank(const unsigned *u, int n, unsigned v)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (u[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// One workgroup, LDS only (<= kCapE pairs): unique bodies of the encounter
// pairs (bitonic sort + scan), pairs as rank pairs, labels propagated to the
// component minimum, members ordered by (component, index) with one more
// sort, r_crit per set.  Ranks follow body order, so "smallest rank" is
// "smallest body index".  The pair list itself is left in append order (the
// ABI returns it sorted on the host).
__global__ __launch_bounds__(kSetsThreads) void k_sets(SetsArgs a)
{
    const Dev &d = a.d;
    __shared__ unsigned int ep[kCapU];   // endpoints, later member keys
    __shared__ unsigned int uq[kCapU];   // unique bodies (ascending)
    __shared__ unsigned int lab[kCapU];  // component labels (ranks)
    __shared__ unsigned int rp[kCapE];   // pairs as rank pairs
    __shared__ int flag[kCapU];          // scan scratch
    __shared__ int tmp[kSetsThreads / 64 + 1];
    __shared__ int base_set, base_mem, s_whole;
    const int t = threadIdx.x;
    const int sys = blockIdx.x;
    const int cnt = d.sys_ecnt[sys];
    const int2 *enc = d.enc + d.sys_eoff[sys];
    if (d.ctr[C_STATUS] & S_FREEZE) return;
    if (t == 0 && cnt > 0) atomicAdd(&d.ctr[C_ENC], (unsigned long long)cnt);
    if (cnt > d.sys_eoff[sys + 1] - d.sys_eoff[sys]) {
        // more pairs than the system's segment holds: the step is left undone
        if (t == 0) latch(d.ctr, S_ENC_OVF);
        return;
    }
    if (cnt > kCapE) {
        // beyond LDS: the same partition in the system's global scratch
        sets_global<kSetsThreads>(a, sys, tmp, base_set, base_mem, s_whole);
        return;
    }
    const int ne = cnt;
    if (ne == 0) return;
    // the bodies taking part (ascending, uq[0..nu)) and every pair as the
    // ranks of its two bodies in that list
    const int so = d.sys_off[sys], nsb = d.sys_off[sys + 1] - so;
    int nu;
    if (nsb <= 32 * kCapU) {
        // from a bitmap of the system's bodies (in flag): the set bits in
        // ascending order are the bodies, a body's rank is the number of set
        // bits before it (popcount prefix over the words, in ep)
        unsigned *bits = reinterpret_cast<unsigned *>(flag);
        int *wpre = reinterpret_cast<int *>(ep);
        const int nw = (nsb + 31) >> 5;
        for (int k = t; k < nw; k += blockDim.x) bits[k] = 0u;
        __syncthreads();
        // the pairs are read once and kept in lab (free until the labels
        // are set up) for the ranks below
        for (int k = t; k < ne; k += blockDim.x) {
            const int2 p = enc[k];
            atomicOr(&bits[(p.x - so) >> 5], 1u << ((p.x - so) & 31));
            atomicOr(&bits[(p.y - so) >> 5], 1u << ((p.y - so) & 31));
            lab[2 * k] = (unsigned)(p.x - so);
            lab[2 * k + 1] = (unsigned)(p.y - so);
        }
        __syncthreads();
        for (int k = t; k < nw; k += blockDim.x) wpre[k] = __popc(bits[k]);
        __syncthreads();
        nu = block_scan_excl(wpre, nw, tmp);
        for (int k = t; k < nw; k += blockDim.x) {
            unsigned w = bits[k];
            int r = wpre[k];
            while (w) {
                uq[r++] = (unsigned)(so + (k << 5) + __ffs(w) - 1);
                w &= w - 1u;
            }
        }
        for (int k = t; k < ne; k += blockDim.x) {
            const int bx = (int)lab[2 * k], by = (int)lab[2 * k + 1];
            const int ri = wpre[bx >> 5] + __popc(bits[bx >> 5] & ((1u << (bx & 31)) - 1u));
            const int rj = wpre[by >> 5] + __popc(bits[by >> 5] & ((1u << (by & 31)) - 1u));
            rp[k] = ((unsigned)ri << 16) | (unsigned)rj;
        }
        __syncthreads();
    } else {
        // larger systems: sort the endpoints, keep the first of each run,
        // rank by binary search
        int m2 = kSetsThreads;
        while (m2 < 2 * ne) m2 <<= 1;
        for (int k = t; k < m2; k += blockDim.x) {
            if (k < 2 * ne) {
                const int2 p = enc[k >> 1];
                ep[k] = (unsigned)((k & 1) ? p.y : p.x);
            } else {
                ep[k] = 0xffffffffu;
            }
        }
        __syncthreads();
        block_sort_u32(ep, m2);
        for (int k = t; k < 2 * ne; k += blockDim.x) flag[k] = (k == 0 || ep[k] != ep[k - 1]) ? 1 : 0;
        __syncthreads();
        for (int k = t; k < 2 * ne; k += blockDim.x) lab[k] = (unsigned)flag[k];
        __syncthreads();
        nu = block_scan_excl(flag, 2 * ne, tmp);
        for (int k = t; k < 2 * ne; k += blockDim.x)
            if (lab[k]) uq[flag[k]] = ep[k];
        __syncthreads();
        for (int k = t; k < ne; k += blockDim.x) {
            const int2 p = enc[k];
            const int ri = lower_rank(uq, nu, (unsigned)p.x);
            const int rj = lower_rank(uq, nu, (unsigned)p.y);
            rp[k] = ((unsigned)ri << 16) | (unsigned)rj;
        }
        __syncthreads();
    }
    for (int k = t; k < nu; k += blockDim.x) lab[k] = (unsigned)k;
    __syncthreads();
    // union-find with union by minimum: a root is only ever linked below a
    // smaller root, so every component ends rooted at its smallest rank
    // whatever the order of the links
    volatile unsigned *vlab = lab;   // re-read: other lanes link roots meanwhile
    for (int k = t; k < ne; k += blockDim.x) {
        unsigned x = rp[k] >> 16, y = rp[k] & 0xffffu;
        for (;;) {
            while (vlab[x] != x) x = vlab[x];
            while (vlab[y] != y) y = vlab[y];
            if (x == y) break;
            if (x > y) {
                const unsigned w = x;
                x = y;
                y = w;
            }
            // link root y below x unless y stopped being a root meanwhile
            const unsigned old = atomicCAS(&lab[y], y, x);
            if (old == y) break;
            y = old;
        }
    }
    __syncthreads();
    for (int k = t; k < nu; k += blockDim.x) {
        unsigned x = k;
        while (lab[x] != x) x = lab[x];
        flag[k] = (int)x;
    }
    __syncthreads();
    for (int k = t; k < nu; k += blockDim.x) lab[k] = (unsigned)flag[k];
    __syncthreads();
    // roots -> set ids in ascending root order
    for (int k = t; k < nu; k += blockDim.x) flag[k] = (lab[k] == (unsigned)k) ? 1 : 0;
    __syncthreads();
    const int nsets = block_scan_excl(flag, nu, tmp);
    // Sec. 2.3, after the steps: a set holding two planets makes the step
    // integrate the whole system with the Hermite -- one set of all its
    // bodies (ascending) with r_crit infinite, so K = 0 and W = 1 for every
    // pair.  Planet counts per set reuse rp (the rank pairs are done with).
    if (a.planet_mass > 0.0) {
        for (int k = t; k < nsets; k += blockDim.x) rp[k] = 0u;
        if (t == 0) s_whole = 0;
        __syncthreads();
        for (int k = t; k < nu; k += blockDim.x)
            if (d.m[uq[k]] >= a.planet_mass && atomicAdd(&rp[flag[lab[k]]], 1u) >= 1u) s_whole = 1;
        __syncthreads();
        if (s_whole) {
            const int o = d.sys_off[sys], ns = d.sys_off[sys + 1] - o;
            if (t == 0) {
                base_set = (int)atomicAdd(&d.ctr[C_NSETS], 1ull);
                base_mem = (int)atomicAdd(&d.ctr[C_NU], (unsigned long long)ns);
            }
            __syncthreads();
            const int bs = base_set, bm = base_mem;
            for (int k = t; k < ns; k += blockDim.x) d.set_mem[bm + k] = o + k;
            if (t == 0) {
                d.set_start[bs] = bm;
                d.set_count[bs] = ns;
                d.set_rc[bs] = INFINITY;
                if (ns <= kWaveMax)
                    d.set_list[(int)atomicAdd(&d.ctr[C_NSMALL], 1ull)] = bs;
                else
                    d.set_list[d.setcap - 1 - (int)atomicAdd(&d.ctr[C_NBIG], 1ull)] = bs;
                if (ns > kCoopMin) atomicAdd(&d.ctr[C_NGRID], 1ull);
                atomicMax(&d.ctr[C_MAXSET], (unsigned long long)ns);
                atomicAdd(&d.ctr[C_TENC], (unsigned long long)ne);
                atomicAdd(&d.ctr[C_WHOLE], 1ull);
            }
            return;
        }
    }
    // members sorted by (root rank, rank)
    int u2 = kSetsThreads;
    while (u2 < nu) u2 <<= 1;
    for (int k = t; k < u2; k += blockDim.x)
        ep[k] = (k < nu) ? ((lab[k] << 16) | (unsigned)k) : 0xffffffffu;
    __syncthreads();
    block_sort_u32(ep, u2);
    // global slots of this system's sets and members
    if (t == 0) {
        base_set = (int)atomicAdd(&d.ctr[C_NSETS], (unsigned long long)nsets);
        base_mem = (int)atomicAdd(&d.ctr[C_NU], (unsigned long long)nu);
    }
    __syncthreads();
    const int bs = base_set, bm = base_mem;
    // member k of the sorted list: body uq[r], local set flag[root]; the
    // local set index is kept in lab[k] (lab is free once the keys are built)
    for (int k = t; k < nu; k += blockDim.x) {
        const unsigned r = ep[k] & 0xffffu;
        d.set_mem[bm + k] = (int)uq[r];
        const unsigned root = ep[k] >> 16;
        const bool first = (k == 0) || ((ep[k - 1] >> 16) != root);
        const int sid = flag[root];
        if (first) {
            d.set_start[bs + sid] = bm + k;
            rp[sid] = (unsigned)k;   // local start (the rank pairs are done with)
        }
        lab[k] = (unsigned)sid;
    }
    __syncthreads();
    // r_crit = a_H max_{i in S} h_i a_i: one thread per member, max through
    // LDS atomics on the bit patterns (non-negative doubles order as
    // integers); flag's storage is reused (nsets <= nu / 2 <= kCapE)
    unsigned long long *rcb = (unsigned long long *)flag;
    for (int k = t; k < nsets; k += blockDim.x) rcb[k] = 0ull;
    __syncthreads();
    for (int k = t; k < nu; k += blockDim.x) {
        const int i = (int)uq[ep[k] & 0xffffu];
        const double rh = d.h[i] * d.A[i];
        atomicMax(&rcb[lab[k]], (unsigned long long)__double_as_longlong(rh));
    }
    __syncthreads();
    for (int sidx = t; sidx < nsets; sidx += blockDim.x)
        d.set_rc[bs + sidx] = a.aH * __longlong_as_double((long long)rcb[sidx]);
    // set sizes from the local starts (and the largest); the work lists of
    // the Hermite kernel: the sets' places in the small and the larger list
    // from one scan of packed counts (small sets in the low, larger ones in
    // the high 16 bits; nsets <= kCapE), one atomic per list for the base
    __syncthreads();   // rcb (flag) read
    unsigned int big = 0;
    for (int sid = t; sid < nsets; sid += blockDim.x) {
        const int n = (sid + 1 < nsets ? (int)rp[sid + 1] : nu) - (int)rp[sid];
        d.set_count[bs + sid] = n;
        if ((unsigned)n > big) big = (unsigned)n;
        if (n > kCoopMin) atomicAdd(&d.ctr[C_NGRID], 1ull);   // rare: the grid phase
        flag[sid] = n <= kWaveMax ? 1 : 0x10000;
    }
    __syncthreads();
    const int tot = block_scan_excl(flag, nsets, tmp);
    if (t == 0) {
        base_set = (int)atomicAdd(&d.ctr[C_NSMALL], (unsigned long long)(tot & 0xffff));
        base_mem = (int)atomicAdd(&d.ctr[C_NBIG], (unsigned long long)(tot >> 16));
    }
    __syncthreads();
    for (int sid = t; sid < nsets; sid += blockDim.x) {
        const int n = (sid + 1 < nsets ? (int)rp[sid + 1] : nu) - (int)rp[sid];
        const int pos = flag[sid];
        if (n <= kWaveMax)
            d.set_list[base_set + (pos & 0xffff)] = bs + sid;
        else
            d.set_list[d.setcap - 1 - (base_mem + (pos >> 16))] = bs + sid;
    }
    note_max_set(&d.ctr[C_MAXSET], big);
    if (t == 0) atomicAdd(&d.ctr[C_TENC], (unsigned long long)ne);
}

// ------------------------------------------------------------------------
// Set partition of a system with more encounter pairs than LDS holds
// (Sec. 2.3 step 4, the same result as k_sets), run by that system's
// workgroup of k_sets (T threads) with everything in the system's global
// scratch -- the bodies in
// encounters from a bitmap of the system (ascending, ranked by popcount
// prefixes), union-find with union by minimum, roots numbered in ascending
// order, members sorted by (root, body) with a bitonic sort, r_crit =
// a_H max h_i a_i per set (Sec. 2.2), the Hermite work lists.  Words that
// atomics change are read back with atomic loads: atomics act in the L2,
// plain loads may be served by the compute unit's L1.
// ------------------------------------------------------------------------
__device__ __forceinline__ unsigned ld_u32(const unsigned *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ int ld_i32(const int *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int T>
__device__ void sets_global(const SetsArgs &a, int sys, int *tmp, int &base_set, int &base_mem,
                            int &s_whole)
{
    const Dev &d = a.d;
    const int t = threadIdx.x;
    {
        const int ne = d.sys_ecnt[sys];
        const int2 *enc = d.enc + d.sys_eoff[sys];
        const int so = d.sys_off[sys], nsb = d.sys_off[sys + 1] - so;
        // scratch of gs_slots(nsb) 64-bit slots (see qsym_common.hpp)
        unsigned long long *g = d.gsa + d.sys_goff[sys];
        const int nw = (int)gs_words(nsb);
        const long long wh = (gs_words(nsb) + 1) / 2, nh = (nsb + 1) / 2;
        unsigned *bits = reinterpret_cast<unsigned *>(g);
        int *wpre = reinterpret_cast<int *>(g + wh);
        int *uq = reinterpret_cast<int *>(g + 2 * wh);
        int *lab = reinterpret_cast<int *>(g + 2 * wh + nh);
        int *root = reinterpret_cast<int *>(g + 2 * wh + 2 * nh);
        unsigned long long *key = g + 2 * wh + 3 * nh;
        // the bodies taking part: set bits of the system's bitmap; a body's
        // rank is the number of set bits before it
        for (int k = t; k < nw; k += T) bits[k] = 0u;
        __syncthreads();
        for (int k = t; k < ne; k += T) {
            const int2 p = enc[k];
            atomicOr(&bits[(p.x - so) >> 5], 1u << ((p.x - so) & 31));
            atomicOr(&bits[(p.y - so) >> 5], 1u << ((p.y - so) & 31));
        }
        __syncthreads();
        for (int k = t; k < nw; k += T) wpre[k] = __popc(ld_u32(&bits[k]));
        __syncthreads();
        const int nu = block_scan_excl(wpre, nw, tmp);
        for (int k = t; k < nw; k += T) {
            unsigned w = ld_u32(&bits[k]);
            int r = wpre[k];
            while (w) {
                uq[r++] = so + (k << 5) + __ffs(w) - 1;
                w &= w - 1u;
            }
        }
        for (int k = t; k < nu; k += T) lab[k] = k;
        __syncthreads();
        // union-find with union by minimum: every component ends rooted at
        // its smallest rank whatever the order of the links
        for (int k = t; k < ne; k += T) {
            const int2 p = enc[k];
            const int bx = p.x - so, by = p.y - so;
            int x = wpre[bx >> 5] + __popc(ld_u32(&bits[bx >> 5]) & ((1u << (bx & 31)) - 1u));
            int y = wpre[by >> 5] + __popc(ld_u32(&bits[by >> 5]) & ((1u << (by & 31)) - 1u));
            for (;;) {
                for (int px; (px = ld_i32(&lab[x])) != x;) x = px;
                for (int py; (py = ld_i32(&lab[y])) != y;) y = py;
                if (x == y) break;
                if (x > y) {
                    const int w = x;
                    x = y;
                    y = w;
                }
                const int old = atomicCAS(&lab[y], y, x);
                if (old == y) break;
                y = old;
            }
        }
        __syncthreads();
        for (int k = t; k < nu; k += T) {
            int x = k;
            for (int px; (px = ld_i32(&lab[x])) != x;) x = px;
            root[k] = x;
        }
        __syncthreads();
        // roots numbered in ascending order: lab[r] = set id of root r
        for (int k = t; k < nu; k += T) lab[k] = root[k] == k ? 1 : 0;
        __syncthreads();
        const int nsets = block_scan_excl(lab, nu, tmp);
        // Sec. 2.3, after the steps: a set holding two planets makes the
        // whole system one set with r_crit infinite (as in k_sets); the
        // planet counts use the key space, which holds nothing yet
        if (a.planet_mass > 0.0) {
            int *pc = reinterpret_cast<int *>(key);
            for (int k = t; k < nsets; k += T) pc[k] = 0;
            if (t == 0) s_whole = 0;
            __syncthreads();
            for (int k = t; k < nu; k += T)
                if (d.m[uq[k]] >= a.planet_mass && atomicAdd(&pc[lab[root[k]]], 1) >= 1) s_whole = 1;
            __syncthreads();
            if (s_whole) {
                if (t == 0) {
                    base_set = (int)atomicAdd(&d.ctr[C_NSETS], 1ull);
                    base_mem = (int)atomicAdd(&d.ctr[C_NU], (unsigned long long)nsb);
                }
                __syncthreads();
                const int bs = base_set, bm = base_mem;
                for (int k = t; k < nsb; k += T) d.set_mem[bm + k] = so + k;
                if (t == 0) {
                    d.set_start[bs] = bm;
                    d.set_count[bs] = nsb;
                    d.set_rc[bs] = INFINITY;
                    if (nsb <= kWaveMax)
                        d.set_list[(int)atomicAdd(&d.ctr[C_NSMALL], 1ull)] = bs;
                    else
                        d.set_list[d.setcap - 1 - (int)atomicAdd(&d.ctr[C_NBIG], 1ull)] = bs;
                    if (nsb > kCoopMin) atomicAdd(&d.ctr[C_NGRID], 1ull);
                    atomicMax(&d.ctr[C_MAXSET], (unsigned long long)nsb);
                    atomicAdd(&d.ctr[C_TENC], (unsigned long long)ne);
                    atomicAdd(&d.ctr[C_WHOLE], 1ull);
                    atomicAdd(&d.ctr[C_TBIGSYS], 1ull);
                }
                __syncthreads();
                return;
            }
        }
        // members sorted by (root rank, rank)
        const int u2 = (int)gs_pow2(nu);
        for (int k = t; k < u2; k += T)
            key[k] = k < nu ? (((unsigned long long)root[k] << 32) | (unsigned)k) : ~0ull;
        __syncthreads();
        for (int kk = 2; kk <= u2; kk <<= 1)
            for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                for (int i = t; i < u2; i += T) {
                    const int ixj = i ^ jj;
                    if (ixj > i) {
                        const unsigned long long x = key[i], y = key[ixj];
                        const bool asc = (i & kk) == 0;
                        if ((x > y) == asc) {
                            key[i] = y;
                            key[ixj] = x;
                        }
                    }
                }
                __syncthreads();
            }
        if (t == 0) {
            base_set = (int)atomicAdd(&d.ctr[C_NSETS], (unsigned long long)nsets);
            base_mem = (int)atomicAdd(&d.ctr[C_NU], (unsigned long long)nu);
        }
        __syncthreads();
        const int bs = base_set, bm = base_mem;
        int *ls = root;   // local start of each set (the roots now ride in the keys)
        for (int k = t; k < nu; k += T) {
            const unsigned long long kv = key[k];
            const int rt = (int)(kv >> 32);
            d.set_mem[bm + k] = uq[(int)(kv & 0xffffffffull)];
            if (k == 0 || (int)(key[k - 1] >> 32) != rt) {
                const int sid = lab[rt];
                d.set_start[bs + sid] = bm + k;
                ls[sid] = k;
            }
        }
        __syncthreads();
        // r_crit = a_H max_{i in S} h_i a_i: maxima of the bit patterns
        // (non-negative doubles order as integers), in the space of uq
        unsigned long long *rcb = reinterpret_cast<unsigned long long *>(uq);
        for (int k = t; k < nsets; k += T) rcb[k] = 0ull;
        __syncthreads();
        for (int k = t; k < nu; k += T) {
            const int i = d.set_mem[bm + k];
            const double rh = d.h[i] * d.A[i];
            atomicMax(&rcb[lab[(int)(key[k] >> 32)]], (unsigned long long)__double_as_longlong(rh));
        }
        __syncthreads();
        // set sizes and the Hermite work lists (small sets from the front,
        // larger ones from the back), places from two scans
        int *smallf = lab;                                // root ids are done with
        int *bigf = reinterpret_cast<int *>(key);         // so are the keys
        int big = 0;
        for (int sid = t; sid < nsets; sid += T) {
            const unsigned long long rb =
                __hip_atomic_load(&rcb[sid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            d.set_rc[bs + sid] = a.aH * __longlong_as_double((long long)rb);
            const int n = (sid + 1 < nsets ? ls[sid + 1] : nu) - ls[sid];
            d.set_count[bs + sid] = n;
            big = max(big, n);
            if (n > kCoopMin) atomicAdd(&d.ctr[C_NGRID], 1ull);
            smallf[sid] = n <= kWaveMax ? 1 : 0;
            bigf[sid] = n <= kWaveMax ? 0 : 1;
        }
        __syncthreads();
        const int nsm = block_scan_excl(smallf, nsets, tmp);
        const int nbg = block_scan_excl(bigf, nsets, tmp);
        if (t == 0) {
            base_set = (int)atomicAdd(&d.ctr[C_NSMALL], (unsigned long long)nsm);
            base_mem = (int)atomicAdd(&d.ctr[C_NBIG], (unsigned long long)nbg);
        }
        __syncthreads();
        for (int sid = t; sid < nsets; sid += T) {
            const int n = (sid + 1 < nsets ? ls[sid + 1] : nu) - ls[sid];
            if (n <= kWaveMax)
                d.set_list[base_set + smallf[sid]] = bs + sid;
            else
                d.set_list[d.setcap - 1 - (base_mem + bigf[sid])] = bs + sid;
        }
        note_max_set(&d.ctr[C_MAXSET], (unsigned)big);
        if (t == 0) {
            atomicAdd(&d.ctr[C_TENC], (unsigned long long)ne);
            atomicAdd(&d.ctr[C_TBIGSYS], 1ull);
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------------
// Sec. 2.1 transition function and Sec. 2.2 / 2.3 set kernels
// ------------------------------------------------------------------------
// sin and cos of x in [0, pi/4] from their Taylor series (Horner in x^2;
// the first omitted terms are below 1e-19 there)
__device__ __forceinline__ double inv_factorial(int n)
{
    double f = 1.0;
    for (int k = 2; k <= n; ++k) f *= (double)k;
    return 1.0 / f;
}

__device__ __forceinline__ void sincos_quarter(double x, double &sn, double &cs)
{
    const double z = x * x;
    double ps = inv_factorial(17);
    ps = fma(ps, z, -inv_factorial(15));
    ps = fma(ps, z, inv_factorial(13));
    ps = fma(ps, z, -inv_factorial(11));
    ps = fma(ps, z, inv_factorial(9));
    ps = fma(ps, z, -inv_factorial(7));
    ps = fma(ps, z, inv_factorial(5));
    ps = fma(ps, z, -inv_factorial(3));
    sn = fma(ps * z, x, x);
    double pc = inv_factorial(18);
    pc = fma(pc, z, -inv_factorial(16));
    pc = fma(pc, z, inv_factorial(14));
    pc = fma(pc, z, -inv_factorial(12));
    pc = fma(pc, z, inv_factorial(10));
    pc = fma(pc, z, -inv_factorial(8));
    pc = fma(pc, z, inv_factorial(6));
    pc = fma(pc, z, -inv_factorial(4));
    pc = fma(pc, z, 0.5);
    cs = fma(-pc, z, 1.0);
}

// per-set constants of the transition function: y = c1 s - 0.1 with
// c1 = 1.1 / r_crit, K' = wc cos(pi y / 2), K'' = -wc^2 sin(pi y / 2)
struct TransConst {
    double rc2, c1, wc, wc2;
};

__device__ __forceinline__ TransConst trans_const(double rc)
{
    TransConst t;
    t.rc2 = rc * rc;
    t.c1 = 1.1 / rc;
    t.wc = (kPi / 2.0) * t.c1;
    t.wc2 = t.wc * t.wc;
    return t;
}

// K(y) = sin(pi y / 2) on 0 < y < 1 (0 below, 1 above) and its first two
// derivatives in s.  Above y = 1/2 the complement is used,
// sin(pi y / 2) = cos(pi (1 - y) / 2), so the series only ever sees
// arguments in [0, pi/4].
__device__ __forceinline__ void transition(double s, const TransConst &tc, double &K, double &Kp,
                                           double &Kpp)
{
    const double y = fma(s, tc.c1, -0.1);
    if (y <= 0.0) {
        K = 0.0; Kp = 0.0; Kpp = 0.0;
    } else if (y >= 1.0) {
        K = 1.0; Kp = 0.0; Kpp = 0.0;
    } else {
        const bool lo = y <= 0.5;
        double sn, cs;
        sincos_quarter((kPi / 2.0) * (lo ? y : 1.0 - y), sn, cs);
        const double sk = lo ? sn : cs, ck = lo ? cs : sn;
        K = sk;
        Kp = tc.wc * ck;
        Kpp = -tc.wc2 * sk;
    }
}

// 1/s and s from s^2 > 0: the hardware reciprocal square root y0 refined
// by the binomial series, 1/s = y0 (1 - e)^(-1/2) with e = 1 - s^2 y0^2
__device__ __forceinline__ void inv_dist(double s2, double &s, double &is)
{
    const double y0 = __builtin_amdgcn_rsq(s2);
    const double e = fma(-s2, y0 * y0, 1.0);
    is = y0 * fma(e, fma(e, 0.375, 0.5), 1.0);
    s = s2 * is;
}

struct HermArgs {
    Dev d;
    double tau, G, epsH, eta, eta_s;
    int max_substeps;
    unsigned long long *rec = nullptr;   // workgroup records (profiling), else null
    unsigned *bar = nullptr;     // grid barrier: [0] arrivals (cumulative), [1] generation, [2] abort
    double *hpart = nullptr;     // [2][gridDim] per-workgroup step minima of the grid sets
};


constexpr int kHermLds = kHermThreads;   // members of one set staged in LDS

// member scratch layout: field f of member slot k at hw[f * memcap + k]
// HS..HS+6: staging of sets too large for LDS (x y z u v w m; during a
// substep the predicted state)
enum { HX = 0, HU = 3, HA = 6, HJ = 9, HS = 12, HFIELDS = 19 };

__device__ __forceinline__ double &hw_at(const Dev &d, int f, int k)
{
    return d.hw[(long long)f * d.memcap + k];
}

struct SetLds {
    double *x, *y, *z, *u, *v, *w, *m;
};

// One level of the sums over aligned lane groups: every lane adds the value
// of its partner in the next larger group.  Within a row of 16 the
// partners come through DPP (quad_perm [1,0,3,2] and [2,3,0,1]: the other
// lane of the pair and of the quad; row_half_mirror and row_mirror: a lane
// of the other quad of the half row, of the other half of the row), which
// costs a VALU move instead of an LDS permute; rows exchange through
// __shfl_xor.  Both partners add the same two values, so every lane of a
// group ends with the same sum.
template <int LEVEL>
__device__ __forceinline__ double group_partner(double v)
{
    if constexpr (LEVEL == 0) return dpp_f64<0xB1>(v);
    else if constexpr (LEVEL == 1) return dpp_f64<0x4E>(v);
    else if constexpr (LEVEL == 2) return dpp_f64<0x141>(v);
    else if constexpr (LEVEL == 3) return dpp_f64<0x140>(v);
    else return __shfl_xor(v, LEVEL == 4 ? 16 : 32, 64);
}

// one level for N values at once: all N partners are moved before any is
// added, so the moves' latencies overlap
template <int LEVEL, int N>
__device__ __forceinline__ void group_level(double *const (&v)[N], int L)
{
    if (L < (2 << LEVEL)) return;
    double p[N];
#pragma unroll
    for (int q = 0; q < N; ++q) p[q] = group_partner<LEVEL>(*v[q]);
#pragma unroll
    for (int q = 0; q < N; ++q) *v[q] += p[q];
}

// sums over the L lanes (a power of two <= 64, wave-uniform) of each
// aligned lane group, of N values
template <int N>
__device__ __forceinline__ void group_sums(double *const (&v)[N], int L)
{
    group_level<0>(v, L);
    group_level<1>(v, L);
    group_level<2>(v, L);
    group_level<3>(v, L);
    group_level<4>(v, L);
    group_level<5>(v, L);
}

__device__ __forceinline__ void group_sum3(double a[3], int L)
{
    double *const v[3] = {&a[0], &a[1], &a[2]};
    group_sums<3>(v, L);
}

__device__ __forceinline__ void group_sum6(double a[3], double b[3], int L)
{
    double *const v[6] = {&a[0], &a[1], &a[2], &b[0], &b[1], &b[2]};
    group_sums<6>(v, L);
}

// partial W-weighted in-set acceleration on member a from members
// b = l, l+L, ... (unsoftened; Sec. 2.3 steps 5 and 7)
__device__ void set_pair_acc(const SetLds &S, int n, int a, int l, int L, double G, double rc,
                             double out[3])
{
    const TransConst tc = trans_const(rc);
    const double xi = S.x[a], yi = S.y[a], zi = S.z[a];
    out[0] = out[1] = out[2] = 0.0;
    // the pairs inside r_crit marked first and only those taken, in the
    // same order (as herm_pairs below)
    for (int b0 = l; b0 < n; b0 += 32 * L) {
        unsigned in = 0u;
        for (int t = 0; t < 32; ++t) {
            const int b = b0 + t * L;
            if (b >= n) break;
            const double dd0 = S.x[b] - xi, dd1 = S.y[b] - yi, dd2 = S.z[b] - zi;
            const double s2 = fma(dd2, dd2, fma(dd1, dd1, dd0 * dd0));
            // beyond r_crit K = 1, K' = 0: W = 0, the pair adds exactly zero
            if (b != a && !(s2 == 0.0 || s2 >= tc.rc2)) in |= 1u << t;
        }
        while (in) {
            const int b = b0 + __builtin_ctz(in) * L;
            in &= in - 1u;
            const double dd0 = S.x[b] - xi, dd1 = S.y[b] - yi, dd2 = S.z[b] - zi;
            const double s2 = fma(dd2, dd2, fma(dd1, dd1, dd0 * dd0));
            double s, is;
            inv_dist(s2, s, is);
            double K, Kp, Kpp;
            transition(s, tc, K, Kp, Kpp);
            const double W = fma(s, Kp, 1.0 - K);
            const double fct = G * S.m[b] * W * (is * is * is);
            out[0] = fma(fct, dd0, out[0]);
            out[1] = fma(fct, dd1, out[1]);
            out[2] = fma(fct, dd2, out[2]);
        }
    }
}

// partial pair acceleration and jerk of H'_Kep (Sec. 2.2) on member a from
// members b = l, l+L, ... at the staged state.  A pair beyond r_crit adds
// exactly zero and is skipped; but a wave runs the pair term whenever any of
// its lanes has a pair inside, and in a set of a hundred members a lane's
// 27 pairs hold about six inside.  So each lane first marks its pairs
// inside (32 at a time, a bit each) and then takes only those, in the same
// ascending order and with the same arithmetic as a loop over all of them.
__device__ void herm_pairs(const SetLds &S, int n, int a, int l, int L, double G, double rc,
                           double eps, double acc[3], double jrk[3])
{
    const TransConst tc = trans_const(rc);
    const double X0 = S.x[a], X1 = S.y[a], X2 = S.z[a];
    const double U0 = S.u[a], U1 = S.v[a], U2 = S.w[a];
    const double eps2 = eps * eps;
    for (int c = 0; c < 3; ++c) acc[c] = jrk[c] = 0.0;
    for (int b0 = l; b0 < n; b0 += 32 * L) {
        unsigned inside = 0u;
        for (int t = 0; t < 32; ++t) {
            const int b = b0 + t * L;
            if (b >= n) break;
            const double d0 = S.x[b] - X0, d1 = S.y[b] - X1, d2 = S.z[b] - X2;
            const double s2 = fma(d2, d2, fma(d1, d1, fma(d0, d0, eps2)));
            // beyond r_crit W = 0 and K'' = 0: the pair adds exactly zero
            if (b != a && !(s2 == 0.0 || s2 >= tc.rc2)) inside |= 1u << t;
        }
        // dot products and sums as explicit fused multiply-adds (the
        // library contracts nothing by itself)
        while (inside) {
            const int b = b0 + __builtin_ctz(inside) * L;
            inside &= inside - 1u;
            const double dd[3] = {S.x[b] - X0, S.y[b] - X1, S.z[b] - X2};
            const double w[3] = {S.u[b] - U0, S.v[b] - U1, S.w[b] - U2};
            const double s2 = fma(dd[2], dd[2], fma(dd[1], dd[1], fma(dd[0], dd[0], eps2)));
            double s, is;
            inv_dist(s2, s, is);
            const double is2 = is * is;
            double K, Kp, Kpp;
            transition(s, tc, K, Kp, Kpp);
            const double W = fma(s, Kp, 1.0 - K);
            const double gm = G * S.m[b] * (is2 * is);
            const double gmW = gm * W;
            const double dw = fma(dd[2], w[2], fma(dd[1], w[1], dd[0] * w[0]));
            const double c3 = 3.0 * dw * is2;
            const double dK = dw * Kpp;
            for (int c = 0; c < 3; ++c) {
                acc[c] = fma(gmW, dd[c], acc[c]);
                jrk[c] = fma(gm, fma(dK, dd[c], fma(-c3, dd[c], w[c]) * W), jrk[c]);
            }
        }
    }
}

// central (star) part, added after the pair sums
__device__ __forceinline__ void herm_central(const double X[3], const double U[3], double mu,
                                             double acc[3], double jrk[3])
{
    const double r2 = X[0] * X[0] + X[1] * X[1] + X[2] * X[2];
    const double r = sqrt(r2);
    const double ir3 = 1.0 / (r2 * r);
    const double ir5 = ir3 / r2;
    const double xv = X[0] * U[0] + X[1] * U[1] + X[2] * U[2];
    for (int c = 0; c < 3; ++c) {
        acc[c] += -mu * X[c] * ir3;
        jrk[c] += -mu * (U[c] * ir3 - 3.0 * xv * X[c] * ir5);
    }
}

// powers of one signed substep hs of the Hermite scheme: the Taylor
// factors hs^k / k! of the predictor and corrector and 1/hs^2, 1/hs^3 of
// the interpolated second and third derivatives (one division per substep)
struct HermStep {
    double hs, c2, c3, c4, c5, i2, i3;
};

__device__ __forceinline__ HermStep herm_step(double hs)
{
    HermStep k;
    const double h2 = hs * hs, h3 = h2 * hs;
    k.hs = hs;
    k.c2 = h2 * 0.5;
    k.c3 = h3 * (1.0 / 6.0);
    k.c4 = h2 * h2 * (1.0 / 24.0);
    k.c5 = h3 * h2 * (1.0 / 120.0);
    const double ih = 1.0 / hs;
    k.i2 = ih * ih;
    k.i3 = k.i2 * ih;
    return k;
}

// predictor: Taylor series of x to the jerk term, of u to the jerk term
__device__ __forceinline__ void herm_predict(const HermStep &k, const double X[3], const double U[3],
                                             const double A[3], const double J[3], double xp[3],
                                             double up[3])
{
    for (int c = 0; c < 3; ++c) {
        xp[c] = X[c] + k.hs * U[c] + k.c2 * A[c] + k.c3 * J[c];
        up[c] = U[c] + k.hs * A[c] + k.c2 * J[c];
    }
}

// corrector: second and third derivatives from (A, J) at the start and
// (a1, j1) at the predicted end, the fourth- and fifth-order terms added to
// the prediction; (A, J) become (a1, j1).  Returns the member's next step
// from the time-step criterion on |a|, |j|, |a''|, |a'''| at the end.
__device__ __forceinline__ double herm_correct(const HermStep &k, double eta, const double a1[3],
                                               const double j1[3], const double xp[3],
                                               const double up[3], double X[3], double U[3],
                                               double A[3], double J[3])
{
    double A2e[3], A3v[3];
    for (int c = 0; c < 3; ++c) {
        const double da = A[c] - a1[c];
        const double A2 = (-6.0 * da - k.hs * (4.0 * J[c] + 2.0 * j1[c])) * k.i2;
        const double A3 = (12.0 * da + 6.0 * k.hs * (J[c] + j1[c])) * k.i3;
        X[c] = xp[c] + A2 * k.c4 + A3 * k.c5;
        U[c] = up[c] + A2 * k.c3 + A3 * k.c4;
        A[c] = a1[c];
        J[c] = j1[c];
        A2e[c] = A2 + k.hs * A3;
        A3v[c] = A3;
    }
    const double na = dnorm3(a1[0], a1[1], a1[2]), nj = dnorm3(j1[0], j1[1], j1[2]);
    const double n2 = dnorm3(A2e[0], A2e[1], A2e[2]);
    const double n3 = dnorm3(A3v[0], A3v[1], A3v[2]);
    return sqrt(eta * (na * n2 + nj * nj) / (nj * n3 + n2 * n2));
}

// minimum over the wave (fmin: NaN only where every lane has NaN): the
// row minima through the DPP levels of the group sums, then the four rows
// read into scalar registers
__device__ __forceinline__ double wave_min(double v)
{
    v = fmin(v, group_partner<0>(v));
    v = fmin(v, group_partner<1>(v));
    v = fmin(v, group_partner<2>(v));
    v = fmin(v, group_partner<3>(v));
    return fmin(fmin(readlane_f64(v, 0), readlane_f64(v, 16)),
                fmin(readlane_f64(v, 32), readlane_f64(v, 48)));
}

// a value equal on all lanes (a wave reduction) moved to scalar registers,
// so the loops and branches that test it are uniform to the compiler too
__device__ __forceinline__ double wave_uniform(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// One set of at most kWaveMax members on one wave: member k on lanes
// [k L, k L + L) (L = largest power of two with L n <= 64), its state in
// registers of those lanes, the staged set state in the wave's own LDS
// slice.  Same steps as the workgroup version below (corrections at q0
// and q1, PEC Hermite with one shared step), with no global memory traffic
// inside the substep loop.
__device__ void hermite_set_wave(const HermArgs &a, int sidx, const SetLds &S, int lane,
                                 int &nsub_out, int &fail_out)
{
    const Dev &d = a.d;
    const int b0 = __builtin_amdgcn_readfirstlane(d.set_start[sidx]);
    const int n = __builtin_amdgcn_readfirstlane(d.set_count[sidx]);
    const double rc = d.set_rc[sidx];
    nsub_out = 0;
    fail_out = 0;
    if (n < 1 || n > kWaveMax) return;   // the set kernel lists 1..kWaveMax members here
    int L = 1;
    while (2 * L * n <= kHermWave) L <<= 1;
    const int k = lane / L, l = lane % L;
    const bool mine = k < n;
    const int kk = mine ? k : 0;   // idle lanes shadow member 0; their results are dropped
    const int i = d.set_mem[b0 + kk];
    const double mu = a.G * d.sys_m0[d.body_sys[i]];
    const double half = a.tau / 2.0;
    double X[3] = {d.x0[i], d.y0[i], d.z0[i]};
    if (mine && l == 0) {
        S.x[k] = X[0];
        S.y[k] = X[1];
        S.z[k] = X[2];
        S.m[k] = d.m[i];
    }
    wave_lds_sync();
    // step 5: v0 -= tau/2 * sum W-weighted in-set forces at q0
    double U[3], A[3], J[3];
    {
        double acc[3];
        set_pair_acc(S, n, kk, l, L, a.G, rc, acc);
        group_sum3(acc, L);
        U[0] = d.vx0[i] - half * acc[0];
        U[1] = d.vy0[i] - half * acc[1];
        U[2] = d.vz0[i] - half * acc[2];
    }
    if (mine && l == 0) {
        S.u[k] = U[0];
        S.v[k] = U[1];
        S.w[k] = U[2];
    }
    wave_lds_sync();
    // initial force and first step
    double hloc = INFINITY;
    herm_pairs(S, n, kk, l, L, a.G, rc, a.epsH, A, J);
    group_sum6(A, J, L);
    herm_central(X, U, mu, A, J);
    {
        const double hb = a.eta_s * dnorm3(A[0], A[1], A[2]) / dnorm3(J[0], J[1], J[2]);
        if (mine && hb > 0.0) hloc = hb;
    }
    double h = wave_uniform(wave_min(hloc));
    const double sgn = a.tau >= 0.0 ? 1.0 : -1.0;
    const double T = fabs(a.tau);
    double tt = 0.0;
    int nsub = 0, fail = 0;
    bool last = (T == 0.0);
    while (!last) {
        if (nsub >= a.max_substeps) {
            fail = 1;
            break;
        }
        if (!(h > 0.0) || h >= T - tt) {
            h = T - tt;
            last = true;
        }
        const HermStep hk = herm_step(sgn * h);
        double xp[3], up[3];
        herm_predict(hk, X, U, A, J, xp, up);
        wave_lds_sync();   // every lane is done reading the previous state
        if (mine && l == 0) {
            S.x[k] = xp[0]; S.y[k] = xp[1]; S.z[k] = xp[2];
            S.u[k] = up[0]; S.v[k] = up[1]; S.w[k] = up[2];
        }
        wave_lds_sync();
        double a1[3], j1[3];
        herm_pairs(S, n, kk, l, L, a.G, rc, a.epsH, a1, j1);
        group_sum6(a1, j1, L);
        herm_central(xp, up, mu, a1, j1);
        const double hb = herm_correct(hk, a.eta, a1, j1, xp, up, X, U, A, J);
        tt += h;
        ++nsub;
        h = wave_uniform(wave_min((mine && hb > 0.0) ? hb : INFINITY));
    }
    // step 7: v1 -= tau/2 * W-weighted in-set forces at q1, write back
    wave_lds_sync();
    if (mine && l == 0) {
        S.x[k] = X[0];
        S.y[k] = X[1];
        S.z[k] = X[2];
    }
    wave_lds_sync();
    double acc[3];
    set_pair_acc(S, n, kk, l, L, a.G, rc, acc);
    group_sum3(acc, L);
    if (mine && l == 0) {
        d.x[i] = X[0];
        d.y[i] = X[1];
        d.z[i] = X[2];
        d.vx[i] = U[0] - half * acc[0];
        d.vy[i] = U[1] - half * acc[1];
        d.vz[i] = U[2] - half * acc[2];
    }
    wave_lds_sync();   // the slice is reused by the wave's next set
    nsub_out = nsub;
    fail_out = fail;
}

// minimum over a workgroup of NT threads: a wave minimum, then the NT / 64
// wave minima through LDS (one barrier); every thread gets the same value.
// red must not be read again before the next barrier.
template <int NT>
__device__ __forceinline__ double block_min_waves(double v, double *red)
{
    v = wave_min(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int w = 1; w < NT / 64; ++w) r = fmin(r, red[w]);
    return wave_uniform(r);
}

// One set of kWaveMax < n <= kHermThreads members on one workgroup: member
// k on the L lanes of group k (L the largest power of two <= 64 with
// L n <= kHermThreads, so no group holds two members), its state (X, U, A,
// J) in registers of those lanes, the staged set in LDS.  Same steps and
// arithmetic as hermite_set_wave; per substep three barriers: the staged
// prediction written, read, and the step-size minimum.
__device__ void hermite_set_block(const HermArgs &a, int sidx, const SetLds &S, double *red,
                                  int &nsub_out, int &fail_out)
{
    const Dev &d = a.d;
    const int t = threadIdx.x;
    const int b0 = __builtin_amdgcn_readfirstlane(d.set_start[sidx]);
    const int n = __builtin_amdgcn_readfirstlane(d.set_count[sidx]);
    const double rc = d.set_rc[sidx];
    int L = 1;
    while (L < 64 && 2 * L * n <= kHermThreads) L <<= 1;
    const int k = t / L, l = t % L;
    const bool mine = k < n;
    const int kk = mine ? k : 0;   // idle groups shadow member 0; their results are dropped
    const int i = d.set_mem[b0 + kk];
    const double mu = a.G * d.sys_m0[d.body_sys[i]];
    const double half = a.tau / 2.0;
    double X[3] = {d.x0[i], d.y0[i], d.z0[i]};
    if (mine && l == 0) {
        S.x[k] = X[0];
        S.y[k] = X[1];
        S.z[k] = X[2];
        S.m[k] = d.m[i];
    }
    __syncthreads();
    // step 5: v0 -= tau/2 * sum W-weighted in-set forces at q0
    double U[3], A[3], J[3];
    {
        double acc[3];
        set_pair_acc(S, n, kk, l, L, a.G, rc, acc);
        group_sum3(acc, L);
        U[0] = d.vx0[i] - half * acc[0];
        U[1] = d.vy0[i] - half * acc[1];
        U[2] = d.vz0[i] - half * acc[2];
    }
    if (mine && l == 0) {
        S.u[k] = U[0];
        S.v[k] = U[1];
        S.w[k] = U[2];
    }
    __syncthreads();
    // initial force and first step
    herm_pairs(S, n, kk, l, L, a.G, rc, a.epsH, A, J);
    group_sum6(A, J, L);
    herm_central(X, U, mu, A, J);
    double hloc = INFINITY;
    {
        const double hb = a.eta_s * dnorm3(A[0], A[1], A[2]) / dnorm3(J[0], J[1], J[2]);
        if (mine && hb > 0.0) hloc = hb;
    }
    double h = block_min_waves<kHermThreads>(hloc, red);
    const double sgn = a.tau >= 0.0 ? 1.0 : -1.0;
    const double T = fabs(a.tau);
    double tt = 0.0;
    int nsub = 0, fail = 0;
    bool last = (T == 0.0);
    while (!last) {
        if (nsub >= a.max_substeps) {
            fail = 1;
            break;
        }
        if (!(h > 0.0) || h >= T - tt) {
            h = T - tt;
            last = true;
        }
        const HermStep hk = herm_step(sgn * h);
        double xp[3], up[3];
        herm_predict(hk, X, U, A, J, xp, up);
        __syncthreads();   // every lane is done reading the previous state (and red)
        if (mine && l == 0) {
            S.x[k] = xp[0]; S.y[k] = xp[1]; S.z[k] = xp[2];
            S.u[k] = up[0]; S.v[k] = up[1]; S.w[k] = up[2];
        }
        __syncthreads();
        double a1[3], j1[3];
        herm_pairs(S, n, kk, l, L, a.G, rc, a.epsH, a1, j1);
        group_sum6(a1, j1, L);
        herm_central(xp, up, mu, a1, j1);
        const double hb = herm_correct(hk, a.eta, a1, j1, xp, up, X, U, A, J);
        tt += h;
        ++nsub;
        h = block_min_waves<kHermThreads>((mine && hb > 0.0) ? hb : INFINITY, red);
    }
    // step 7: v1 -= tau/2 * W-weighted in-set forces at q1, write back
    __syncthreads();
    if (mine && l == 0) {
        S.x[k] = X[0];
        S.y[k] = X[1];
        S.z[k] = X[2];
    }
    __syncthreads();
    double acc[3];
    set_pair_acc(S, n, kk, l, L, a.G, rc, acc);
    group_sum3(acc, L);
    if (mine && l == 0) {
        d.x[i] = X[0];
        d.y[i] = X[1];
        d.z[i] = X[2];
        d.vx[i] = U[0] - half * acc[0];
        d.vy[i] = U[1] - half * acc[1];
        d.vz[i] = U[2] - half * acc[2];
    }
    __syncthreads();   // the staging arrays are reused by the next set
    nsub_out = nsub;
    fail_out = fail;
}

template <int NT>
__device__ void hermite_grid_sets(const HermArgs &a, double *red, int *s_ok);

// Sec. 2.3 steps 5-7 for every set.  Sets of more than kWaveMax and at most
// kCoopMin members first, one workgroup each (hermite_set_block: the set
// staged in LDS, each member's state in the registers of its lane group);
// then the small sets, one wave each (hermite_set_wave), both in a fixed
// assignment; every set is integrated on its own, so the assignment changes
// nothing in the results.  Then, when the step has any, the sets above
// kCoopMin members on the whole grid, one after the other
// (hermite_grid_sets): from about 250 members its two grid barriers per
// substep cost less than the n^2 / 512 pair terms per lane of one
// workgroup.  The grid is one workgroup per compute unit, all resident
// (checked when the context is created), and the sets' count is known to
// every workgroup from the set kernel, so a step without such sets has no
// grid barrier at all.
__global__ __launch_bounds__(kHermThreads) void k_hermite(HermArgs a)
{
    static_assert(kCoopMin <= kHermThreads && kHermThreads <= kHermLds,
                  "a workgroup set has at most one member per lane group");
    const Dev &d = a.d;
    __shared__ double s_x[kHermLds], s_y[kHermLds], s_z[kHermLds];
    __shared__ double s_u[kHermLds], s_v[kHermLds], s_w[kHermLds], s_m[kHermLds];
    __shared__ double lds[kHermThreads / 64];
    const int t = threadIdx.x;
    wg_start(a.rec);
    const int nwg = gridDim.x, wpb = kHermThreads / 64;
    if (d.ctr[C_STATUS] & S_FREEZE) return;   // a step left undone
    const int nbig = (int)d.ctr[C_NBIG];
    // Sets are assigned statically, with no work-queue counter: thousands
    // of atomics on one counter congest its L2 channel, and every wave with
    // a lane whose load maps there waits for them.  Workgroup b takes the
    // larger sets b, b + grid, ... (at most one each unless there are more
    // larger sets than workgroups).
    int nsub_b = 0, fail_b = 0;   // statistics of thread 0, added after the loop
    for (int q = blockIdx.x; q < nbig; q += nwg) {
        const int sidx = d.set_list[d.setcap - 1 - q];
        if (d.set_count[sidx] > kCoopMin) continue;   // the grid phase takes it
        int nsub, fail;
        hermite_set_block(a, sidx, SetLds{s_x, s_y, s_z, s_u, s_v, s_w, s_m}, lds, nsub, fail);
        if (t == 0) {
            nsub_b += nsub;
            fail_b |= fail;
        }
    }
    if (t == 0 && nsub_b > 0) {
        atomicAdd(&d.ctr[C_SUB], (unsigned long long)nsub_b);
        atomicAdd(&d.ctr[C_TSUB], (unsigned long long)nsub_b);
    }
    if (t == 0 && fail_b) latch(d.ctr, S_HERMITE);
    // small sets, one wave each, in the wave's slice of the staging arrays:
    // round robin over the waves, those of the workgroups without a larger
    // set first
    const int w = __builtin_amdgcn_readfirstlane(t >> 6), lane = t & 63;
    const SetLds S = {s_x + w * kWaveMax, s_y + w * kWaveMax, s_z + w * kWaveMax,
                      s_u + w * kWaveMax, s_v + w * kWaveMax, s_w + w * kWaveMax,
                      s_m + w * kWaveMax};
    const int nsmall = (int)d.ctr[C_NSMALL];
    const int busy = min(nbig, nwg);
    const int rank = ((int)blockIdx.x - busy + nwg) % nwg;
    // The loop runs on scalar values only and keeps the statistics out of
    // its body: lane-0 branches at both ends of a loop body can be merged
    // by the compiler across the back edge, which splits the wave.
    int nsub_w = 0, fail_w = 0;
    for (int q = rank * wpb + w; q < nsmall; q += nwg * wpb) {
        int nsub, fail;
        hermite_set_wave(a, d.set_list[q], S, lane, nsub, fail);
        nsub_w += nsub;
        fail_w |= fail;
    }
    if (lane == 0 && nsub_w > 0) {
        atomicAdd(&d.ctr[C_SUB], (unsigned long long)nsub_w);
        atomicAdd(&d.ctr[C_TSUB], (unsigned long long)nsub_w);
    }
    if (lane == 0 && fail_w) latch(d.ctr, S_HERMITE);
    if (d.ctr[C_NGRID] != 0) {
        __shared__ int s_ok;
        hermite_grid_sets<kHermThreads>(a, lds, &s_ok);
    }
    wg_finish(a.rec);
}


// ------------------------------------------------------------------------
// Sets of more than kCoopMin members (the giant sets a nearly parabolic
// body makes through its Hill radius, or a whole system): the same steps
// as hermite_set_block, spread over the whole grid of k_hermite.  Member k belongs to lane group
// k mod NG (L lanes, NG = grid lanes / L); its pair sums run over the staged
// set in global memory; grid-wide barriers separate the phases of a
// substep, and the step size is the minimum of per-block partial minima
// read by every block (double-buffered by substep parity), so all blocks
// take the same sequence of steps.  The barrier waits are bounded: a wait
// that runs out raises an abort flag that every block polls, every block
// leaves, and the Hermite status bit is latched.
// ------------------------------------------------------------------------

// longest wait at one barrier before giving up, in ticks of the 100 MHz
// real-time counter (10 s: far beyond any phase of a legitimate set)
constexpr unsigned long long kGridWaitTicks = 1000000000ull;

// Grid-wide barrier over the arrivals counter (cumulative, so barrier p
// completes at gridDim * p arrivals) and a generation word.  The block
// barrier first waits for the stores of all the block's waves (they are in
// L2 then); one thread per block then fences at agent scope (L2 written back)
// before it arrives and again after the wait (this CU's L1 and this XCD's
// L2 invalidated, for every wave of the block), so the stores of all blocks
// before the barrier are visible to all blocks after it.  An agent-scope
// fence in every wave instead costs thousands of whole-L2 write-backs and
// invalidations per barrier.  Returns false when the wait ran out or
// another block aborted.
__device__ bool grid_sync(unsigned *bar, unsigned &phase, int *s_ok)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        int ok = 1;
        const unsigned target = phase + 1;
        const unsigned prev =
            __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev + 1 == gridDim.x * target) {
            __hip_atomic_store(&bar[1], target, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
            // relaxed polls (an acquire load would invalidate the caches on
            // every poll); the fence after the wait is the acquire
            while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                    __builtin_amdgcn_s_memrealtime() - t0 > kGridWaitTicks) {
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        if (!ok) __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        *s_ok = ok;
        phase = target;
    }
    __syncthreads();
    return __builtin_amdgcn_readfirstlane(*s_ok) != 0;
}

// a failed barrier ends the grid phase in this block (the others follow
// through the abort flag) and reports the set as failed
#define GSYNC()                                           \
    do {                                                  \
        if (!grid_sync(a.bar, phase, s_ok)) {             \
            if (threadIdx.x == 0) latch(d.ctr, S_HERMITE); \
            return;                                       \
        }                                                 \
    } while (0)

template <int NT>
__device__ void hermite_grid_sets(const HermArgs &a, double *red, int *s_ok)
{
    const Dev &d = a.d;
    const int t = threadIdx.x;
    const int gtid = blockIdx.x * NT + t;
    const int nthr = gridDim.x * NT;
    const long long fs = d.memcap;
    unsigned phase = 0;
    int par = 0;
    const int nbig = (int)d.ctr[C_NBIG];
    for (int q = 0; q < nbig; ++q) {
        const int sidx = d.set_list[d.setcap - 1 - q];
        const int n = d.set_count[sidx];
        if (n <= kCoopMin) continue;
        const int b0 = d.set_start[sidx];
        const double rc = d.set_rc[sidx];
        double *gs = d.hw + (long long)HS * fs + b0;
        const SetLds S{gs, gs + fs, gs + 2 * fs, gs + 3 * fs, gs + 4 * fs, gs + 5 * fs, gs + 6 * fs};
        int L = 1;
        while (L < 64 && 2 * L * n <= nthr) L <<= 1;
        const int NG = nthr / L;
        const int g = gtid / L, l = gtid % L;
        const double mu = a.G * d.sys_m0[d.body_sys[d.set_mem[b0]]];
        const double half = a.tau / 2.0;
        // stage q0 and masses
        for (int k = gtid; k < n; k += nthr) {
            const int i = d.set_mem[b0 + k];
            S.x[k] = d.x0[i];
            S.y[k] = d.y0[i];
            S.z[k] = d.z0[i];
            S.m[k] = d.m[i];
        }
        GSYNC();
        // step 5: v0 -= tau/2 * W-weighted in-set forces at q0
        for (int k0 = 0; k0 < n; k0 += NG) {
            const int k = k0 + g;
            const int kk = k < n ? k : 0;
            double acc[3];
            set_pair_acc(S, n, kk, l, L, a.G, rc, acc);
            group_sum3(acc, L);
            if (k < n && l == 0) {
                const int i = d.set_mem[b0 + k];
                hw_at(d, HX + 0, b0 + k) = S.x[k];
                hw_at(d, HX + 1, b0 + k) = S.y[k];
                hw_at(d, HX + 2, b0 + k) = S.z[k];
                hw_at(d, HU + 0, b0 + k) = d.vx0[i] - half * acc[0];
                hw_at(d, HU + 1, b0 + k) = d.vy0[i] - half * acc[1];
                hw_at(d, HU + 2, b0 + k) = d.vz0[i] - half * acc[2];
            }
        }
        GSYNC();
        for (int k = gtid; k < n; k += nthr) {
            S.u[k] = hw_at(d, HU + 0, b0 + k);
            S.v[k] = hw_at(d, HU + 1, b0 + k);
            S.w[k] = hw_at(d, HU + 2, b0 + k);
        }
        GSYNC();
        // initial force and first step
        double hloc = INFINITY;
        for (int k0 = 0; k0 < n; k0 += NG) {
            const int k = k0 + g;
            const int kk = k < n ? k : 0;
            double acc[3], jr[3];
            herm_pairs(S, n, kk, l, L, a.G, rc, a.epsH, acc, jr);
            group_sum6(acc, jr, L);
            if (k < n && l == 0) {
                const double X[3] = {S.x[k], S.y[k], S.z[k]}, U[3] = {S.u[k], S.v[k], S.w[k]};
                herm_central(X, U, mu, acc, jr);
                for (int c = 0; c < 3; ++c) {
                    hw_at(d, HA + c, b0 + k) = acc[c];
                    hw_at(d, HJ + c, b0 + k) = jr[c];
                }
                const double hb =
                    a.eta_s * dnorm3(acc[0], acc[1], acc[2]) / dnorm3(jr[0], jr[1], jr[2]);
                if (hb > 0.0 && hb < hloc) hloc = hb;
            }
        }
        {
            const double bm = block_min_waves<NT>(hloc, red);
            if (t == 0) a.hpart[par * gridDim.x + blockIdx.x] = bm;
        }
        GSYNC();
        // the step minimum over the blocks' minima: one load per thread
        double h = INFINITY;
        for (int b = t; b < (int)gridDim.x; b += NT) h = fmin(h, a.hpart[par * gridDim.x + b]);
        h = block_min_waves<NT>(h, red);
        par ^= 1;
        const double sgn = a.tau >= 0.0 ? 1.0 : -1.0;
        const double T = fabs(a.tau);
        double tt = 0.0;
        int nsub = 0, fail = 0;
        bool last = (T == 0.0);
        while (!last) {
            if (nsub >= a.max_substeps) {
                fail = 1;
                break;
            }
            if (!(h > 0.0) || h >= T - tt) {
                h = T - tt;
                last = true;
            }
            const HermStep hk = herm_step(sgn * h);
            // predict into the staged copy: every member's force reads it, the
            // corrector takes it as the prediction
            for (int k = gtid; k < n; k += nthr) {
                double X[3], U[3], A[3], J[3], xp[3], up[3];
                for (int c = 0; c < 3; ++c) {
                    X[c] = hw_at(d, HX + c, b0 + k);
                    U[c] = hw_at(d, HU + c, b0 + k);
                    A[c] = hw_at(d, HA + c, b0 + k);
                    J[c] = hw_at(d, HJ + c, b0 + k);
                }
                herm_predict(hk, X, U, A, J, xp, up);
                S.x[k] = xp[0]; S.y[k] = xp[1]; S.z[k] = xp[2];
                S.u[k] = up[0]; S.v[k] = up[1]; S.w[k] = up[2];
            }
            GSYNC();
            double hn = INFINITY;
            for (int k0 = 0; k0 < n; k0 += NG) {
                const int k = k0 + g;
                const int kk = k < n ? k : 0;
                double a1[3], j1[3];
                herm_pairs(S, n, kk, l, L, a.G, rc, a.epsH, a1, j1);
                group_sum6(a1, j1, L);
                if (k < n && l == 0) {
                    const double xp[3] = {S.x[k], S.y[k], S.z[k]}, up[3] = {S.u[k], S.v[k], S.w[k]};
                    herm_central(xp, up, mu, a1, j1);
                    double X[3], U[3], A[3], J[3];
                    for (int c = 0; c < 3; ++c) {
                        A[c] = hw_at(d, HA + c, b0 + k);
                        J[c] = hw_at(d, HJ + c, b0 + k);
                    }
                    const double hb = herm_correct(hk, a.eta, a1, j1, xp, up, X, U, A, J);
                    for (int c = 0; c < 3; ++c) {
                        hw_at(d, HX + c, b0 + k) = X[c];
                        hw_at(d, HU + c, b0 + k) = U[c];
                        hw_at(d, HA + c, b0 + k) = A[c];
                        hw_at(d, HJ + c, b0 + k) = J[c];
                    }
                    if (hb > 0.0 && hb < hn) hn = hb;
                }
            }
            {
                const double bm = block_min_waves<NT>(hn, red);
                if (t == 0) a.hpart[par * gridDim.x + blockIdx.x] = bm;
            }
            GSYNC();
            double hnext = INFINITY;
            for (int b = t; b < (int)gridDim.x; b += NT)
                hnext = fmin(hnext, a.hpart[par * gridDim.x + b]);
            hnext = block_min_waves<NT>(hnext, red);
            par ^= 1;
            tt += h;
            ++nsub;
            h = hnext;
        }
        // step 7: stage q1, v1 -= tau/2 * W-weighted in-set forces at q1
        for (int k = gtid; k < n; k += nthr) {
            S.x[k] = hw_at(d, HX + 0, b0 + k);
            S.y[k] = hw_at(d, HX + 1, b0 + k);
            S.z[k] = hw_at(d, HX + 2, b0 + k);
        }
        GSYNC();
        for (int k0 = 0; k0 < n; k0 += NG) {
            const int k = k0 + g;
            const int kk = k < n ? k : 0;
            double acc[3];
            set_pair_acc(S, n, kk, l, L, a.G, rc, acc);
            group_sum3(acc, L);
            if (k < n && l == 0) {
                const int i = d.set_mem[b0 + k];
                d.x[i] = S.x[k];
                d.y[i] = S.y[k];
                d.z[i] = S.z[k];
                d.vx[i] = hw_at(d, HU + 0, b0 + k) - half * acc[0];
                d.vy[i] = hw_at(d, HU + 1, b0 + k) - half * acc[1];
                d.vz[i] = hw_at(d, HU + 2, b0 + k) - half * acc[2];
            }
        }
        if (gtid == 0) {
            atomicAdd(&d.ctr[C_SUB], (unsigned long long)nsub);
            atomicAdd(&d.ctr[C_TSUB], (unsigned long long)nsub);
            if (fail) latch(d.ctr, S_HERMITE);
        }
        // every block is done with this set's staging before the next one
        GSYNC();
    }
}

// ------------------------------------------------------------------------
// Energy (Sec. 2: H = H_Dft + H_Kep + H_Int).  The pair sum takes every
// pair i < j of a system once, m_j / r_ij with r^-1 from the hardware
// reciprocal square root refined by the binomial series of (1 - e)^(-1/2),
// e = 1 - r^2 y0^2 (exact to FP64 rounding, as the kick's r^-3).  The
// pairs are cut into units of 128 i (two per lane: the i-block's two
// halves) x 64 j (staged in the wave's own LDS slice, so no workgroup
// barrier) over the upper triangle of every system.  Two i per lane halve
// the LDS traffic per pair: every lane reads every j of the slice, and
// with one i per lane those reads, not the arithmetic, bound the sum.  The
// units' 64 columns are dealt to the waves in equal contiguous ranges that
// may begin or end inside a unit.  A wave adds its sums per system into a
// record -- the kinetic, central-potential and momentum terms of the
// bodies whose first unit begins in its range, and the pair sum -- and
// k_energy_final adds each system's records in order (deterministic).  A
// coincident pair (r = 0, which the definition leaves out) makes a lane's
// unit sum NaN through rsq(0) = inf: that lane sums the unit again with
// every pair tested.
// ------------------------------------------------------------------------
constexpr int kERec = 6;            // kinetic, central potential, px, py, pz, pair sum
constexpr double kFarI = -1e18;     // padding lanes: far apart from padding j (kFar)

struct EnergyArgs {
    Dev d;
    double G;
    int nsys;
};

// sum over the unit's columns [c0, c1) of m_j / r for one i, every pair
// tested (r > 0, and j > i on a diagonal sub-block)
__device__ __forceinline__ double energy_cols_masked(const double *sx, const double *sy,
                                                     const double *sz, const double *sm, int c0,
                                                     int c1, double xi, double yi, double zi,
                                                     int lane, bool diag)
{
    double acc = 0.0;
    for (int k = c0; k < c1; ++k) {
        const double dx = sx[k] - xi, dy = sy[k] - yi, dz = sz[k] - zi;
        const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
        const bool keep = r2 > 0.0 && (!diag || k > lane);
        const double rk = keep ? r2 : 1.0;
        const double y0 = __builtin_amdgcn_rsq(rk);
        const double e = fma(-rk, y0 * y0, 1.0);
        const double w = fma(e, fma(e, 0.375, 0.5), 1.0);
        acc = fma(keep ? sm[k] * y0 : 0.0, w, acc);
    }
    return acc;
}

// both i of the lane over the columns [c0, c1): the first half meets the
// whole slice, the second half too (DIAG1 = false) or only j > i (the
// slice is its own 64-block, DIAG1 = true)
template <bool DIAG1>
__device__ __forceinline__ void energy_cols2(const double *sx, const double *sy, const double *sz,
                                             const double *sm, int c0, int c1, double x0,
                                             double y0, double z0, double x1, double y1,
                                             double z1, int lane, double &acc0, double &acc1)
{
    double a0 = 0.0, a1 = 0.0;
#pragma unroll 4
    for (int k = c0; k < c1; ++k) {
        const double xj = sx[k], yj = sy[k], zj = sz[k], mj = sm[k];
        {
            const double dx = xj - x0, dy = yj - y0, dz = zj - z0;
            const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            const double y = __builtin_amdgcn_rsq(r2);
            const double e = fma(-r2, y * y, 1.0);
            const double w = fma(e, fma(e, 0.375, 0.5), 1.0);
            a0 = fma(mj * y, w, a0);
        }
        {
            const double dx = xj - x1, dy = yj - y1, dz = zj - z1;
            const double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
            // on the diagonal block only j > i (the rest through a finite
            // stand-in that adds zero)
            const bool keep = !DIAG1 || k > lane;
            const double rk = keep ? r2 : 1.0;
            const double y = __builtin_amdgcn_rsq(rk);
            const double e = fma(-rk, y * y, 1.0);
            const double w = fma(e, fma(e, 0.375, 0.5), 1.0);
            a1 = fma(keep ? mj * y : 0.0, w, a1);
        }
    }
    acc0 = a0;
    acc1 = a1;
}

// sum over the wave, the same bits on every lane (lane 0's butterfly)
__device__ __forceinline__ double wave_sum0(double v)
{
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return wave_uniform(v);
}

// first unit of row b of a system with nj 64-blocks of j: row b' holds the
// j-blocks t >= 2 b', nj - 2 b' units
__device__ __forceinline__ long long energy_row0(long long b, long long nj)
{
    return b * nj - b * (b - 1);
}

__global__ __launch_bounds__(256) void k_energy_pairs(EnergyArgs a)
{
    const Dev &d = a.d;
    __shared__ double lds[4][4][64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int w = blockIdx.x * 4 + wv;
    const long long C0 = d.e_wcol[w], C1 = d.e_wcol[w + 1];
    if (C0 >= C1) return;   // (waves only; no workgroup barrier follows)
    double *sx = lds[wv][0], *sy = lds[wv][1], *sz = lds[wv][2], *sm = lds[wv][3];
    // the system and unit (b, t) of the first column: systems by binary
    // search of their first units, the row b from the row starts
    long long U = C0 >> 6;
    int lo = 0, hi = a.nsys - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (d.sys_u0[mid] <= U) lo = mid; else hi = mid - 1;
    }
    int s = lo;
    while (d.sys_u0[s + 1] <= U) ++s;   // systems without units
    int so = d.sys_off[s], n = d.sys_off[s + 1] - so;
    int nj = (n + 63) >> 6, ni = (n + 127) >> 7;
    const long long v = U - d.sys_u0[s];
    const double q = (double)nj + 1.0;
    int b = (int)((q - sqrt(fmax(q * q - 4.0 * (double)v, 0.0))) / 2.0);
    b = max(0, min(b, ni - 1));
    while (b > 0 && energy_row0(b, nj) > v) --b;
    while (b + 1 < ni && energy_row0(b + 1, nj) <= v) ++b;
    int t = 2 * b + (int)(v - energy_row0(b, nj));
    int rec = d.e_wrec[w];
    double R[kERec] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    const double G = a.G;
    // operands of this lane's two i and its j: loaded one unit ahead, so
    // the loads of the next unit are in flight during the pairs of this one
    auto load_i = [&](int so_, int n_, int i_, double &x, double &y, double &z, double &m,
                      bool &ok) {
        ok = i_ < n_;
        x = ok ? d.x[so_ + i_] : kFarI;
        y = ok ? d.y[so_ + i_] : kFarI;
        z = ok ? d.z[so_ + i_] : kFarI;
        m = ok ? d.m[so_ + i_] : 0.0;
    };
    auto load_j = [&](int so_, int n_, int t_, double &x, double &y, double &z, double &m) {
        const int j = so_ + 64 * t_ + lane;
        const bool ok = 64 * t_ + lane < n_;
        x = ok ? d.x[j] : kFar;
        y = ok ? d.y[j] : kFar;
        z = ok ? d.z[j] : kFar;
        m = ok ? d.m[j] : 0.0;
    };
    double x0, y0, z0, m0, x1, y1, z1, m1;
    bool ok0, ok1;
    load_i(so, n, 128 * b + lane, x0, y0, z0, m0, ok0);
    load_i(so, n, 128 * b + 64 + lane, x1, y1, z1, m1, ok1);
    double jx, jy, jz, jm;
    load_j(so, n, t, jx, jy, jz, jm);
    long long C = C0;
    for (;;) {
        const long long ubase = C & ~63LL;
        const int c0 = (int)(C - ubase);
        const int c1 = C1 - ubase < 64 ? (int)(C1 - ubase) : 64;
        sx[lane] = jx;
        sy[lane] = jy;
        sz[lane] = jz;
        sm[lane] = jm;
        wave_lds_sync();
        // the next unit: the next j-block of the row, the next row, the
        // next system with units; its operands requested now
        const bool more = ubase + c1 < C1;
        int s2 = s, so2 = so, n2 = n, nj2 = nj, ni2 = ni, b2 = b, t2 = t + 1;
        bool newsys = false;
        double px0 = 0.0, py0 = 0.0, pz0 = 0.0, pm0 = 0.0;
        double px1 = 0.0, py1 = 0.0, pz1 = 0.0, pm1 = 0.0;
        bool pok0 = false, pok1 = false;
        if (more) {
            if (t2 == nj2) {
                b2 = b + 1;
                if (b2 == ni2) {
                    newsys = true;
                    do {
                        ++s2;
                    } while (d.sys_u0[s2 + 1] == d.sys_u0[s2]);
                    so2 = d.sys_off[s2];
                    n2 = d.sys_off[s2 + 1] - so2;
                    nj2 = (n2 + 63) >> 6;
                    ni2 = (n2 + 127) >> 7;
                    b2 = 0;
                }
                t2 = 2 * b2;
                load_i(so2, n2, 128 * b2 + lane, px0, py0, pz0, pm0, pok0);
                load_i(so2, n2, 128 * b2 + 64 + lane, px1, py1, pz1, pm1, pok1);
            }
            load_j(so2, n2, t2, jx, jy, jz, jm);
        }
        double acc0 = 0.0, acc1 = 0.0;
        if (t == 2 * b) {
            // the slice is the first half's own 64-block; the second half
            // lies past it
            acc0 = energy_cols_masked(sx, sy, sz, sm, c0, c1, x0, y0, z0, lane, true);
            if (c0 == 0) {
                // the bodies of this i-block: kinetic, central and momentum
                // terms (once: in the range holding the block's first unit)
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    if (!(u == 0 ? ok0 : ok1)) continue;
                    const int i = so + 128 * b + 64 * u + lane;
                    const double xi = u == 0 ? x0 : x1, yi = u == 0 ? y0 : y1;
                    const double zi = u == 0 ? z0 : z1, mi = u == 0 ? m0 : m1;
                    const double vx = d.vx[i], vy = d.vy[i], vz = d.vz[i];
                    R[0] += 0.5 * mi * (vx * vx + vy * vy + vz * vz);
                    R[1] += G * d.sys_m0[s] * mi / dnorm3(xi, yi, zi);
                    R[2] += mi * vx;
                    R[3] += mi * vy;
                    R[4] += mi * vz;
                }
            }
        } else {
            const bool diag1 = t == 2 * b + 1;
            if (diag1)
                energy_cols2<true>(sx, sy, sz, sm, c0, c1, x0, y0, z0, x1, y1, z1, lane, acc0, acc1);
            else
                energy_cols2<false>(sx, sy, sz, sm, c0, c1, x0, y0, z0, x1, y1, z1, lane, acc0, acc1);
            if (isnan(acc0))
                acc0 = energy_cols_masked(sx, sy, sz, sm, c0, c1, x0, y0, z0, lane, false);
            if (isnan(acc1))
                acc1 = energy_cols_masked(sx, sy, sz, sm, c0, c1, x1, y1, z1, lane, diag1);
        }
        R[5] = fma(m0, acc0, R[5]);
        R[5] = fma(m1, acc1, R[5]);
        wave_lds_sync();   // the slice is restaged for the next unit
        if (!more) break;
        if (newsys) {
#pragma unroll
            for (int k = 0; k < kERec; ++k) {
                const double r = wave_sum0(R[k]);
                if (lane == 0) d.erec[(long long)kERec * rec + k] = r;
                R[k] = 0.0;
            }
            ++rec;
        }
        if (b2 != b || newsys) {
            x0 = px0; y0 = py0; z0 = pz0; m0 = pm0; ok0 = pok0;
            x1 = px1; y1 = py1; z1 = pz1; m1 = pm1; ok1 = pok1;
        }
        s = s2;
        so = so2;
        n = n2;
        nj = nj2;
        ni = ni2;
        b = b2;
        t = t2;
        C = ubase + c1;
    }
#pragma unroll
    for (int k = 0; k < kERec; ++k) {
        const double r = wave_sum0(R[k]);
        if (lane == 0) d.erec[(long long)kERec * rec + k] = r;
    }
}

// E of each system from its records, added in order
__global__ __launch_bounds__(256) void k_energy_final(EnergyArgs a)
{
    __shared__ double lds[256];
    const Dev &d = a.d;
    const int s = blockIdx.x;
    const double m0 = d.sys_m0[s];
    double r[kERec] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int q = d.sys_r0[s] + threadIdx.x; q < d.sys_r0[s + 1]; q += 256)
#pragma unroll
        for (int k = 0; k < kERec; ++k) r[k] += d.erec[(long long)kERec * q + k];
#pragma unroll
    for (int k = 0; k < kERec; ++k) r[k] = block_sum<256>(r[k], lds);
    if (threadIdx.x == 0)
        d.E[s] = r[0] + (r[2] * r[2] + r[3] * r[3] + r[4] * r[4]) / (2.0 * m0) - r[1] - a.G * r[5];
}


}  // namespace qsym
