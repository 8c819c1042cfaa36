// Crude encounter sweep (Sec. 2.4, first sweep) on a hashed uniform grid:
// the same candidate pairs as the sweep fused into the first kick, in
// expected O(N) instead of O(N^2) tests.  Selected by qsym_params.sweep = 1.
//
// Every pair is decided by crude_exact, the test of the definition, so the
// candidate set does not depend on the sweep; the grid only has to be
// conservative.  For bodies i, j the exact limit is
//   lim = c_s (R_up + tau (ve_i + ve_j)),
//   R_up = a_E (h_i + h_j)(A_i + A_j) / 2   (mutual Hill radii), or
//   R_up = a_E (h_i A_i + h_j A_j)           (sum of Hill radii).
// With A_i, A_j <= A_lim the mutual form is at most a_E (h_i + h_j) A_lim,
// so lim <= rho_i + rho_j with the separable per-body radius
//   rho_i = c_s (a_E h_i A_lim + tau ve_i)     (sum form: a_E h_i A_i),
// and a pair closer than lim is closer than 2 rho_lim on every axis when
// both radii are at most rho_lim.  Per system A_lim = 2 mean(A) and
// rho_lim = 1.5 mean(rho), from chunk sums of A, h (or h A) and ve that the
// drift's pre-pass leaves (rho is linear in h and ve); the grid cell is
// 2 rho_lim (times 1 + 1e-9 for rounding).  "Small" bodies (A <= A_lim,
// rho <= rho_lim, a free slot in their bucket, within 1e6 cells of the
// origin) go into the grid and test their own cell and half of the 26
// around it; every other body (planets, nearly parabolic or distant
// bodies, overflow of a crowded bucket) is "large" and tests its whole
// system.  A pair is tested exactly once: small-small within a cell from
// the lower index, across cells from the cell the half-shell offset points
// away from, small-large and large-large (from the higher index) in the
// large pass.
// ------------------------------------------------------------------------
#pragma once

#include "qsym_kernels.hpp"

namespace qsym {

constexpr int kSweepCap = 32;        // bodies per hash bucket before overflow to the large list
constexpr int kSweepThreads = 256;
constexpr int kSweepLargeTile = 4096;  // bodies per work item of the large pass
constexpr int kSweepBuf = 1024;        // candidates a workgroup gathers before one global append
constexpr double kSweepFar = 1e6;    // cell coordinates beyond this go to the large list

struct SweepArgs {
    KickArgs ka;       // d, candidate capacity, hill_mode, a_E, c_s, |tau| of crude_exact
    int nsys;
    int ntot;
    int nsmall;        // blocks of k_sweep_search for the small bodies
    int tiles;         // large-pass work items per large body: ceil(max system size / tile)
};

__device__ __forceinline__ unsigned sweep_hash(int s, int cx, int cy, int cz, unsigned mask)
{
    unsigned long long h = (unsigned long long)(unsigned)cx * 73856093ull;
    h ^= (unsigned long long)(unsigned)cy * 19349663ull;
    h ^= (unsigned long long)(unsigned)cz * 83492791ull;
    h ^= (unsigned long long)(unsigned)s * 2654435761ull;
    h ^= h >> 29;
    return (unsigned)h & mask;
}

// The search's candidates are gathered per workgroup in LDS and appended with
// one atomic per workgroup: an atomic per wave with a hit, thousands on the
// one candidate counter in a kernel of a few tens of microseconds, queue on
// its line.  A full buffer falls back to appending directly.
struct SweepOut {
    int2 *buf;
    unsigned *n;
};

// crude_exact on packed operands: the same operations in the same order, so
// the same decision (i < j)
__device__ __forceinline__ void crude_rec(const KickArgs &ka, const SweepOut &o, int i,
                                          const SweepRec &ri, int j, const SweepRec &rj)
{
    const Dev &d = ka.d;
    const double dx = rj.x - ri.x;
    const double dy = rj.y - ri.y;
    const double dz = rj.z - ri.z;
    const double r2 = dx * dx + dy * dy + dz * dz;
    double Rup;
    if (ka.hill_mode == 0)
        Rup = ka.aE * (ri.h + rj.h) * (ri.A + rj.A) / 2.0;
    else
        Rup = ka.aE * (ri.h * ri.A + rj.h * rj.A);
    const double lim = ka.cs * (Rup + ka.tau_abs * (ri.cv + rj.cv));
    if (r2 < lim * lim) {
        const unsigned q = atomicAdd(o.n, 1u);
        if (q < (unsigned)kSweepBuf) {
            o.buf[q] = make_int2(i, j);
        } else {
            const unsigned long long slot = atomicAdd(&d.ctr[C_CAND], 1ull);
            if ((long long)slot < ka.cap) d.cand[slot] = make_int2(i, j);
        }
    }
}

// the workgroup's gathered candidates onto the list (every thread calls it)
__device__ __forceinline__ void sweep_flush(const KickArgs &ka, const SweepOut &o,
                                            unsigned long long *s_base)
{
    const Dev &d = ka.d;
    __syncthreads();
    const unsigned n = min(*o.n, (unsigned)kSweepBuf);
    if (threadIdx.x == 0 && n) *s_base = atomicAdd(&d.ctr[C_CAND], (unsigned long long)n);
    __syncthreads();
    for (unsigned k = threadIdx.x; k < n; k += blockDim.x) {
        const unsigned long long slot = *s_base + k;
        if ((long long)slot < ka.cap) d.cand[slot] = o.buf[k];
    }
}

__device__ __forceinline__ double sweep_rho(const KickArgs &ka, int i, double Alim)
{
    const Dev &d = ka.d;
    const double hA = ka.hill_mode == 0 ? d.ch[i] * Alim : d.ch[i];
    return ka.cs * (ka.aE * hA + ka.tau_abs * d.cv[i]);
}

// one workgroup per 256-body chunk (the drift's chunks): the system's grid
// constants from the chunk sums (every chunk of a system computes the same
// values in the same order), then each body of the chunk into its cell's
// bucket or onto the large list
__global__ __launch_bounds__(kChunk) void k_sweep_bin(SweepArgs a)
{
    const KickArgs &ka = a.ka;
    const Dev &d = ka.d;
    __shared__ double lds[kChunk];
    const int t = threadIdx.x;
    const int4 bc = d.bchunk[blockIdx.x];
    const int s = bc.x;
    const int c0 = d.sys_c0[s], c1 = d.sys_c0[s + 1];
    double S[3];
    for (int k = 0; k < 3; ++k) {
        double acc = 0.0;
        for (int c = c0 + t; c < c1; c += kChunk) acc += d.sw_part[3 * c + k];
        S[k] = block_sum<kChunk>(acc, lds);
    }
    const double n = (double)(d.sys_off[s + 1] - d.sys_off[s]);
    const double Alim = ka.hill_mode == 0 ? 2.0 * S[0] / n : 0.0;
    const double hA = ka.hill_mode == 0 ? (S[1] / n) * Alim : S[1] / n;
    const double rlim = 1.5 * ka.cs * (ka.aE * hA + ka.tau_abs * (S[2] / n));
    const double cell = 2.0 * rlim * (1.0 + 1e-9);
    if (t == 0 && (int)blockIdx.x == c0) d.sys_sw[s] = make_double4(Alim, rlim, cell, 0.0);
    if (t >= bc.z) return;
    const int i = bc.y + t;
    const double rho = sweep_rho(ka, i, Alim);
    bool large = !(cell > 0.0) || !(cell < INFINITY) || !(rho <= rlim) ||
                 (ka.hill_mode == 0 && !(d.A[i] <= Alim));
    int cx = 0, cy = 0, cz = 0;
    if (!large) {
        const double inv = 1.0 / cell;
        const double fx = floor(d.x[i] * inv), fy = floor(d.y[i] * inv), fz = floor(d.z[i] * inv);
        if (!(fabs(fx) < kSweepFar && fabs(fy) < kSweepFar && fabs(fz) < kSweepFar)) {
            large = true;
        } else {
            cx = (int)fx;
            cy = (int)fy;
            cz = (int)fz;
            const unsigned bk = sweep_hash(s, cx, cy, cz, (unsigned)d.sw_nb - 1u);
            const int k = atomicAdd(&d.sw_cnt[bk], 1);
            if (k < kSweepCap)
                d.sw_slot[(long long)bk * kSweepCap + k] = i;
            else
                large = true;
        }
    }
    SweepRec r;
    r.x = d.x[i];
    r.y = d.y[i];
    r.z = d.z[i];
    r.h = d.h[i];
    r.A = d.A[i];
    r.cv = d.cv[i];
    r.cx = cx;
    r.cy = cy;
    r.cz = cz;
    r.sys = large ? -(s + 1) : s;
    d.sw_rec[i] = r;
    if (large) d.sw_large[(int)atomicAdd(&d.ctr[C_NLARGE], 1ull)] = i;
}

// blocks [0, nsmall): thread g takes small body i = g / 14 and cell
// k = g % 14 around its own: k = 0 its own cell (later bodies only),
// k = 1..13 the half of the 26 neighbours whose offset (dz, dy, dx) is
// lexicographically positive (every body there).  Each unordered pair of
// adjacent cells is met from exactly one side, each pair within a cell
// once.  Blocks beyond: the large bodies against their systems, in work
// items of (large body, tile of kSweepLargeTile bodies).
__global__ __launch_bounds__(kSweepThreads) void k_sweep_search(SweepArgs a)
{
    const KickArgs &ka = a.ka;
    const Dev &d = ka.d;
    const int t = threadIdx.x;
    __shared__ int2 s_buf[kSweepBuf];
    __shared__ unsigned s_n;
    __shared__ unsigned long long s_base;
    if (t == 0) s_n = 0u;
    __syncthreads();
    const SweepOut o{s_buf, &s_n};
    if ((int)blockIdx.x < a.nsmall) {
        const long long g = (long long)blockIdx.x * kSweepThreads + t;
        const int i = (int)(g / 14), nbr = (int)(g % 14);
        const bool ok = g < 14ll * a.ntot;
        const SweepRec ri = d.sw_rec[ok ? i : 0];
        if (ok && ri.sys >= 0) {
            const int s = ri.sys;
            // half-shell offset number nbr - 1 of the 13 with (dz, dy, dx) > 0:
            // codes 14..26 of 9 (dz + 1) + 3 (dy + 1) + (dx + 1)
            const int code = nbr == 0 ? 13 : 13 + nbr;
            const int nx = ri.cx + code % 3 - 1, ny = ri.cy + (code / 3) % 3 - 1;
            const int nz = ri.cz + code / 9 - 1;
            const unsigned bk = sweep_hash(s, nx, ny, nz, (unsigned)d.sw_nb - 1u);
            const int nb = min(d.sw_cnt[bk], kSweepCap);
            for (int k = 0; k < nb; ++k) {
                const int j = d.sw_slot[(long long)bk * kSweepCap + k];
                if (nbr == 0 && j <= i) continue;
                const SweepRec rj = d.sw_rec[j];
                // another cell or system in the same bucket
                if (rj.cx != nx || rj.cy != ny || rj.cz != nz || rj.sys != s) continue;
                if (i < j)
                    crude_rec(ka, o, i, ri, j, rj);
                else
                    crude_rec(ka, o, j, rj, i, ri);
            }
        }
    } else {
        const int nl = (int)d.ctr[C_NLARGE];
        const int items = nl * a.tiles;
        const int stride = gridDim.x - a.nsmall;
        for (int it = blockIdx.x - a.nsmall; it < items; it += stride) {
            const int L = d.sw_large[it / a.tiles];
            const SweepRec rL = d.sw_rec[L];
            const int s = -rL.sys - 1;
            const int o0 = d.sys_off[s], n = d.sys_off[s + 1] - o0;
            const int j0 = (it % a.tiles) * kSweepLargeTile;
            const int j1 = min(n, j0 + kSweepLargeTile);
            for (int k = j0 + t; k < j1; k += kSweepThreads) {
                const int j = o0 + k;
                if (j == L) continue;
                const SweepRec rj = d.sw_rec[j];
                if (rj.sys < 0 && j > L) continue;   // a large-large pair from its higher index
                if (L < j)
                    crude_rec(ka, o, L, rL, j, rj);
                else
                    crude_rec(ka, o, j, rj, L, rL);
            }
        }
    }
    sweep_flush(ka, o, &s_base);
}

}  // namespace qsym
