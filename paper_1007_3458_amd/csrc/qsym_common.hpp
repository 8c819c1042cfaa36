// qsym_common.hpp -- device-side data layout shared by the kernels and the
// host code of the MI355X DH hybrid-step library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace qsym {

constexpr int kChunk = 256;        // bodies per workgroup of the O(N) kernels
constexpr int kChunkK = 64;        // bodies per workgroup of the Kepler pass
constexpr int kCapE = 4096;        // encounter pairs of one system partitioned on chip (LDS)
constexpr int kCapU = 2 * kCapE;   // bodies of one system taking part in encounters (LDS)
constexpr int kHist = 32;
// The Kepler pass's statistics (iteration histogram, total, largest) are
// kept in kStatStripes copies, kStatStride entries (512 B) apart: the
// workgroups of one launch add to different copies, so their atomics spread
// over many memory channels instead of queueing on one line; the host adds
// the copies up when it reads the statistics.
constexpr int kStatStripes = 64;
constexpr int kStatStride = 64;   // entries: [0, kHist) histogram, kHist total, kHist + 1 largest,
                                  // kHist + 2 solves restarted from the first-order guess
constexpr int kSMax = 64;          // largest j-split of one system
constexpr int kSetsThreads = 512;  // workgroup of the set-partition kernel
constexpr int kHermThreads = 512;  // workgroup of the Hermite kernel
constexpr int kHermWave = 64;      // lanes of the one-wave Hermite
constexpr int kWaveMax = 16;       // sets up to this size run on one wave, larger on a workgroup
constexpr int kCoopMin = 256;      // sets above this size run on the whole grid
constexpr int kGridMax = 1024;     // largest grid of the grid-wide Hermite
constexpr double kPi = 3.14159265358979323846;

// counters / status word in device memory (unsigned 64-bit for atomics;
// the Kepler statistics are striped apart, see kStatStripes)
enum Ctr {
    C_CAND = 0,   // crude candidates of the last sweep (true count)
    C_ENC,        // fine-sweep encounter pairs of the last step (true count)
    C_NSETS,      // sets of the last step
    C_MAXSET,     // largest set of the last step
    C_SUB,        // Hermite substeps of the last step
    C_TENC,       // total encounters
    C_TSUB,       // total substeps
    C_STEPS,      // steps taken
    C_STATUS,     // latched status bits
    C_NU,         // bodies in encounters, last step
    C_NSMALL,     // sets of at most kWaveMax members (one wave each), last step
    C_NBIG,       // larger sets (one workgroup each), last step
    C_NGRID,      // sets above kCoopMin members (the grid phase), last step
    C_WHOLE,      // systems integrated whole (all steps)
    C_NLARGE,     // grid sweep: bodies on the large list, last step
    C_TBIGSYS,    // systems whose sets were partitioned in global memory, all steps
    C_FALLBACK,   // steps whose candidate list overflowed: all-pairs fine sweep instead
    C_OVERFLOW,   // steps left undone because a system's encounter pairs overflowed
    C_COUNT
};

enum Status : unsigned long long {
    S_CAND_OVF = 1,
    S_ENC_OVF = 2,
    S_KEPLER = 4,
    S_HERMITE = 8,
    S_NONFINITE = 16,
    S_SET_BIG = 32,
};

// Status bits that stop the integration: a step that raises one leaves the
// state as it was at the step's start (the first drift keeps a copy, the
// last one puts it back), and every later step does the same until a new
// state is set.
constexpr unsigned long long S_FREEZE = S_ENC_OVF;

// Global-memory scratch of the set partition of one system of n bodies (in
// 64-bit slots): body bitmap, its word prefix counts, the bodies in
// encounters, union-find labels, root flags, and the member sort keys.
__host__ __device__ inline long long gs_words(long long n) { return (n + 31) / 32; }
__host__ __device__ inline long long gs_pow2(long long n)
{
    long long p = 1;
    while (p < n) p <<= 1;
    return p;
}
__host__ __device__ inline long long gs_slots(long long n)
{
    return 2 * ((gs_words(n) + 1) / 2) + 3 * ((n + 1) / 2) + gs_pow2(n);
}

// one workgroup of the pair kernels: i-bodies [i0, i0+ni) of system sys
// against j-bodies [j0, j0+nj) (its j-chunk number `chunk`)
struct KickItem {
    int sys, i0, ni, j0, nj, chunk, slot;   // slot: j-side partial slot (symmetric kick)
};

// one body's operands of the crude test, packed into one 64-byte line for
// the grid sweep: position, h, a, ve, grid cell, and its system (negative,
// -(sys + 1), for bodies on the large list)
struct SweepRec {
    double x, y, z, h, A, cv;
    int cx, cy, cz, sys;
};

// device pointers into the caller-provided workspace
struct Dev {
    double *x, *y, *z, *vx, *vy, *vz, *m, *h;   // state (global body index)
    double *x0, *y0, *z0, *vx0, *vy0, *vz0;     // state after the first kick
    double *A, *ch, *cv;                        // a_i; crude-sweep per-body terms
    double *acc;                                // kick partial sums
    double *pm;                                 // momentum partials [Kepler-pass chunk][3]
    int *body_sys;                              // system of each body
    int *sys_off;                               // [nsys+1] first body of each system
    double *sys_m0;                             // central masses
    int4 *sys_K;                                // [2][nsys] partial-slot layout per kick shape
    long long *sys_poff;                        // offset of its partials in acc
    int *sys_c0;                                // [nsys+1] first O(N) chunk
    int *sys_k0;                                // [nsys+1] first Kepler-pass chunk
    int4 *bchunk;                               // O(N) chunks (sys, first, count, 0)
    int4 *kchunk;                               // kChunkK-body chunks of the Kepler pass
    KickItem *items;                            // [2][max_items] kick work items
    KickItem *eitems;                           // energy work items
    int *sys_e0;                                // [nsys+1] first energy item
    int2 *cand;                                 // crude candidates
    int2 *enc;                                  // encounter pairs, per-system segments
    int *sys_eoff;                              // [nsys+1] segment offsets (capacities)
    int *sys_ecnt;                              // [nsys] pairs appended this step
    int *set_start;                             // [setcap] first member slot of each set
    int *set_count;                             // [setcap] members of each set
    int *set_mem;                               // [memcap] member body indices
    double *set_rc;                             // [setcap] r_crit per set
    int *set_list;                              // [setcap] small sets from 0 up, big from the end down
    int setcap;                                 // set slots
    long long *sys_goff;                        // [nsys] their scratch offset in gsa (-1: none)
    unsigned long long *gsa;                    // global set-partition scratch
    double *bk;                                 // [6][np] state at the start of the step
    int *krow;                                  // [2][rows] items per row (balanced-row kick)
    unsigned *gbar;                             // grid barrier of the Hermite's grid phase (3 words)
    double *hpart;                              // [2][kGridMax] its per-block step minima
    int *sw_cnt;                                // grid sweep: [sw_nb] bucket counts
    int *sw_slot;                               // [sw_nb][kSweepCap] bodies per bucket
    SweepRec *sw_rec;                           // [np] packed crude-test operands and cell
    int *sw_large;                              // [np] bodies of the large list
    double4 *sys_sw;                            // [nsys] A_lim, rho_lim, cell size
    double *sw_part;                            // [chunk][3] sums of a, h (or h a), ve
    int sw_nb;                                  // buckets (a power of two)
    int memcap;                                 // member slots (Hermite scratch stride)
    double *hw;                                 // Hermite member scratch
    unsigned long long *ctr;                    // counters and status
    unsigned long long *kstat;                  // [kStatStripes][kStatStride] Kepler statistics
    double *erec;                               // energy records [record][6] (k_energy_pairs)
    long long *e_wcol;                          // [waves+1] first pair column of each wave
    int *e_wrec;                                // [waves] first record of each wave
    long long *sys_u0;                          // [nsys+1] first energy unit of each system
    int *sys_r0;                                // [nsys+1] first energy record of each system
    double *E;                                  // energies per system
    float *guess;                               // learned Kepler start: weights + scalers
};

}  // namespace qsym
