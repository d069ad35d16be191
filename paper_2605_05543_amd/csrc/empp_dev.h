// empp_dev.h -- device-side types and helpers shared by the HIP kernels of
// libempp.so.  gfx950 only; compiled with hipcc --offload-arch=gfx950.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace empp {

// CODATA 2018 (c, e, m_e exact or recommended; mu0 recommended).
constexpr double kC_LIGHT = 299792458.0;
constexpr double kMU0 = 1.25663706212e-6;

#ifndef EMPP_PAIR_BLOCK
#define EMPP_PAIR_BLOCK 512
#endif
constexpr int kBlock = EMPP_PAIR_BLOCK;  // threads per block of the mixed pair kernel and per-particle kernels
// Threads per block of the FP64 pair kernel: 1024 targets share each staged
// history tile (one block per CU at 128 registers per lane).
#ifndef EMPP_FP64_BLOCK
#define EMPP_FP64_BLOCK 1024
#endif
constexpr int kBlockFp64 = EMPP_FP64_BLOCK;

// Deepest supported history (slots): the pair kernel's LDS tile for it, one
// history of 32-byte records plus its light distances, fills a CU's 160 KiB.
constexpr int kMaxDepth = 4064;
constexpr int kMaxSplits = 1024;   // source chunks of one launch

// History layout in HBM (library-owned workspace):
//   ring_w[j * D + p] = {x, y, z, 0}     position of source j at physical slot p
//   ring_v[j * D + p] = {vx, vy, vz, 1/h} velocity leaving that slot and the
//                                         inverse length of its segment (0: newest)
//   T[p]                                  slot time
// Slot p holds logical slot "back" b (0 = newest) when p = (head - b) mod D.
// A source's whole history is one contiguous 32*D-byte block, so a block
// of targets stages it into LDS with straight coalesced loads.

struct PairParams {
    const double4 *ring_w;
    const double4 *ring_v;
    const double4 *rec;  // light-cone records [N][D], newest slot first (lightcone_records_kernel)
    const double *T;
    int64_t n_src;      // sources N
    int32_t D;
    int32_t head;       // physical index of the newest slot
    double t;           // present time (== T[head]; the pair kernels read T[head])
    double kq;          // Coulomb constant times source charge
    // targets: external points x[3][m] (x != nullptr) or the particles'
    // newest positions (x == nullptr, then target a is particle a and the
    // pair (a, a) is skipped).
    const double *x;
    const int64_t *self_index;  // external mode only, may be null
    const int32_t *order;       // step mode: target slot -> particle (spatial order), may be null
    int32_t nit;                // bisection steps: ceil(log2(D - 1))
    int64_t m;
    int64_t src_per_split;
    int32_t nsplit;
    int32_t tile;               // sources staged per LDS tile
    int32_t nbuf;               // LDS tile buffers (FP64 kernel: 1 or 2)
    int32_t groups;             // groups of `tile` sources per staged tile (FP64 kernel)
    double *part;               // [nsplit][12][m] partial (sum, comp)
    int32_t *kstar;             // [m][N] or null
    unsigned long long *err;    // [2]: first failing pair, status bits
    unsigned long long *counters;  // [5] pairs, before, probes, rescues, fallbacks
    // surrogate / guided search
    int32_t guess;
    float dt_inv_f;
    double dt;
    const float *G;             // surrogate guesses G[source * g_groups + (a >> g_shift)]
    int64_t g_groups;           // target groups of the launch
    int32_t g_shift;            // guess mode 1: log2 of the targets per guess; mode 3: 0 (one per pair)
    // guess modes: 0 bisection, 1 surrogate correction per target group,
    // 2 straight-line look-back, 3 surrogate delay per pair, 4/5 warm start
    // warm start (step mode): bracket of every (source j, target slot a)
    // from the previous step at kc[j * m + a]: back offset b* (1..D-1) or
    // kBracketBefore.  Read by the warm-start search (kc_cold = 0) and
    // written by it; on a cold step the bisection fills it.
    uint16_t *kc;
    int32_t kc_cold;
    // adaptive step (Sec. 2.4): min |eta| and max |v_i - v_j(t_r)|^2 over
    // the pairs with |eta| >= eta_allow, folded into ad[0] (atomicMin) and
    // ad[1] (atomicMax) as double bit patterns; null when the step is fixed
    unsigned long long *ad;
    double eta_allow;
    // reconstruction inside the bracket: 0 = local linear (Eq. linear, the
    // method), 1 = midpoint values (Eq. mid, accuracy ablation)
    int32_t recon;
};

constexpr uint16_t kBracketBefore = 0xFFFF;

// Search modes (pair-kernel template argument) whose pass stages the
// precomputed light-cone records of lightcone_records_kernel (the guided
// searches, 1-3, and the warm start, 4) rather than computing them from the
// positions while staging (the bisection, 0, and the cache-filling
// bisection, 5).
__host__ __device__ constexpr bool pass_uses_records(int guess) { return guess >= 1 && guess <= 4; }

struct PushParams {
    double4 *ring_w;
    double4 *ring_v;
    double *T;
    double *u;          // [3][N]
    double *E;          // [3][N] self-field of the step (output of the merge)
    double *B;
    const double *part; // [nsplit][12][N], in the pair launch's target order
    const int32_t *order; // target order -> particle index
    int32_t nsplit;
    int64_t N;
    int32_t D;
    int32_t head;       // newest physical slot before the push
    double dt;
    double t_now;       // time of the newest slot before the push
    double t_next;      // time of the new slot
    double eps;         // q dt / (2 m)
    int32_t ext_field;
    double dip_k;       // b0 * re^3: (mu0/4pi) M0 for the centred dipole
    int32_t self_field; // 0: stage-II transport (E = 0, B = B_geo only)
    // adaptive step: ad = this step's {eta_min, v_max^2} slot (null: fixed
    // dt); the step is c_dt eta_min / v_max clamped to [dt_min, dt_max],
    // t_now is read from T[head], and ad_next/dt_out are reset/written
    unsigned long long *ad;
    unsigned long long *ad_next;
    double *dt_out;
    double c_dt, dt_min, dt_max;
    double q, m;
};

// Block of a pair-kernel launch -> (target block bx, source chunk split).
// The grid is one-dimensional, nbx * nsplit blocks.  Workgroups go to the 8
// XCDs round-robin by linear index; when the chunk count is a multiple of 8
// every chunk is given to one XCD, so the target blocks that stage its
// histories run there together and share that XCD's L2.
__device__ inline void pair_block_coords(int nbx, int nsplit, int &bx, int &split)
{
    const int L = blockIdx.x;
    if ((nsplit & 7) == 0) {
        const int xcd = L & 7, k = L >> 3;
        const int round = k / nbx;
        split = xcd + 8 * round;
        bx = k - round * nbx;
    } else {
        split = L / nbx;
        bx = L - split * nbx;
    }
}

// Stage II (transport after the handoff): positions pos[i] = {x, y, z, 0},
// proper velocities u[3][N]; the step is
// dt = min(dt_max, gyro_k * min_i gamma_i / |B(y_i)|), the minimum being
// kept in three rotating slots of double bit patterns (positive doubles
// order like their unsigned bit patterns): step k reads slot k % 3, builds
// slot (k + 1) % 3 with atomicMin and clears slot (k + 2) % 3.
struct TransportParams {
    double4 *pos;
    double *u;
    int64_t N;
    double q_over_2m;
    double dip_k;
    int32_t ext_field;
    double dt_max;
    double gyro_k;
    unsigned long long *key;  // [3]
    double *t;                // [1] present time
    int64_t step;
};

constexpr unsigned long long kPosInfBits = 0x7FF0000000000000ull;

// Error word: err[0] = (target << 32 | source) of the lowest failing pair
// (atomicMin), err[1] = OR of status bits.
constexpr unsigned long long kErrCoincident = 1ull;
constexpr unsigned long long kErrDiscriminant = 2ull;

__device__ inline void report_error(unsigned long long *err, int64_t a, int64_t j,
                                    unsigned long long bit)
{
    unsigned long long key = ((unsigned long long)(uint32_t)a << 32) | (uint32_t)j;
    atomicMin(&err[0], key);
    atomicOr(&err[1], bit);
}

// Reciprocal of a positive normal double: hardware estimate plus one
// Newton-Raphson step, which squares the estimate's relative error (about
// 2^-26) to the last bits of the mantissa.
__device__ inline double rcp64(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}

// Neumaier accumulation of x into (s, c).
__device__ inline void neumaier(double &s, double &c, double x)
{
    double t = s + x;
    double big = fabs(s) >= fabs(x) ? s : x;
    double small = fabs(s) >= fabs(x) ? x : s;
    c += (big - t) + small;
    s = t;
}

}  // namespace empp
