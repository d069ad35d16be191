// pair_kernel.h -- the all-pairs Lienard-Wiechert pass shared by the FP64
// and the mixed-precision pair kernels (Secs. 2.1-2.2 of arXiv 2605.05543).
//
// One thread owns one target.  A block of kBlockFp64 (1024) targets walks its
// chunk of sources in staged tiles of up to four sources: the tile's
// histories, as the per-sample part of the split light-cone test (offsets
// from each source's newest sample and L^2 - |offset|^2, see pair_common.h),
// are staged once into LDS, double-buffered behind one barrier per tile, and
// every target of the block then searches them, so each history byte read
// from L2/HBM serves 1024 targets.  The sources of a tile are searched in
// groups of S in lockstep (a fixed number of bisection steps, no divergence);
// then, source by source, the two bracket velocity records are fetched and
// the pair field evaluated.  Targets are visited in a spatial (Morton) order so that
// the lanes of a wavefront probe nearby history slots.  Sums are kept per
// target in registers: a plain partial merged into a compensated total
// (Neumaier in FP64 every 32 sources, Knuth's two-sum in FP32 every 8);
// source chunks write (sum, compensation) partials, in the launch's target
// order, that the merge kernel adds in a fixed order (and maps to particle
// indices), so results do not depend on scheduling.
//
// Every sign test is the FP64 test of the paper's bracket, in both
// precisions: the bracket index is bit-identical across paths and search
// modes.  MIX selects the mixed-precision field evaluation (root,
// reconstruction and LW terms in FP32 around FP64 coefficients).
#pragma once

#include "pair_common.h"

#include <algorithm>
#include <type_traits>

namespace empp {

// Records per half-array of a double-buffered LDS tile: 32 KiB of the
// records' first 16-byte halves, then 32 KiB of their second halves.
constexpr int kHalfRecs = 2048;

// Sources searched in lockstep by a thread, per search mode (measured at
// N = 65536, D = 512): two for the mixed path's straight-line and
// surrogate guesses, whose short searches leave room for a second one in
// flight (surrogate: 32.27 -> 31.87 ms); one elsewhere, where the second
// search's registers cost more than its overlap gains (FP64 straight-line
// guess 31.07 ms with one, 32.26 with two, which spill; the bisection, 126
// VGPRs either way, 35.19 and 35.31).
constexpr int lockstep_sources(bool mix, int guess) { return mix && (guess == 2 || guess == 1) ? 2 : 1; }

// LDS buffers: two of 64 KiB (staging overlapped with the search) while a
// staged tile fits in kHalfRecs records, else one sized to the tile
// (depths above 2048; kMaxDepth slots fill the CU's 160 KiB with the slot
// light distances and the per-source data).
constexpr int pair_nbuf(int D, int tile) { return (int64_t)tile * D <= kHalfRecs ? 2 : 1; }

// Per-source data of the staged tiles, in 16-byte units: the straight-line
// data of the guided searches (per buffer and source {beta, 1 - beta^2} and
// {1 / (1 - beta^2), -, -, -}), the surrogate's correction per buffer,
// wavefront and source, and the newest samples w_n of three tiles' sources.
constexpr int kLineRecs = 2 * 2 * 4 + 2 * (kBlockFp64 / 64) * 4 / 4 + 3 * 4 * 2;

// slot_table: the kernels with the tile buffer count fixed at compile time
// (double-buffered tiles, D <= 2048) also keep, per logical slot, the byte
// offsets of its ring row entry and of the next newer one.
constexpr size_t pair_lds_bytes(int D, int tile, bool slot_table = false)
{
    const size_t half = pair_nbuf(D, tile) == 2 ? kHalfRecs : (size_t)tile * D;
    return (size_t)pair_nbuf(D, tile) * 2 * half * sizeof(double2) + (size_t)((D + 1) & ~1) * sizeof(double) +
           kLineRecs * sizeof(float4) + (slot_table ? (size_t)((D + 3) & ~3) * sizeof(uint32_t) : 0);
}

// Sources per staged LDS tile for a history depth: as many as fill a
// buffer of kHalfRecs records, at most four (one barrier per staged tile).
constexpr int pair_staged_tile(int D) { return D <= kHalfRecs ? std::min(4, kHalfRecs / D) : 1; }

static_assert(pair_lds_bytes(kMaxDepth, pair_staged_tile(kMaxDepth)) <= 160 * 1024,
              "the deepest history's tile, light distances and per-source data fit a CU's LDS");
static_assert(pair_lds_bytes(kHalfRecs, pair_staged_tile(kHalfRecs), true) <= 160 * 1024,
              "the deepest double-buffered tiles fit with the slot table");
// its 16-bit byte offsets of 32-byte ring entries
static_assert((kHalfRecs - 1) * 32 < 65536, "slot table offsets fit 16 bits");

namespace {

// sqrt of a positive normal double from the hardware reciprocal square
// root and one Newton correction of x y: the estimate's relative error
// (about 2^-26) is squared, to within a few units in the last place (no
// special-value handling, x > 0 here).  The root enters the pair's field
// through c (t_r - t_1), at most one step of light travel, against
// |eta| of millimetres, so this is far below the field tolerance.
__device__ inline double sqrt_pos(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double sq = x * y;
    const double r = __builtin_fma(-sq, sq, x);
    return __builtin_fma(r, 0.5 * y, sq);
}

// Retarded root, reconstruction and LW field of one pair (Eqs. dt,
// linear, linear2, LW_E, LW_B).  (dx, dy, dz) = r - w_1, the target's
// offset from the bracket's older sample, L1 = c (t - t_1);
// v1 = {v_1, 1/(t_2 - t_1)}, v2 = {v_2, -} the velocity records of the
// bracket ends; dw = w_2 - w_1 (midpoint ablation only).  Writes E and B
// into f[0..5].  Returns false on a numerical failure (negative
// discriminant, eta <= 0).
__device__ inline bool lw_pair(double dx, double dy, double dz, double L1, double4 v1, double4 v2, bool before,
                               double kq, double f[6], double &eta_len, double3 &v_ret, bool mid, double3 dw)
{
    const double c = kC_LIGHT;
    const double c2 = c * c;
    // C2 dt^2 + 2 C1h dt + C0 = 0 (Eq. dt with C1 = 2 C1h); the physical
    // root -(C1h + sqrt(C1h^2 - C2 C0))/C2 in Vieta's form.
    double C2 = c2 - (v1.x * v1.x + v1.y * v1.y + v1.z * v1.z);
    double C1h = (dx * v1.x + dy * v1.y + dz * v1.z) - c * L1;
    double C0 = L1 * L1 - (dx * dx + dy * dy + dz * dz);
    double disc = C1h * C1h - C2 * C0;
    bool ok = disc > 0.0;
    double sq = sqrt_pos(ok ? disc : 1.0);
    double dtr = C0 * rcp64(sq - C1h);
    // reconstruction: w = w1 + v1 dt; v = v1 + (v2 - v1) df; a = (v2 - v1)/h
    double inv_h = before ? 0.0 : v1.w;
    double gx = v2.x - v1.x, gy = v2.y - v1.y, gz = v2.z - v1.z;
    double ax = gx * inv_h, ay = gy * inv_h, az = gz * inv_h;  // zero out of history
    double df = dtr * inv_h;
    double vrx = v1.x + gx * df, vry = v1.y + gy * df, vrz = v1.z + gz * df;
    double ex = dx - v1.x * dtr, ey = dy - v1.y * dtr, ez = dz - v1.z * dtr;  // eta
    // |eta| = c (t - t_r) on the reconstructed segment
    double en = L1 - c * dtr;
    if (mid && !before) {
        // Eq. (mid): the bracket ends' means, eta = r - (w_1 + w_2)/2
        ex = dx - 0.5 * dw.x;
        ey = dy - 0.5 * dw.y;
        ez = dz - 0.5 * dw.z;
        en = sqrt(ex * ex + ey * ey + ez * ez);
        vrx = 0.5 * (v1.x + v2.x);
        vry = 0.5 * (v1.y + v2.y);
        vrz = 0.5 * (v1.z + v2.z);
        ok = true;
    }
    double ev = c * en - (ex * vrx + ey * vry + ez * vrz);  // eta . v'
    ok = ok && (en > 0.0) && (ev > 0.0);
    double inv = rcp64(en * ev);
    double ien = ev * inv, iev = en * inv;
    const double ic = 1.0 / c;
    const double icn = ien * ic;
    double hx = ex * icn, hy = ey * icn, hz = ez * icn;  // eta_hat / c
    double px = c2 * hx - vrx, py = c2 * hy - vry, pz = c2 * hz - vrz;  // v'
    double vv = vrx * vrx + vry * vry + vrz * vrz;
    // (c^2 - v^2) v' + eta x (v' x a), the cross product expanded as
    // v' (eta . a) - a (eta . v') with eta . v' = ev
    double ea = ex * ax + ey * ay + ez * az;
    double pref = kq * en * (iev * iev * iev);
    double k1 = pref * ((c2 - vv) + ea), k2 = pref * ev;
    double Ex = k1 * px - k2 * ax;
    double Ey = k1 * py - k2 * ay;
    double Ez = k1 * pz - k2 * az;
    f[0] = Ex;
    f[1] = Ey;
    f[2] = Ez;
    // B = eta_hat x E / c
    f[3] = hy * Ez - hz * Ey;
    f[4] = hz * Ex - hx * Ez;
    f[5] = hx * Ey - hy * Ex;
    eta_len = en;
    v_ret = make_double3(vrx, vry, vrz);
    return ok;
}

// Knuth two-sum: s + e == a + b exactly.
__device__ inline void two_sum(float &s, float &e, float x)
{
    float t = s + x;
    float bb = t - s;
    float err = (s - (t - bb)) + (x - bb);
    s = t;
    e += err;
}

struct MixedPair {
    double3 d;           // r - w_1, the target's offset from the bracket's older sample
    double4 v1, v2;      // FP64 velocity records of the bracket ends
};

// Root, reconstruction and LW field from FP64 inputs.  The coefficients of
// the quadratic, the velocity at the root and u = eta - |eta| v/c (which
// carries the cancellation 1 - eta_hat.beta of nearly forward pairs) are
// formed in FP64; the root, the normalisations and the LW products in FP32.
// Since eta = d - v_1 dt and |eta| = L1 - c dt, u = d - (L1/c) v_r +
// dt (v_r - v_1): the FP64 offset d enters directly and no large terms
// cancel in FP32.  Writes E, B into f[0..5]; rescued = the FP32 root failed
// its residual test and was recomputed in FP64.  Returns false on a
// numerical failure.
// The FP64 re-solve is the same arithmetic in every search mode (refined
// hardware square root and reciprocal), so fields do not depend on the
// search.  BRANCH_RESCUE only decides how it is compiled: a branch around
// it (an empty volatile asm cannot be speculated), or left to the compiler,
// which may evaluate it for every pair and select (measured: a branch pays
// in the bisection pass, 43.2 -> 36.7 ms at N = 65536, D = 512; the guided
// passes are 1-2 % faster with the compiler's choice).
template <bool BRANCH_RESCUE>
__device__ __forceinline__ bool lw_pair_mixed(double L1d, MixedPair q, bool before,
                                              float kq, float f[6], bool &rescued)
{
    const double c = kC_LIGHT;
    const double ic = 1.0 / kC_LIGHT;
    const float cf = (float)kC_LIGHT;
    // FP64: offset to the bracket sample and the quadratic's coefficients
    double dxd = q.d.x, dyd = q.d.y, dzd = q.d.z;
    double C0d = L1d * L1d - (dxd * dxd + dyd * dyd + dzd * dzd);
    double C2d = c * c - (q.v1.x * q.v1.x + q.v1.y * q.v1.y + q.v1.z * q.v1.z);
    double C1hd = (dxd * q.v1.x + dyd * q.v1.y + dzd * q.v1.z) - c * L1d;
    double discd = C1hd * C1hd - C2d * C0d;
    bool ok = discd > 0.0;
    // FP32 root in the form without cancellation, checked by its residual
    float C0 = (float)C0d, C1h = (float)C1hd, C2 = (float)C2d;
    float sq = __builtin_amdgcn_sqrtf(ok ? (float)discd : 1.0f);
    float dtr = C1h <= 0.0f ? C0 * __builtin_amdgcn_rcpf(sq - C1h) : -(C1h + sq) * __builtin_amdgcn_rcpf(C2);
    float res = __builtin_fmaf(__builtin_fmaf(C2, dtr, 2.0f * C1h), dtr, C0);
    float tol = 8.0f * 5.9604645e-8f * (fabsf(C2) * dtr * dtr + 2.0f * fabsf(C1h * dtr) + fabsf(C0));
    rescued = !(fabsf(res) <= tol);
    if (rescued) {
        if constexpr (BRANCH_RESCUE)
            asm volatile("");
        // refined hardware estimates; both divisors are positive
        double sqd = sqrt_pos(ok ? discd : 1.0);
        double rd = C1hd <= 0.0 ? C0d * rcp64(sqd - C1hd) : -(C1hd + sqd) * rcp64(C2d);
        dtr = (float)rd;
    }
    // FP64: velocity at the root and u = d - (L1/c) v_r + dt (v_r - v_1)
    double inv_hd = before ? 0.0 : q.v1.w;
    double dtd = (double)dtr;
    double gxd = q.v2.x - q.v1.x, gyd = q.v2.y - q.v1.y, gzd = q.v2.z - q.v1.z;
    double dfd = dtd * inv_hd;
    double vrxd = q.v1.x + gxd * dfd, vryd = q.v1.y + gyd * dfd, vrzd = q.v1.z + gzd * dfd;
    double Lc = L1d * ic, tg = dtd * dfd;
    double uxd = dxd - Lc * vrxd + tg * gxd, uyd = dyd - Lc * vryd + tg * gyd, uzd = dzd - Lc * vrzd + tg * gzd;
    // FP32 from here
    float dx = (float)dxd, dy = (float)dyd, dz = (float)dzd;
    float vx = (float)q.v1.x, vy = (float)q.v1.y, vz = (float)q.v1.z;
    float inv_h = (float)inv_hd;
    float gx = (float)gxd, gy = (float)gyd, gz = (float)gzd;
    float ax = gx * inv_h, ay = gy * inv_h, az = gz * inv_h;  // zero out of history
    float df = (float)dfd;
    float ux = (float)uxd, uy = (float)uyd, uz = (float)uzd;
    float ex = dx - vx * dtr, ey = dy - vy * dtr, ez = dz - vz * dtr;  // eta
    float en = (float)L1d - cf * dtr;                                 // |eta| = c (t - t_r)
    ok = ok && en > 0.0f;
    float ien = __builtin_amdgcn_rcpf(en);
    float px = cf * ux * ien, py = cf * uy * ien, pz = cf * uz * ien;  // v' = c eta_hat - v_r
    float ev = ex * px + ey * py + ez * pz;                           // eta . v' = c |eta| kappa
    ok = ok && ev > 0.0f;
    float iev = __builtin_amdgcn_rcpf(ev);
    const float icn = ien * (float)ic;
    float hx = ex * icn, hy = ey * icn, hz = ez * icn;  // eta_hat / c
    // c^2 - |v_r|^2 from the FP64 value at v_1 plus the small correction
    float cv = C2 - df * (2.0f * (vx * gx + vy * gy + vz * gz) + df * (gx * gx + gy * gy + gz * gz));
    // eta x (v' x a) = v' (eta . a) - a (eta . v')
    float ea = ex * ax + ey * ay + ez * az;
    float pref = kq * en * (iev * iev * iev);
    float k1 = pref * (cv + ea), k2 = pref * ev;
    float Ex = k1 * px - k2 * ax;
    float Ey = k1 * py - k2 * ay;
    float Ez = k1 * pz - k2 * az;
    f[0] = Ex;
    f[1] = Ey;
    f[2] = Ez;
    // B = eta_hat x E / c
    f[3] = hy * Ez - hz * Ey;
    f[4] = hz * Ex - hx * Ez;
    f[5] = hx * Ey - hy * Ex;
    return ok;
}

}  // namespace

// NIT: -1, the tile buffer count read at run time; 0, two buffers known at
// compile time (D <= 2048); > 0, two buffers and the bisection unrolled for
// NIT halvings, ceil(log2(D - 1)) of the launch's depth (GUESS 0).
template <bool MIX, bool KSTAR, bool COUNT, int GUESS, int S, bool ADAPT, bool MID, int NIT = -1>
__device__ __forceinline__ void pair_body(const PairParams &p)
{
    extern __shared__ double4 lds[];
    // LDS address of the dynamic buffer (32-bit, for offset arithmetic)
    const uint32_t lds_base = (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)lds;
    const int D = p.D;
    const int tid = threadIdx.x;
    const int nbx = (int)((p.m + kBlockFp64 - 1) / kBlockFp64);
    int bxi, split;
    pair_block_coords(nbx, p.nsplit, bxi, split);
    const int64_t a = (int64_t)bxi * kBlockFp64 + tid;
    const bool active = a < p.m;
    const int64_t j0 = (int64_t)split * p.src_per_split;
    int64_t j1 = j0 + p.src_per_split;
    if (j1 > p.n_src)
        j1 = p.n_src;

    double rx = 0, ry = 0, rz = 0;
    double3 vt = make_double3(0.0, 0.0, 0.0);  // target's present velocity (adaptive step)
    double eta_min = __longlong_as_double((long long)kPosInfBits), dv2_max = 0.0;
    int64_t self = -1, tgt = a;  // tgt: index the outputs are written at
    if (active) {
        if (p.x) {
            rx = p.x[a];
            ry = p.x[p.m + a];
            rz = p.x[2 * p.m + a];
            self = p.self_index ? p.self_index[a] : -1;
        } else {
            tgt = p.order ? (int64_t)p.order[a] : a;
            double4 w = p.ring_w[tgt * D + p.head];
            rx = w.x;
            ry = w.y;
            rz = w.z;
            self = tgt;
            if (ADAPT) {
                double4 vn = p.ring_v[tgt * D + p.head];
                vt = make_double3(vn.x, vn.y, vn.z);
            }
        }
    }
    static_assert(!MIX || (!ADAPT && !MID && GUESS <= 3), "mixed precision: fixed step, no warm start");
    static_assert(NIT <= 0 || (GUESS == 0 && NIT <= 11), "an unrolled bisection has at most 11 halvings");
    // field sums: FP64 with Neumaier compensation, or FP32 with two-sum
    using Real = std::conditional_t<MIX, float, double>;
    Real sum[6] = {0, 0, 0, 0, 0, 0}, comp[6] = {0, 0, 0, 0, 0, 0};
    Real acc[6] = {0, 0, 0, 0, 0, 0};
    constexpr int kPlainRun = MIX ? 8 : 32;  // sources per plain partial
    const float kqf = (float)p.kq;
    int groups_in_acc = 0;
    int probes = 0, nbefore = 0, npairs = 0, nfall = 0, nresc = 0;
    // first (lowest) source of a failing pair; sources number below 2^31
    int32_t fail_j = INT32_MAX;
    const float inv_cdt = (float)(1.0 / (kC_LIGHT * p.dt));
    const int64_t grp_index = a >> p.g_shift;  // surrogate group of this target

    // LDS: nbuf tile buffers, then the light distance of every logical slot
    // (shared by all sources).  A buffer holds its TS * D records
    // {-2 D, A} of the split sign test (lightcone_record) as two arrays of
    // 16-byte halves, {-2 D_x, -2 D_y} then {-2 D_z, A}, hrec halves apart:
    // lanes that probe different slots then spread over twice as many LDS
    // bank groups as with 32-byte records.  With two buffers the distance is
    // the fixed kHalfRecs, so a probe's two reads share one address (the
    // second one at an immediate offset).
    const int nbuf = NIT >= 0 ? 2 : p.nbuf;
    // A staged tile holds G groups of S sources; the S sources of a group
    // are searched in lockstep, and one barrier per staged tile serves all
    // its groups.
    const int G = p.groups;
    const int TS = S * G;
    const int hrec = nbuf == 2 ? kHalfRecs : TS * D;
    double2 *const halves = reinterpret_cast<double2 *>(lds);
    double *Ls = reinterpret_cast<double *>(halves + nbuf * 2 * hrec);
    float4 *line = reinterpret_cast<float4 *>(Ls + ((D + 1) & ~1));
    float *gcorr = reinterpret_cast<float *>(line + 2 * 2 * 4);  // [buffer][wavefront][source]
    // newest samples w_n of the sources of three consecutive staged tiles
    // (tile i in slot i % 3), as {x, y}, {z, -}: written two tiles ahead of
    // the tile's search, read when its records are staged and searched
    double2 *wnr = reinterpret_cast<double2 *>(gcorr + 2 * (kBlockFp64 / 64) * 4);
    // slot table (NIT >= 0): for back offset b, the byte offset in a ring row
    // of physical slot (head - b) mod D and, above 16 bits, of the next newer
    // slot's (the bracket's two velocity records)
    constexpr bool kSlotTable = NIT >= 0;
    uint32_t *slot_off = reinterpret_cast<uint32_t *>(wnr + 3 * 4 * 2);
    auto write_wn = [&](int it_tile, int64_t jt, int ns) {
        if (tid < ns) {
            const double4 w = p.ring_w[(jt + tid) * D + p.head];
            wnr[((it_tile % 3) * 4 + tid) * 2] = make_double2(w.x, w.y);
            wnr[((it_tile % 3) * 4 + tid) * 2 + 1] = make_double2(w.z, 0.0);
        }
    };
    auto read_wn = [&](int it_tile, int s) {
        const double2 a = wnr[((it_tile % 3) * 4 + s) * 2], b = wnr[((it_tile % 3) * 4 + s) * 2 + 1];
        return make_double4(a.x, a.y, b.x, 0.0);
    };
    // guess mode 1: the surrogate's correction for groups of 64 or more
    // targets (whole wavefronts) is staged with the tile; mode 3: one
    // normalised delay per pair, read from the guess array
    const bool stage_g = GUESS == 1;
    struct TileView {
        const double2 *xy, *zl;
        __device__ double4 rec(int i) const
        {
            const double2 a = xy[i], b = zl[i];
            return make_double4(a.x, a.y, b.x, b.y);
        }
    };
    auto view = [&](int bi, int g) {
        const double2 *base = halves + bi * 2 * hrec + g * S * D;
        return TileView{base, base + hrec};
    };
    // the present time is the newest slot's (the clock lives in T)
    const double tnow = p.T[p.head];
    for (int b = tid; b < D; b += kBlockFp64) {
        int ph = p.head - b;
        ph += ph < 0 ? D : 0;
        Ls[b] = kC_LIGHT * (tnow - p.T[ph]);
        if constexpr (kSlotTable) {
            const int ph2 = ph + 1 == D ? 0 : ph + 1;  // back offset b - 1 (read for b >= 1)
            slot_off[b] = (uint32_t)ph * (uint32_t)sizeof(double4) | (uint32_t)ph2 * (uint32_t)sizeof(double4) << 16;
        }
    }
    // Record q of a tile: source q / D (q < TS D, TS <= 4), slot q % D.
    // The guided searches stage the pass's records written by
    // lightcone_records_kernel (the tile's ns sources' D records are
    // contiguous from p.rec[jt D]); the bisection, whose pass is bound by
    // latency rather than issue, computes them from the positions while
    // staging and saves the extra kernel.  What is loaded from HBM/L2 (a
    // record or a position) is prefetched into registers one tile ahead (the
    // first two of each thread), so its latency overlaps the previous tile's
    // work; deeper histories load the rest in place.
    constexpr bool kRecords = pass_uses_records(GUESS);
    auto src_of = [&](int q) { return (q >= D) + (q >= 2 * D) + (q >= 3 * D); };
    auto fetch = [&](int64_t jt, int ns, int q) -> double4 {
        double4 w = make_double4(0.0, 0.0, 0.0, 0.0);
        if constexpr (kRecords) {
            if (q < ns * D)
                w = p.rec[jt * D + q];
        } else {
            const int s = src_of(q);
            const int b = q - s * D;
            if (b < D && s < ns) {
                int ph = p.head - b;
                ph += ph < 0 ? D : 0;
                w = p.ring_w[(jt + s) * D + ph];
            }
        }
        return w;
    };
    auto put = [&](int bi, int it_tile, int ns, int q, double4 w) {
        if (q < ns * D) {
            double4 rec = w;
            if constexpr (!kRecords) {
                const int s = src_of(q);
                rec = lightcone_record(read_wn(it_tile, s), w, Ls[q - s * D]);
            }
            double2 *xy = halves + bi * 2 * hrec + q;
            xy[0] = make_double2(rec.x, rec.y);
            xy[hrec] = make_double2(rec.z, rec.w);
        }
    };
    auto stage = [&](int bi, int it_tile, int64_t jt, int ns, double4 r0, double4 r1) {
        if ((GUESS == 1 || GUESS == 2) && tid < ns) {
            // the source's newest velocity, for straight-line look-backs
            const double4 vn = p.ring_v[(jt + tid) * D + p.head];
            const double ic = 1.0 / kC_LIGHT;
            const double bx = vn.x * ic, by = vn.y * ic, bz = vn.z * ic;
            const double g2 = 1.0 - (bx * bx + by * by + bz * bz);
            line[(bi * 4 + tid) * 2] = make_float4((float)bx, (float)by, (float)bz, (float)g2);
            line[(bi * 4 + tid) * 2 + 1] = make_float4((float)(1.0 / g2), 0.0f, 0.0f, 0.0f);
        }
        if (stage_g && tid < (kBlockFp64 / 64) * 4) {
            const int w = tid >> 2, sj = tid & 3;
            const int64_t aw = (int64_t)bxi * kBlockFp64 + w * 64;
            if (sj < ns && aw < p.m)
                gcorr[(bi * (kBlockFp64 / 64) + w) * 4 + sj] = p.G[(jt + sj) * p.g_groups + (aw >> p.g_shift)];
        }
        put(bi, it_tile, ns, tid, r0);
        put(bi, it_tile, ns, tid + kBlockFp64, r1);
        for (int q = tid + 2 * kBlockFp64; q < ns * D; q += kBlockFp64)
            put(bi, it_tile, ns, q, fetch(jt, ns, q));
    };
    auto tile_size = [&](int64_t jt) { return (int)((j1 - jt) < TS ? (j1 - jt) : TS); };
    double4 pf0 = make_double4(0.0, 0.0, 0.0, 0.0), pf1 = pf0;
    if (j0 < j1) {
        pf0 = fetch(j0, tile_size(j0), tid);
        pf1 = fetch(j0, tile_size(j0), tid + kBlockFp64);
    }
    // Two buffers: tile i + 1 is written while tile i is searched, and one
    // barrier per tile both publishes tile i + 1 and retires tile i's
    // buffer for tile i + 2.  One buffer (deep histories): stage, then
    // search, with a barrier on either side.
    if (j0 < j1) {
        write_wn(0, j0, tile_size(j0));
        if (nbuf == 2 && j0 + TS < j1)
            write_wn(1, j0 + TS, tile_size(j0 + TS));
    }
    if (nbuf == 2 && j0 < j1) {
        __syncthreads();
        stage(0, 0, j0, tile_size(j0), pf0, pf1);
        if (j0 + TS < j1) {
            pf0 = fetch(j0 + TS, tile_size(j0 + TS), tid);
            pf1 = fetch(j0 + TS, tile_size(j0 + TS), tid + kBlockFp64);
        }
        __syncthreads();
    }
    // previous-step brackets of the next tile's sources (warm start)
    uint16_t knext[S], kcur[S];
    auto load_brackets = [&](int64_t jt) {
#pragma unroll
        for (int s = 0; s < S; ++s)
            knext[s] = active && jt + s < j1 ? p.kc[(jt + s) * p.m + a] : kBracketBefore;
    };
    if (GUESS == 4 && j0 < j1)
        load_brackets(j0);
    int it = 0;
    for (int64_t jts = j0; jts < j1; jts += TS, ++it) {
        const int cb = nbuf == 2 ? (it & 1) : 0;
        if (nbuf == 2) {
            if (jts + TS < j1) {
                stage(cb ^ 1, it + 1, jts + TS, tile_size(jts + TS), pf0, pf1);
                if (jts + 2 * TS < j1) {
                    pf0 = fetch(jts + 2 * TS, tile_size(jts + 2 * TS), tid);
                    pf1 = fetch(jts + 2 * TS, tile_size(jts + 2 * TS), tid + kBlockFp64);
                    write_wn(it + 2, jts + 2 * TS, tile_size(jts + 2 * TS));
                }
            }
        } else {
            __syncthreads();
            stage(0, it, jts, tile_size(jts), pf0, pf1);
            __syncthreads();
            if (jts + TS < j1) {
                pf0 = fetch(jts + TS, tile_size(jts + TS), tid);
                pf1 = fetch(jts + TS, tile_size(jts + TS), tid + kBlockFp64);
                write_wn(it + 1, jts + TS, tile_size(jts + TS));
            }
        }
      for (int grp = 0; grp < G && jts + grp * S < j1; ++grp) {
        const int64_t jt = jts + grp * S;
        const int ns = (int)((j1 - jt) < S ? (j1 - jt) : S);
        if (GUESS == 4) {
#pragma unroll
            for (int s = 0; s < S; ++s)
                kcur[s] = knext[s];
            if (jt + S < j1)
                load_brackets(jt + S);
        }
        const TileView cur = view(cb, grp);
        if (active) {
            bool valid[S];
            int64_t jj[S];
            int bk[S];
            // the target's offset d0 = r - w_n from each source's newest
            // sample, and |d0|^2 (the pair's part of the sign test)
            double d0x[S], d0y[S], d0z[S], R0[S];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                jj[s] = jt + (s < ns ? s : 0);
                valid[s] = s < ns && jj[s] != self;
                if (KSTAR && s < ns && jj[s] == self)
                    p.kstar[a * p.n_src + jj[s]] = 0;
                const double4 wn = read_wn(it, grp * S + s);
                d0x[s] = rx - wn.x;
                d0y[s] = ry - wn.y;
                d0z[s] = rz - wn.z;
                R0[s] = offset_sq(d0x[s], d0y[s], d0z[s]);
                // a target on the source's present position: eta = 0 (one
                // compare: |d0|^2 is 0 only when d0 is, for offsets above
                // 1e-154 m)
                if (valid[s] && R0[s] == 0.0) {
                    fail_j = min(fail_j, (int32_t)jj[s]);
                    valid[s] = false;
                }
            }
            auto inside_cone = [&](int s, double4 rec) { return lightcone_positive(rec, d0x[s], d0y[s], d0z[s], R0[s]); };

            // bracket velocity records (they carry 1/(t_2 - t_1)), root,
            // reconstruction, LW field and accumulation of tile source s
            auto load_v = [&](int s, int b, double4 &v1, double4 &v2) {
                const int bb = b < 0 ? D - 1 : b;
                uint32_t o1, o2;  // byte offsets of the two records in the source's row
                if constexpr (kSlotTable) {
                    const uint32_t w = slot_off[bb];
                    o1 = w & 0xffffu;
                    o2 = w >> 16;
                } else {
                    int ph1 = p.head - bb;
                    ph1 += ph1 < 0 ? D : 0;
                    const int ph2 = ph1 + 1 == D ? 0 : ph1 + 1;
                    o1 = (uint32_t)ph1 * (uint32_t)sizeof(double4);
                    o2 = (uint32_t)ph2 * (uint32_t)sizeof(double4);
                }
                // uniform row base plus 32-bit lane offsets
                const char *row = reinterpret_cast<const char *>(p.ring_v + jj[s] * D);
                v1 = *reinterpret_cast<const double4 *>(row + o1);
                // unused (inv_h = 0) out of history
                v2 = *reinterpret_cast<const double4 *>(row + o2);
            };
            auto finish = [&](int s, int b, double4 v1, double4 v2) {
                const bool before = b < 0;
                const int bb = before ? D - 1 : b;
                Real f[6];
                double en = 0.0;
                double3 vr = make_double3(0.0, 0.0, 0.0);
                bool ok;
                // r - w_1 = d0 + D from the staged -2 D
                const double4 r1 = cur.rec(s * D + bb);
                const double3 d1 = make_double3(__builtin_fma(-0.5, r1.x, d0x[s]), __builtin_fma(-0.5, r1.y, d0y[s]),
                                                __builtin_fma(-0.5, r1.z, d0z[s]));
                if constexpr (MIX) {
                    bool resc = false;
                    ok = lw_pair_mixed<GUESS == 0>(Ls[bb], MixedPair{d1, v1, v2}, before, kqf, f, resc);
                    if (COUNT && valid[s])
                        nresc += resc ? 1 : 0;
                } else {
                    double3 dw = make_double3(0.0, 0.0, 0.0);
                    if (MID) {
                        // w_2 - w_1 = D_1 - D_2 from the staged -2 D of both ends
                        const double4 r2 = cur.rec(s * D + (bb > 0 ? bb - 1 : 0));
                        dw = make_double3(-0.5 * (r1.x - r2.x), -0.5 * (r1.y - r2.y), -0.5 * (r1.z - r2.z));
                    }
                    ok = lw_pair(d1.x, d1.y, d1.z, Ls[bb], v1, v2, before, p.kq, f, en, vr, MID, dw);
                }
                if (valid[s]) {
                    if (ok) {
#pragma unroll
                        for (int k = 0; k < 6; ++k)
                            acc[k] += f[k];
                        if (ADAPT && en >= p.eta_allow) {
                            const double dx = vt.x - vr.x, dy = vt.y - vr.y, dz = vt.z - vr.z;
                            eta_min = fmin(eta_min, en);
                            dv2_max = fmax(dv2_max, dx * dx + dy * dy + dz * dz);
                        }
                    } else {
                        fail_j = min(fail_j, (int32_t)jj[s]);
                    }
                    if (KSTAR)
                        p.kstar[a * p.n_src + jj[s]] = before ? -1 : b;
                    if (COUNT) {
                        npairs += 1;
                        nbefore += before ? 1 : 0;
                    }
                }
            };

            if (GUESS == 0 || GUESS >= 4) {
                if (GUESS != 4) {
                    // The paper's search: oldest sample first, then bisection
                    // of the whole history; a fixed number of halvings keeps
                    // the S searches in lockstep (extra halvings of a one-step
                    // bracket change nothing).
                    bool inside[S];
                    // LDS byte address of the record of xb: f(xb) <= 0, the
                    // bracket lies in (xb, xb + n]
                    uint32_t xo[S];
                    // LDS byte address of the group's first record (its first half)
                    const uint32_t xy0 =
                        lds_base + (uint32_t)(cb * 2 * hrec + grp * S * D) * (uint32_t)sizeof(double2);
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        inside[s] = inside_cone(s, cur.rec(s * D + D - 1));
                        xo[s] = xy0 + (uint32_t)(s * D) * (uint32_t)sizeof(double2);
                    }
                    bool any = false;
#pragma unroll
                    for (int s = 0; s < S; ++s)
                        any = any || (inside[s] && valid[s]);
                    // one halving of width n: probe xb + floor(n / 2)
                    auto probe = [&](int half, auto zl_off) {
                        const uint32_t hb = (uint32_t)half * (uint32_t)sizeof(double2);
#pragma unroll
                        for (int s = 0; s < S; ++s) {
                            const uint32_t mo = xo[s] + hb;
                            typedef double dv2 __attribute__((ext_vector_type(2)));
                            const dv2 va = *(const __attribute__((address_space(3))) dv2 *)(uintptr_t)mo;
                            const dv2 vb =
                                *(const __attribute__((address_space(3))) dv2 *)(uintptr_t)(mo + (uint32_t)zl_off);
                            const double4 rec = make_double4(va.x, va.y, vb.x, vb.y);
                            xo[s] = inside_cone(s, rec) ? xo[s] : mo;
                        }
                    };
                    // The halving widths n = D - 1, n - floor(n / 2), ...
                    // depend on D only (uniform across lanes).  With the
                    // number of halvings known at compile time (NIT) the
                    // sequence is unrolled: no loop compare or branch per
                    // probe, the same probes as the loop.
                    auto halve = [&](auto zl_off) {
                        int n = D - 1;
                        if constexpr (NIT > 0) {
#pragma unroll
                            for (int k = 0; k < NIT; ++k) {
                                const int half = n >> 1;
                                probe(half, zl_off);
                                n -= half;
                            }
                        } else {
                            while (n > 1) {
                                const int half = n >> 1;
                                probe(half, zl_off);
                                n -= half;
                            }
                        }
                    };
                    if (__any(any)) {
                        if (nbuf == 2)
                            halve(std::integral_constant<uint32_t, kHalfRecs * sizeof(double2)>{});
                        else
                            halve((uint32_t)hrec * (uint32_t)sizeof(double2));
                    }
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        bk[s] = inside[s] ? (int)((xo[s] - xy0) / (uint32_t)sizeof(double2)) - s * D + 1 : -1;
                        if (COUNT && valid[s])
                            probes += inside[s] ? 1 + p.nit : 1;
                    }
                } else {
                    // Warm start from the previous step's bracket (back
                    // offsets are relative to the newest slot, so a pair
                    // whose geometry is unchanged keeps its value): confirm
                    // it with the two samples that define it, issued
                    // together for the S sources; a pair whose bracket moved
                    // gallops from the old one.
                    bool hit[S];
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        const int g = kcur[s];
                        const bool was_before = g == kBracketBefore;
                        const bool in_range = g >= 1 && g < D;
                        const int ga = in_range ? g : D - 1;  // 1 <= ga <= D - 1
                        const bool fa = inside_cone(s, cur.rec(s * D + ga));
                        const bool fb = inside_cone(s, cur.rec(s * D + ga - 1));
                        hit[s] = was_before ? !fa : (in_range && fa && !fb);
                        // a bracket index leaves this block only if it is
                        // one (the entry of an excluded pair is never
                        // written and may hold anything)
                        bk[s] = in_range ? g : -1;
                        if (COUNT && valid[s])
                            probes += was_before || g == 1 ? 1 : 2;
                    }
                    for (int s = 0; s < S; ++s) {
                        if (!hit[s] && valid[s]) {
                            auto test = [&](int bb) { return inside_cone(s, cur.rec(s * D + bb)); };
                            const int g = kcur[s];
                            int fb = 0;
                            bk[s] = search_guided(test, D, g == kBracketBefore || g >= D ? (float)(D - 1) : (float)g, 6,
                                                  probes, fb);
                            nfall += fb;
                        }
                    }
                }
                if (GUESS >= 4) {
#pragma unroll
                    for (int s = 0; s < S; ++s)
                        if (valid[s])
                            p.kc[jj[s] * p.m + a] = bk[s] < 0 ? kBracketBefore : (uint16_t)bk[s];
                }
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    double4 v1, v2;
                    load_v(s, bk[s], v1, v2);
                    finish(s, bk[s], v1, v2);
                }
            } else {
                // guided searches, one source at a time
#pragma unroll
                for (int s = 0; s < S; ++s) {
                    int b = -1;
                    if (valid[s]) {
                        auto test = [&](int bb) { return inside_cone(s, cur.rec(s * D + bb)); };
                        const float Rx = (float)d0x[s], Ry = (float)d0y[s], Rz = (float)d0z[s];
                        const float r2 = Rx * Rx + Ry * Ry + Rz * Rz;
                        float g;
                        if (GUESS == 1 || GUESS == 2) {
                            // straight-line look-back: with beta the source's
                            // newest velocity / c, the positive root of
                            // (1 - beta^2) s^2 - 2 (R.beta) s - R^2 = 0
                            const float4 l0 = line[(cb * 4 + grp * S + s) * 2];
                            const float ig2 = line[(cb * 4 + grp * S + s) * 2 + 1].x;
                            const float rb = Rx * l0.x + Ry * l0.y + Rz * l0.z;
                            g = (rb + __builtin_amdgcn_sqrtf(__builtin_fmaf(rb, rb, l0.w * r2))) * ig2 * inv_cdt;
                            // surrogate, one evaluation per group: the group's
                            // correction factor to straight-line motion
                            if (GUESS == 1)
                                g *= gcorr[(cb * (kBlockFp64 / 64) + (tid >> 6)) * 4 + grp * S + s];
                        } else {
                            // surrogate per pair: predicted c (t - t_r) / |r - w_n| times the distance
                            float gh = p.G[jj[s] * p.g_groups + grp_index];
                            g = gh * __builtin_amdgcn_sqrtf(r2) * inv_cdt;
                        }
                        int fb = 0;
                        b = search_guided(test, D, g, 6, probes, fb);
                        nfall += fb;
                    }
                    double4 v1, v2;
                    load_v(s, b, v1, v2);
                    finish(s, b, v1, v2);
                }
            }
        }
        // plain partial sums over kPlainRun sources, then one compensated
        // merge (the same cadence for every search mode: results are
        // bit-identical)
        if (++groups_in_acc * S == kPlainRun) {
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                if constexpr (MIX)
                    two_sum(sum[k], comp[k], acc[k]);
                else
                    neumaier(sum[k], comp[k], acc[k]);
                acc[k] = 0;
            }
            groups_in_acc = 0;
        }
      }
        if (nbuf == 2)
            __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        if constexpr (MIX)
            two_sum(sum[k], comp[k], acc[k]);
        else
            neumaier(sum[k], comp[k], acc[k]);
    }
    if (active) {
        // partials in the launch's target order (consecutive threads write
        // consecutive entries); the merge maps them to particle indices
        double *out = p.part + (int64_t)split * 12 * p.m + a;
        for (int k = 0; k < 6; ++k) {
            out[k * p.m] = (double)sum[k];
            out[(6 + k) * p.m] = (double)comp[k];
        }
        if (fail_j != INT32_MAX)
            report_error(p.err, tgt, fail_j, kErrCoincident);
    }
    if (ADAPT) {
        // one atomic pair per wavefront
        for (int off = 32; off > 0; off >>= 1) {
            eta_min = fmin(eta_min, __shfl_xor(eta_min, off));
            dv2_max = fmax(dv2_max, __shfl_xor(dv2_max, off));
        }
        if ((tid & 63) == 0) {
            atomicMin(&p.ad[0], (unsigned long long)__double_as_longlong(eta_min));
            atomicMax(&p.ad[1], (unsigned long long)__double_as_longlong(dv2_max));
        }
    }
    if (COUNT) {
        // one atomic per wavefront
        unsigned long long c0 = npairs, c1 = nbefore, c2 = probes, c3 = nfall, c4 = nresc;
        for (int off = 32; off > 0; off >>= 1) {
            c0 += __shfl_down(c0, off);
            c1 += __shfl_down(c1, off);
            c2 += __shfl_down(c2, off);
            c3 += __shfl_down(c3, off);
            c4 += __shfl_down(c4, off);
        }
        if ((tid & 63) == 0) {
            atomicAdd(&p.counters[0], c0);
            atomicAdd(&p.counters[1], c1);
            atomicAdd(&p.counters[2], c2);
            atomicAdd(&p.counters[4], c3);
            if (MIX)
                atomicAdd(&p.counters[3], c4);
        }
    }
}

}  // namespace empp
