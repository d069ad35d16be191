// pair_common.h -- light-cone sign test and history searches used by the
// pair kernels (Sec. 2.2 of arXiv 2605.05543).
#pragma once

#include "empp_dev.h"

namespace empp {

// Light-cone sign of a stored sample (Sec. 2.2), split into a part of the
// sample and a part of the pair.  With the source's newest sample w_n, the
// target's offset d0 = r - w_n and the sample's offset D = w_n - w_k,
// |r - w_k|^2 = |d0|^2 + 2 d0.D + |D|^2, so with L = c (t - T_k)
//   f_k > 0  <=>  A - 2 d0.D > |d0|^2,   A = L^2 - |D|^2.
// The staged record of a sample is {-2 D, A}; a test is then three fused
// multiply-adds and a compare.  Every step is one rounding in a fixed
// order (A = L*L, minus D_x^2, D_y^2, D_z^2 by FMA; q = A plus d0_x (-2 D_x),
// y, z by FMA; |d0|^2 = d0_x^2 plus d0_y^2, d0_z^2 by FMA), the same
// decision as the CPU reference of the method.
__device__ inline double4 lightcone_record(double4 wn, double4 wk, double L)
{
    const double Dx = wn.x - wk.x, Dy = wn.y - wk.y, Dz = wn.z - wk.z;
    double A = L * L;
    A = __builtin_fma(-Dx, Dx, A);
    A = __builtin_fma(-Dy, Dy, A);
    A = __builtin_fma(-Dz, Dz, A);
    return make_double4(-2.0 * Dx, -2.0 * Dy, -2.0 * Dz, A);
}

__device__ inline double offset_sq(double d0x, double d0y, double d0z)
{
    double R = d0x * d0x;
    R = __builtin_fma(d0y, d0y, R);
    return __builtin_fma(d0z, d0z, R);
}

__device__ inline bool lightcone_positive(double4 rec, double d0x, double d0y, double d0z, double R0sq)
{
    double q = __builtin_fma(d0x, rec.x, rec.w);
    q = __builtin_fma(d0y, rec.y, q);
    q = __builtin_fma(d0z, rec.z, q);
    return q > R0sq;
}

// Bisection of the paper: test the oldest sample first (if it is not
// inside the past light cone the retarded time precedes the history);
// otherwise halve [oldest, newest] until the bracket is one step wide.
// Works in "back" offsets b (0 = newest).  Because f_k decreases strictly
// along the history, the bracket found is the unique one:
// b* = min { b : f_b > 0 }.  Returns b* or -1 (before the history).
template <typename Test>
__device__ __forceinline__ int search_bisect(Test test, int D, int &probes)
{
    probes += 1;
    if (!test(D - 1))
        return -1;
    int lo = D - 1, hi = 0;  // f(lo) > 0, f(hi) <= 0 (newest: t - T = 0)
    while (lo - hi > 1) {
        int mid = (lo + hi) >> 1;
        probes += 1;
        if (test(mid))
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Guided search: start at a guessed back offset g and test g and g-1
// together (both loads in flight at once); when the guess is right this is
// the whole search.  Otherwise gallop (1, 2, 4, ... slots) towards the
// bracket and bisect inside the last gallop step.  Reaches the same b* as
// search_bisect for any guess.  A non-finite guess or more than
// max_gallop doublings falls back to plain bisection of what is left
// (counted in fallbacks).
template <typename Test>
__device__ __forceinline__ int search_guided(Test test, int D, float guess, int max_gallop, int &probes, int &fallback)
{
    if (!(guess == guess) || !(fabsf(guess) < 1e9f)) {
        fallback = 1;
        return search_bisect(test, D, probes);
    }
    int g = (int)ceilf(guess);
    g = g < 1 ? 1 : (g > D - 1 ? D - 1 : g);
    const bool fg = test(g);
    const bool fg1 = g > 1 && test(g - 1);  // b = 0 is never inside
    probes += g > 1 ? 2 : 1;
    if (fg && !fg1)
        return g;
    int lo, hi;  // f(lo) > 0 (older side), f(hi) <= 0 (newer side)
    if (fg) {
        lo = g - 1;
        hi = 0;
        int step = 1, n = 0;
        while (true) {
            int cand = lo - step;
            if (cand <= 0)
                break;  // hi = 0 (newest sample is never inside)
            probes += 1;
            if (test(cand)) {
                lo = cand;
            } else {
                hi = cand;
                break;
            }
            step <<= 1;
            if (++n > max_gallop) {
                fallback = 1;
                break;  // bisect the rest of [hi=0, lo]
            }
        }
    } else {
        hi = g;
        lo = -1;
        int step = 1, n = 0;
        while (true) {
            int cand = hi + step;
            if (cand >= D - 1 || n >= max_gallop) {
                if (n >= max_gallop)
                    fallback = 1;
                if (hi == D - 1)
                    return -1;  // the oldest sample was the guess
                probes += 1;
                if (test(D - 1))
                    lo = D - 1;
                else
                    return -1;
                break;
            }
            probes += 1;
            if (test(cand)) {
                lo = cand;
                break;
            }
            hi = cand;
            step <<= 1;
            ++n;
        }
    }
    while (lo - hi > 1) {
        int mid = (lo + hi) >> 1;
        probes += 1;
        if (test(mid))
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

}  // namespace empp
