// pair_common.h -- light-cone sign test and history searches used by the
// pair kernels (Sec. 2.2 of arXiv 2605.05543).
#pragma once

#include "empp_dev.h"

namespace empp {

// Staged history record of one source at one logical slot:
// {x, y, z, L2} with L2 = L*L (rounded once), L = c (t - T_k) the light
// distance back to the slot.  The sign test f_k > 0 is
// L2 - dx*dx - dy*dy - dz*dz > 0 with the three squares taken off by fused
// multiply-adds in the order x, y, z: one rounding per step, the same
// decision as any IEEE evaluation of that expression.
__device__ inline bool lightcone_positive(double4 rec, double rx, double ry, double rz)
{
    double dx = rx - rec.x;
    double dy = ry - rec.y;
    double dz = rz - rec.z;
    double q = __builtin_fma(-dx, dx, rec.w);
    q = __builtin_fma(-dy, dy, q);
    q = __builtin_fma(-dz, dz, q);
    return q > 0.0;
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
