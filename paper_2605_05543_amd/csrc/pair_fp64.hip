// pair_fp64.hip -- all-pairs Lienard-Wiechert field evaluation in double
// precision (Secs. 2.1-2.2 of arXiv 2605.05543): the plain path, its
// adaptive-step reductions, the warm-started search and the midpoint
// ablation.  The pass itself is pair_body in pair_kernel.h.
#include "pair_kernel.h"

namespace empp {

template <bool KSTAR, bool COUNT, int GUESS, int S, bool ADAPT, bool MID = false>
__global__ __launch_bounds__(kBlockFp64, 4) void pair_fp64_kernel(PairParams p)
{
    pair_body<false, KSTAR, COUNT, GUESS, S, ADAPT, MID>(p);
}

// Sources per staged LDS tile (used to size the source chunks).
int pair_fp64_tile(int D) { return pair_staged_tile(D); }

// Host-side launcher (called from the C ABI layer).
hipError_t launch_pair_fp64(const PairParams &p0, hipStream_t stream, bool kstar, bool count)
{
    PairParams p = p0;
    const int staged = pair_staged_tile(p.D);
    p.tile = kLockstep;
    p.groups = staged / kLockstep;
    p.nbuf = pair_nbuf(p.D, staged);
    const int64_t nblocks = (p.m + kBlockFp64 - 1) / kBlockFp64 * p.nsplit;
    if (nblocks < 1 || nblocks > INT32_MAX)
        return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)nblocks);
    size_t lds = pair_lds_bytes(p.D, staged);
#define EMPP_LAUNCH(K, C, G, S, A)                                                                           \
    do {                                                                                                    \
        if (lds > 65536)                                                                                    \
            (void)hipFuncSetAttribute((const void *)pair_fp64_kernel<K, C, G, S, A>,                        \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                \
        hipLaunchKernelGGL((pair_fp64_kernel<K, C, G, S, A>), grid, dim3(kBlockFp64), lds, stream, p);          \
    } while (0)
#define EMPP_LAUNCH_MID(K)                                                                                   \
    do {                                                                                                    \
        if (lds > 65536)                                                                                    \
            (void)hipFuncSetAttribute((const void *)pair_fp64_kernel<K, false, 0, 1, false, true>,          \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                \
        hipLaunchKernelGGL((pair_fp64_kernel<K, false, 0, 1, false, true>), grid, dim3(kBlockFp64), lds, stream, p); \
    } while (0)
#define EMPP_BY_TILE(K, C, G, A) EMPP_LAUNCH(K, C, G, kLockstep, A)
#define EMPP_BY_ADAPT(C, G) \
    do { if (p.ad) EMPP_LAUNCH(false, C, G, 1, true); else EMPP_BY_TILE(false, C, G, false); } while (0)
    if (p.ad && (kstar || p.x || p.guess == 1 || p.guess == 3))
        return hipErrorInvalidValue;  // the adaptive step is taken in step mode
    if (p.recon == 1) {
        // midpoint ablation: the paper's bisection, fixed step, any target mode
        if (p.ad || count)
            return hipErrorInvalidValue;
        if (kstar)
            EMPP_LAUNCH_MID(true);
        else
            EMPP_LAUNCH_MID(false);
        return hipGetLastError();
    }
    if (p.guess == 4) {
        // warm start: step mode only (no per-pair k* output); the first
        // step of a run bisects and fills the cache (search mode 5)
        if (kstar || !p.kc || p.x)
            return hipErrorInvalidValue;
        if (p.kc_cold) {
            if (count) EMPP_BY_ADAPT(true, 5); else EMPP_BY_ADAPT(false, 5);
        } else {
            if (count) EMPP_BY_ADAPT(true, 4); else EMPP_BY_ADAPT(false, 4);
        }
    } else if (kstar) {
        if (p.guess == 2) {
            if (count) EMPP_BY_TILE(true, true, 2, false); else EMPP_BY_TILE(true, false, 2, false);
        } else if (p.guess == 3) {
            if (count) EMPP_BY_TILE(true, true, 3, false); else EMPP_BY_TILE(true, false, 3, false);
        } else if (p.guess == 1) {
            if (count) EMPP_BY_TILE(true, true, 1, false); else EMPP_BY_TILE(true, false, 1, false);
        } else {
            if (count) EMPP_BY_TILE(true, true, 0, false); else EMPP_BY_TILE(true, false, 0, false);
        }
    } else if (p.guess == 3) {
        if (count) EMPP_BY_TILE(false, true, 3, false); else EMPP_BY_TILE(false, false, 3, false);
    } else if (p.guess == 1) {
        if (count) EMPP_BY_TILE(false, true, 1, false); else EMPP_BY_TILE(false, false, 1, false);
    } else if (p.guess == 2) {
        if (count) EMPP_BY_ADAPT(true, 2); else EMPP_BY_ADAPT(false, 2);
    } else {
        if (count) EMPP_BY_ADAPT(true, 0); else EMPP_BY_ADAPT(false, 0);
    }
#undef EMPP_BY_ADAPT
#undef EMPP_LAUNCH_MID
#undef EMPP_BY_TILE
#undef EMPP_LAUNCH
    return hipGetLastError();
}

}  // namespace empp
