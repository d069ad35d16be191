// pair_fp64.hip -- all-pairs Lienard-Wiechert field evaluation in double
// precision (Secs. 2.1-2.2 of arXiv 2605.05543): the plain path, its
// adaptive-step reductions, the warm-started search and the midpoint
// ablation.  The pass itself is pair_body in pair_kernel.h.
#include "pair_kernel.h"

namespace empp {

template <bool KSTAR, bool COUNT, int GUESS, int S, bool ADAPT, bool MID = false, int NIT = -1>
__global__ __launch_bounds__(kBlockFp64, 4) void pair_fp64_kernel(PairParams p)
{
    pair_body<false, KSTAR, COUNT, GUESS, S, ADAPT, MID, NIT>(p);
}

// Sources per staged LDS tile (used to size the source chunks).
int pair_fp64_tile(int D) { return pair_staged_tile(D); }

namespace {

// One launch of a kernel instantiation: S sources per lockstep group,
// staged / S groups per staged LDS tile.
template <bool K, bool C, int G, int S, bool A, bool MID = false, int NIT = -1>
void launch_one(PairParams p, int staged, size_t lds, dim3 grid, hipStream_t stream)
{
    p.tile = S;
    p.groups = staged / S;
    if (NIT >= 0)
        lds = pair_lds_bytes(p.D, staged, true);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)pair_fp64_kernel<K, C, G, S, A, MID, NIT>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((pair_fp64_kernel<K, C, G, S, A, MID, NIT>), grid, dim3(kBlockFp64), lds, stream, p);
}

// The plain bisection with its halvings unrolled for the launch's depth
// (the fields path: no bracket output, no counters; fixed or adaptive step)
// where the tiles are double-buffered (D <= 2048); deeper histories loop.
template <bool A>
void launch_plain(const PairParams &p, int staged, size_t lds, dim3 grid, hipStream_t stream)
{
    switch (p.nbuf == 2 ? p.nit : 0) {
#define EMPP_NIT(N) \
    case N: launch_one<false, false, 0, 1, A, false, N>(p, staged, lds, grid, stream); return;
        EMPP_NIT(1) EMPP_NIT(2) EMPP_NIT(3) EMPP_NIT(4) EMPP_NIT(5) EMPP_NIT(6)
        EMPP_NIT(7) EMPP_NIT(8) EMPP_NIT(9) EMPP_NIT(10) EMPP_NIT(11)
#undef EMPP_NIT
    default: launch_one<false, false, 0, 1, A, false, -1>(p, staged, lds, grid, stream);
    }
}

// Guided fields launches over double-buffered tiles take the kernel with
// the buffer count fixed at compile time.
template <bool K, bool C, int G, int S, bool A>
void launch_tiles(const PairParams &p, int staged, size_t lds, dim3 grid, hipStream_t stream)
{
    if constexpr (!K && !C && !A && G >= 1 && G <= 4) {
        if (p.nbuf == 2) {
            launch_one<K, C, G, S, A, false, 0>(p, staged, lds, grid, stream);
            return;
        }
    }
    launch_one<K, C, G, S, A>(p, staged, lds, grid, stream);
}

// The lockstep width the search mode measured fastest with, where a staged
// tile holds two sources; the adaptive reductions use one.
template <bool K, bool C, int G, bool A>
void launch_mode(const PairParams &p, int staged, size_t lds, dim3 grid, hipStream_t stream)
{
    if constexpr (!A && lockstep_sources(false, G) == 2) {
        if (staged >= 2) {
            launch_tiles<K, C, G, 2, A>(p, staged, lds, grid, stream);
            return;
        }
    }
    launch_tiles<K, C, G, 1, A>(p, staged, lds, grid, stream);
}

}  // namespace

// Host-side launcher (called from the C ABI layer).
hipError_t launch_pair_fp64(const PairParams &p0, hipStream_t stream, bool kstar, bool count)
{
    PairParams p = p0;
    const int staged = pair_staged_tile(p.D);
    p.nbuf = pair_nbuf(p.D, staged);
    const int64_t nblocks = (p.m + kBlockFp64 - 1) / kBlockFp64 * p.nsplit;
    if (nblocks < 1 || nblocks > INT32_MAX)
        return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)nblocks);
    const size_t lds = pair_lds_bytes(p.D, staged);
#define EMPP_MODE(K, C, G, A) launch_mode<K, C, G, A>(p, staged, lds, grid, stream)
#define EMPP_BY_ADAPT(C, G) \
    do { if (p.ad) EMPP_MODE(false, C, G, true); else EMPP_MODE(false, C, G, false); } while (0)
    if (p.ad && (kstar || p.x || p.guess == 1 || p.guess == 3))
        return hipErrorInvalidValue;  // the adaptive step is taken in step mode
    if (p.recon == 1) {
        // midpoint ablation: the paper's bisection, fixed step, any target mode
        if (p.ad || count)
            return hipErrorInvalidValue;
        if (kstar)
            launch_one<true, false, 0, 1, false, true>(p, staged, lds, grid, stream);
        else
            launch_one<false, false, 0, 1, false, true>(p, staged, lds, grid, stream);
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
            if (count) EMPP_MODE(true, true, 2, false); else EMPP_MODE(true, false, 2, false);
        } else if (p.guess == 3) {
            if (count) EMPP_MODE(true, true, 3, false); else EMPP_MODE(true, false, 3, false);
        } else if (p.guess == 1) {
            if (count) EMPP_MODE(true, true, 1, false); else EMPP_MODE(true, false, 1, false);
        } else {
            if (count) EMPP_MODE(true, true, 0, false); else EMPP_MODE(true, false, 0, false);
        }
    } else if (p.guess == 3) {
        if (count) EMPP_MODE(false, true, 3, false); else EMPP_MODE(false, false, 3, false);
    } else if (p.guess == 1) {
        if (count) EMPP_MODE(false, true, 1, false); else EMPP_MODE(false, false, 1, false);
    } else if (p.guess == 2) {
        if (count) EMPP_BY_ADAPT(true, 2); else EMPP_BY_ADAPT(false, 2);
    } else if (count) {
        EMPP_BY_ADAPT(true, 0);
    } else {
        static_assert(lockstep_sources(false, 0) == 1, "the plain bisection searches one source at a time");
        if (p.ad)
            launch_plain<true>(p, staged, lds, grid, stream);
        else
            launch_plain<false>(p, staged, lds, grid, stream);
    }
#undef EMPP_BY_ADAPT
#undef EMPP_MODE
    return hipGetLastError();
}

}  // namespace empp
