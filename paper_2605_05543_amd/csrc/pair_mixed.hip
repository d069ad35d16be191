// pair_mixed.hip -- mixed-precision all-pairs Lienard-Wiechert evaluation
// (Secs. 2.1-2.2 of arXiv 2605.05543 with the precision split below).
//
// The pass is the FP64 kernel's (pair_body in pair_kernel.h): the same
// LDS-staged FP64 history tiles and the same FP64 sign tests, so the bracket
// index is bit-identical to the FP64 path.  On gfx950 an FP32 and an FP64
// vector instruction issue at the same rate, so FP32 sign tests (which need
// a rounding band and an FP64 re-test inside it) would cost more than the
// exact test they stand in for.  The precision split is in the field
// evaluation of each pair (lw_pair_mixed):
//  * FP64: the offset r - w_1 to the bracket sample, the light-cone residual
//    at the root C0 = L1^2 - |r - w_1|^2 and the other coefficients of the
//    quadratic, the velocity at the root, the vector eta - |eta| v/c whose
//    length is the cancellation-prone 1 - eta_hat.beta, and the root
//    whenever the FP32 root fails its residual test (a rescue);
//  * FP32: the root, the reconstruction and the LW terms; the field sum is
//    accumulated with Knuth's two-sum into an FP32 (sum, error) pair.
#include "pair_kernel.h"

namespace empp {

extern const bool kHaveMixed = true;

template <bool KSTAR, bool COUNT, int GUESS, int S, int NIT = -1>
__global__ __launch_bounds__(kBlockFp64, 4) void pair_mixed_kernel(PairParams p)
{
    pair_body<true, KSTAR, COUNT, GUESS, S, false, false, NIT>(p);
}

namespace {

template <bool K, bool C, int G, int S, int NIT = -1>
void launch_one(PairParams p, int staged, size_t lds, dim3 grid, hipStream_t stream)
{
    p.tile = S;
    p.groups = staged / S;
    if (NIT >= 0)
        lds = pair_lds_bytes(p.D, staged, true);
    if (lds > 65536)
        (void)hipFuncSetAttribute((const void *)pair_mixed_kernel<K, C, G, S, NIT>,
                                  hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((pair_mixed_kernel<K, C, G, S, NIT>), grid, dim3(kBlockFp64), lds, stream, p);
}

// The bisection with its halvings unrolled for the launch's depth (no
// bracket output, no counters) where the tiles are double-buffered
// (D <= 2048); deeper histories loop.
void launch_plain(const PairParams &p, int staged, size_t lds, dim3 grid, hipStream_t stream)
{
    static_assert(lockstep_sources(true, 0) == 1, "the bisection searches one source at a time");
    switch (p.nbuf == 2 ? p.nit : 0) {
#define EMPP_NIT(N) \
    case N: launch_one<false, false, 0, 1, N>(p, staged, lds, grid, stream); return;
        EMPP_NIT(1) EMPP_NIT(2) EMPP_NIT(3) EMPP_NIT(4) EMPP_NIT(5) EMPP_NIT(6)
        EMPP_NIT(7) EMPP_NIT(8) EMPP_NIT(9) EMPP_NIT(10) EMPP_NIT(11)
#undef EMPP_NIT
    default: launch_one<false, false, 0, 1, -1>(p, staged, lds, grid, stream);
    }
}

// Guided fields launches over double-buffered tiles take the kernel with
// the buffer count fixed at compile time.
template <bool K, bool C, int G, int S>
void launch_tiles(const PairParams &p, int staged, size_t lds, dim3 grid, hipStream_t stream)
{
    if constexpr (!K && !C && G >= 1) {
        if (p.nbuf == 2) {
            launch_one<K, C, G, S, 0>(p, staged, lds, grid, stream);
            return;
        }
    }
    launch_one<K, C, G, S>(p, staged, lds, grid, stream);
}

template <bool K, bool C, int G>
void launch_mode(const PairParams &p, int staged, size_t lds, dim3 grid, hipStream_t stream)
{
    if constexpr (lockstep_sources(true, G) == 2) {
        if (staged >= 2) {
            launch_tiles<K, C, G, 2>(p, staged, lds, grid, stream);
            return;
        }
    }
    launch_tiles<K, C, G, 1>(p, staged, lds, grid, stream);
}

}  // namespace

hipError_t launch_pair_mixed(const PairParams &p0, hipStream_t stream, bool kstar, bool count)
{
    PairParams p = p0;
    if (p.guess > 3 || p.ad || p.recon == 1)
        return hipErrorInvalidValue;  // fixed step, no warm start, linear reconstruction
    const int staged = pair_staged_tile(p.D);
    p.nbuf = pair_nbuf(p.D, staged);
    const int64_t nblocks = (p.m + kBlockFp64 - 1) / kBlockFp64 * p.nsplit;
    if (nblocks < 1 || nblocks > INT32_MAX)
        return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)nblocks);
    const size_t lds = pair_lds_bytes(p.D, staged);
#define EMPP_BY_GUESS(K, C)                                                                                  \
    do {                                                                                                    \
        if (p.guess == 3) launch_mode<K, C, 3>(p, staged, lds, grid, stream);                                \
        else if (p.guess == 2) launch_mode<K, C, 2>(p, staged, lds, grid, stream);                           \
        else if (p.guess == 1) launch_mode<K, C, 1>(p, staged, lds, grid, stream);                           \
        else launch_mode<K, C, 0>(p, staged, lds, grid, stream);                                             \
    } while (0)
    if (!kstar && !count && p.guess == 0) {
        launch_plain(p, staged, lds, grid, stream);
    } else if (kstar) {
        if (count) EMPP_BY_GUESS(true, true); else EMPP_BY_GUESS(true, false);
    } else {
        if (count) EMPP_BY_GUESS(false, true); else EMPP_BY_GUESS(false, false);
    }
#undef EMPP_BY_GUESS
    return hipGetLastError();
}

}  // namespace empp
