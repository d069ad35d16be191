// mlp_dev.h -- shapes and device structures of the retarded-delay
// surrogate network (10 -> 128 -> 128 -> 1, SiLU).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace empp {

constexpr int kIn = 10;
constexpr int kHid = 128;
// flat parameter vector: W1[128][10], b1[128], W2[128][128], b2[128], W3[128], b3
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kHid * kIn;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid;
constexpr int kParams = kOffB3 + 1;  // 18049
// blocks of a training launch at most; its barrier buffer holds the
// arrival counter and one flag per block, each in a line of kSyncLine u64
constexpr int kSyncMaxBlocks = 512;
constexpr int kSyncLine = 16;
// a block's partial gradient: kParams values and its sum of squared
// residuals, padded to whole 16-byte units
constexpr int kPartStride = (kParams + 1 + 3) & ~3;

// Slot order of the 128-deep products (16x16x32 matrix-core steps): in each
// block of 32 columns, stored column 8 g + r holds column 4 g + r (r < 4)
// or 16 + 4 g + r - 4 (r >= 4), the rows that lane group g holds of two
// stacked 16-row activation tiles.
__host__ __device__ constexpr int col_of_slot(int q)
{
    const int b = q & ~31, w = q & 31, g = w >> 3, r = w & 7;
    return b + (r < 4 ? 4 * g + r : 12 + 4 * g + r);
}
__host__ __device__ constexpr int slot_of_col(int k)
{
    const int b = k & ~31, w = k & 31, u = w & 15;
    return b + 8 * (u >> 2) + (u & 3) + 4 * (w >> 4);
}
__host__ __device__ constexpr bool slot_order_is_a_permutation()
{
    for (int q = 0; q < 128; ++q)
        if (slot_of_col(col_of_slot(q)) != q || col_of_slot(q) < 0 || col_of_slot(q) >= 128)
            return false;
    return true;
}
static_assert(slot_order_is_a_permutation(), "slot order must be a permutation of 0..127");

// Network as the kernels read it: bf16 matrices (W1 padded to 16 inputs,
// W2 and its transpose with their columns in slot order), bf16-rounded
// vectors stored as floats.
struct MlpPacked {
    unsigned short W1[kHid * 16];
    unsigned short W2[kHid * kHid];
    unsigned short W2T[kHid * kHid];  // W2T[k][slot_of_col(j)] = W2[j][k]
    float b1[kHid], b2[kHid], W3[kHid], b3;
};

// A training launch (see mlp_train_kernel).
struct TrainRun {
    MlpPacked *net;
    const float *X, *y;
    int64_t count;     // rows available
    int32_t batch;     // rows per optimizer step
    int32_t steps;     // optimizer steps of this launch
    int64_t step0;     // index of the launch's first step within the run
    int64_t total;     // steps of the run (learning-rate schedule)
    int64_t adam0;     // Adam steps taken before this launch
    double lr, lr_final;
    int32_t apply;     // 0: one gradient evaluation, no update
    float *part;       // [gridDim.x][kPartStride]
    float *grad;       // [kParams + 1]: summed gradient, then the sum of squared residuals
    float *master, *m, *v;
    float *loss_first; // the run's first sum of squared residuals
    unsigned long long *sync;  // barrier counter and per-block flags
    unsigned long long sync_base;
    unsigned int *fail;  // set when a barrier wait gives up
};

struct SampleParams {
    const double4 *ring_w;
    const double4 *ring_v;
    const double *T;
    int64_t N;
    int32_t D;
    int32_t head;
    double t;
    double inv_sigma;  // 1 / sigma_ref
    uint64_t seed;
};

struct GuessParams {
    const double4 *ring_w;
    const double4 *ring_v;
    const double *T;
    const double3 *centroid;  // [ngroups]
    int64_t N;
    int64_t ngroups;
    int32_t D;
    int32_t head;
    double inv_sigma;
    // 0: G = the network's c (t - t_r) / |r - w_n|; 1: G = that prediction
    // divided by the straight-line value at the same point (the group's
    // correction factor, applied per target to its own straight-line delay)
    int32_t ratio;
};

}  // namespace empp
