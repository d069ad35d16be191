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

// Network as the kernels read it: bf16 matrices (W1 padded to 16 inputs),
// bf16-rounded vectors stored as floats.
struct MlpPacked {
    unsigned short W1[kHid * 16];
    unsigned short W2[kHid * kHid];
    float b1[kHid], b2[kHid], W3[kHid], b3;
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
