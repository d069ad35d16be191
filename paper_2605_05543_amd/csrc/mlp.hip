// mlp.hip -- the retarded-delay surrogate network 10 -> 128 -> 128 -> 1
// (SiLU hidden layers) with BF16 weights and activations on the matrix
// cores, FP32 accumulation: the 10-input layer on v_mfma_f32_16x16x16_bf16,
// every 128-deep product (layer 2, its backward, the weight gradients) on
// gfx950's v_mfma_f32_16x16x32_bf16.  Inference, training (forward,
// backward, the fixed-order gradient sum and Adam in one launch per
// optimizer step) and the sampling of training pairs from the histories.
//
// The model predicts the normalised retarded delay g = c (t - t_r) /
// |r - w_n| of a (target, source) pair as g_line exp(z): g_line is the
// value for a source coasting with its newest velocity (a closed form of
// the features) and the network output z corrects it, so an untrained
// network (z = 0) reproduces the straight-line guess.  A guided search
// starts from the prediction; it never decides a result: the exact search
// finishes every bracket.
//
// Layout of the flat parameter vector (FP32 masters, 18049 values):
//   W1[128][10], b1[128], W2[128][128], b2[128], W3[1][128], b3[1].
// Matrix-core layouts used throughout (checked on gfx950): for D = A B,
// lane l, lane group g = l / 16,
//   16x16x16: A[l % 16][4 g + r], B[4 g + r][l % 16], r = 0..3;
//   16x16x32: A[l % 16][s(g, r)], B[s(g, r)][l % 16], r = 0..7, where the
//             pairing of A and B slots is the only thing the sum needs;
//   both:     D[4 g + r][l % 16], r = 0..3.
// Layers are evaluated transposed, H^T = W X^T, so the D layout of one
// layer is the B layout of the next: activations stay in registers.  Two
// D tiles (rows 0..15 and 16..31 of a 32-deep block) give lane group g the
// rows 4 g + r and 16 + 4 g + r: that is the slot order s(g, r) of every
// 16x16x32 product here, and weight rows are stored with their columns in
// that order, so one 16-byte LDS read gives a lane its 8 A values.
#include "empp_dev.h"
#include "mlp_dev.h"
#include "pair_common.h"

namespace empp {

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma16(s4 a, s4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }
__device__ __forceinline__ f4 mfma32(s8 a, s8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, a), __builtin_bit_cast(bf8, b), c, 0, 0, 0);
}
// the 8 K values of a lane: 4 from each of two 16-deep halves
__device__ __forceinline__ s8 cat(s4 lo, s4 hi) { return __builtin_shufflevector(lo, hi, 0, 1, 2, 3, 4, 5, 6, 7); }

// Round to the nearest bfloat16, ties to even (finite inputs).
__device__ __forceinline__ unsigned short bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_value(unsigned short h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float silu(float x) { return x / (1.0f + __expf(-x)); }
// Inference form: hardware exp2 and reciprocal (a few ulp of float, far
// below the bf16 rounding the activations then take).
__device__ __forceinline__ float silu_fast(float x)
{
    return x * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-1.4426950408889634f * x));
}
__device__ __forceinline__ float silu_grad(float x)
{
    float s = 1.0f / (1.0f + __expf(-x));
    return s * (1.0f + x * (1.0f - s));
}

// Network weights staged in LDS: W1 [128][16] (K padded, column 10 is 0),
// W2 [128][128] (columns in slot order), the bf16-rounded biases and W3 as
// floats.  Rows are padded so that the 16 rows one A-fragment read touches
// start on distinct banks: 20 halfwords for the 8-byte reads of W1, 136
// (68 dwords, 4 mod 32) for the 16-byte reads of W2, which put 8 lanes on
// 8 disjoint groups of 4 banks.
constexpr int kW1S = 20, kW2S = 136;
struct NetLds {
    unsigned short W1[kHid * kW1S];
    alignas(16) unsigned short W2[kHid * kW2S];
    float b1[kHid], b2[kHid], W3[kHid], b3;
};

// Every network kernel runs 256-thread blocks.
constexpr int kMlpThreads = 256;

// A [128][128] bf16 matrix from global memory into LDS rows of kW2S
// halfwords, eight halfwords per copy.
__device__ __forceinline__ void load_matrix(unsigned short *dst, const unsigned short *src)
{
    const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
    uint4 *d4 = reinterpret_cast<uint4 *>(dst);
#pragma unroll
    for (int k = 0; k < kHid * kHid / 8 / kMlpThreads; ++k) {
        const int i = threadIdx.x + k * kMlpThreads;
        d4[(i / (kHid / 8)) * (kW2S / 8) + i % (kHid / 8)] = s4[i];
    }
}

__device__ void load_net(NetLds &s, const MlpPacked *net)
{
    // two halfwords per copy for W1; rows keep their padded stride
    const uint32_t *src1 = reinterpret_cast<const uint32_t *>(net->W1);
    uint32_t *dst1 = reinterpret_cast<uint32_t *>(s.W1);
#pragma unroll
    for (int k = 0; k < kHid * 16 / 2 / kMlpThreads; ++k) {
        const int i = threadIdx.x + k * kMlpThreads;
        dst1[(i / 8) * (kW1S / 2) + i % 8] = src1[i];
    }
    load_matrix(s.W2, net->W2);
    if (threadIdx.x < kHid) {
        const int i = threadIdx.x;
        s.b1[i] = net->b1[i];
        s.b2[i] = net->b2[i];
        s.W3[i] = net->W3[i];
    }
    if (threadIdx.x == 0)
        s.b3 = net->b3;
}

__device__ __forceinline__ s8 lds_s8(const unsigned short *p)
{
    return __builtin_bit_cast(s8, *reinterpret_cast<const uint4 *>(p));
}

__device__ __forceinline__ s4 lds_s4(const unsigned short *p)
{
    uint2 v = *reinterpret_cast<const uint2 *>(p);
    s4 r;
    r[0] = (short)(v.x & 0xffff);
    r[1] = (short)(v.x >> 16);
    r[2] = (short)(v.y & 0xffff);
    r[3] = (short)(v.y >> 16);
    return r;
}

// Four floats to bf16 (round to nearest even) with the gfx950 packed
// conversion instruction (v_cvt_pk_bf16_f32), two values per instruction.
__device__ __forceinline__ s4 pack4(float a, float b, float c, float d)
{
    typedef float f2v __attribute__((ext_vector_type(2)));
    typedef __bf16 b2v __attribute__((ext_vector_type(2)));
    const b2v lo = __builtin_convertvector((f2v){a, b}, b2v);
    const b2v hi = __builtin_convertvector((f2v){c, d}, b2v);
    const uint32_t ul = __builtin_bit_cast(uint32_t, lo), uh = __builtin_bit_cast(uint32_t, hi);
    s4 r;
    r[0] = (short)(ul & 0xffffu);
    r[1] = (short)(ul >> 16);
    r[2] = (short)(uh & 0xffffu);
    r[3] = (short)(uh >> 16);
    return r;
}

// Forward pass of 16 rows held by one wavefront.  x4: the 4 features
// 4 (l/16) .. 4 (l/16) + 3 of row l % 16 (zero beyond 10).  Returns z of
// row l % 16 (valid in every lane).  For training (KEEP) it keeps the
// pre-activations in registers and writes the bf16 activations H1^T and
// H2^T ([unit][row], 16 rows) to the wavefront's LDS tiles.
struct FwdState {
    f4 a1[8], a2[8];            // pre-activations (D layout)
    unsigned short *h1t, *h2t;  // LDS tiles of H1^T, H2^T
};

template <bool KEEP>
__device__ __forceinline__ float net_forward(const NetLds &s, s4 xb, FwdState &st)
{
    const int l = threadIdx.x & 63;
    const int g = l >> 4, col = l & 15;
    // layer 1: H1^T = W1 X^T, 8 tiles of 16 hidden units
    s4 h1[8];
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
        s4 a = lds_s4(&s.W1[(mt * 16 + col) * kW1S + 4 * g]);
        f4 d = mfma16(a, xb, f4{0, 0, 0, 0});
        float v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float pre = d[r] + s.b1[mt * 16 + 4 * g + r];
            if (KEEP)
                st.a1[mt][r] = pre;
            v[r] = KEEP ? silu(pre) : silu_fast(pre);
        }
        h1[mt] = pack4(v[0], v[1], v[2], v[3]);
        if (KEEP) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                st.h1t[(mt * 16 + 4 * g + r) * 16 + col] = (unsigned short)h1[mt][r];
        }
    }
    // layer 2: H2^T = W2 H1^T
    float z = 0.0f;
    auto tile2 = [&](int mt) {
        f4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            s8 a = lds_s8(&s.W2[(mt * 16 + col) * kW2S + kt * 32 + 8 * g]);
            acc = mfma32(a, cat(h1[2 * kt], h1[2 * kt + 1]), acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int j = mt * 16 + 4 * g + r;
            float pre = acc[r] + s.b2[j];
            float h = KEEP ? silu(pre) : silu_fast(pre);
            if (KEEP) {
                st.a2[mt][r] = pre;
                st.h2t[j * 16 + col] = bf16_bits(h);
            }
            z += s.W3[j] * h;
        }
    };
    if (KEEP) {
        // training keeps every tile's values: static register indices
#pragma unroll
        for (int mt = 0; mt < 8; ++mt)
            tile2(mt);
    } else {
        // inference: four output tiles at a time bounds the A fragments of
        // W2 held in registers
#pragma unroll 4
        for (int mt = 0; mt < 8; ++mt)
            tile2(mt);
    }
    // layer 3: sum the four lane groups that share a row
    z += __shfl_xor(z, 16);
    z += __shfl_xor(z, 32);
    return z + s.b3;
}

__device__ __forceinline__ s4 feature_operand(const float *row_features /* 10 values */)
{
    const int g = (threadIdx.x & 63) >> 4;
    float v[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        int k = 4 * g + r;
        v[r] = k < kIn ? row_features[k] : 0.0f;
    }
    return pack4(v[0], v[1], v[2], v[3]);
}

// Inference forward of T row tiles (16 rows each) held by one wavefront:
// every A fragment of W1 and W2 read from LDS feeds T matrix-core products,
// so the LDS traffic per row falls by T.  Returns z of row l % 16 of tile t
// in z[t] (valid in every lane).
template <int T>
__device__ __forceinline__ void net_forward_tiles(const NetLds &s, const s4 xb[T], float z[T])
{
    const int l = threadIdx.x & 63;
    const int g = l >> 4, col = l & 15;
    s4 h1[T][8];
#pragma unroll
    for (int mt = 0; mt < 8; ++mt) {
        s4 a = lds_s4(&s.W1[(mt * 16 + col) * kW1S + 4 * g]);
#pragma unroll
        for (int t = 0; t < T; ++t) {
            f4 d = mfma16(a, xb[t], f4{0, 0, 0, 0});
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                v[r] = silu_fast(d[r] + s.b1[mt * 16 + 4 * g + r]);
            h1[t][mt] = pack4(v[0], v[1], v[2], v[3]);
        }
    }
#pragma unroll
    for (int t = 0; t < T; ++t)
        z[t] = 0.0f;
#pragma unroll 2
    for (int mt = 0; mt < 8; ++mt) {
        f4 acc[T];
#pragma unroll
        for (int t = 0; t < T; ++t)
            acc[t] = f4{0, 0, 0, 0};
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            s8 a = lds_s8(&s.W2[(mt * 16 + col) * kW2S + kt * 32 + 8 * g]);
#pragma unroll
            for (int t = 0; t < T; ++t)
                acc[t] = mfma32(a, cat(h1[t][2 * kt], h1[t][2 * kt + 1]), acc[t]);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = mt * 16 + 4 * g + r;
            const float b2 = s.b2[j], w3 = s.W3[j];
#pragma unroll
            for (int t = 0; t < T; ++t)
                z[t] += w3 * silu_fast(acc[t][r] + b2);
        }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
        z[t] += __shfl_xor(z[t], 16);
        z[t] += __shfl_xor(z[t], 32);
        z[t] += s.b3;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Inference on explicit feature rows: X [n][10] -> z [n].
__global__ __launch_bounds__(256) void mlp_forward_kernel(const MlpPacked *net, const float *X, int64_t n, float *z)
{
    __shared__ NetLds s;
    load_net(s, net);
    __syncthreads();
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int64_t base = ((int64_t)blockIdx.x * 4 + w) * 16; base < n; base += (int64_t)gridDim.x * 64) {
        int64_t row = base + (l & 15);
        float f[kIn];
#pragma unroll
        for (int k = 0; k < kIn; ++k)
            f[k] = row < n ? X[row * kIn + k] : 0.0f;
        FwdState st;
        float zz = net_forward<false>(s, feature_operand(f), st);
        if (l < 16 && row < n)
            z[row] = zz;
    }
}

// ---------------------------------------------------------------------------
// Training, many optimizer steps per launch.  Phase 1: forward + backward
// of every row, gradients of the mean squared error of z against y
// accumulated per block (matrix cores for every product, biases through
// an appended column of ones), written as one partial gradient per block:
// part[block][kPartStride], the flat gradient and the block's sum of
// squared residuals.  Phase 2, after a grid-wide barrier (the launch is
// cooperative, so every block is resident): each parameter's partials are
// summed in a fixed order (FP64, so the result does not depend on
// scheduling), then Adam (bias-corrected) updates the FP32 master and the
// packed bf16 copy the next step's forward pass reads.
struct TrainLds {
    NetLds net;
    alignas(16) unsigned short W2T[kHid * kW2S];  // W2 transposed (columns in slot order)
    unsigned short H1T[4][kHid * 16];              // per wave: H1^T [j][i]
    unsigned short dA2T[4][kHid * 16];             // dA2^T [j][i]
    unsigned short dA1T[4][kHid * 16];             // dA1^T [j][i]
    unsigned short H2T[4][kHid * 16];              // H2^T [j][i]
    unsigned short XeT[4][16 * 16];                // [X | 1]^T [k][i] (column 10 of X is 1)
    unsigned short dzT[4][16 * 16];                // [dz | 0]^T [k][i] (k = 0: dz_i)
};
static_assert(sizeof(TrainLds) <= 160 * 1024, "training tile exceeds the 160 KiB of LDS");

// A store that other blocks read after the next grid barrier, written
// through to device scope, so that the barrier's release has little left
// in the XCD's L2 to write back.
template <typename T>
__device__ __forceinline__ void store_shared(T &dst, T val)
{
    __hip_atomic_store(&dst, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Phase 1 for this block's rows X[n][10], y[n] (64 per chunk, chunks
// strided by the grid): the block's partial gradient into out.
__device__ void block_gradient(TrainLds &s, const MlpPacked *net, const float *X, const float *y, int64_t n,
                               float scale, float *out)
{
    load_net(s.net, net);
    load_matrix(s.W2T, net->W2T);
    __syncthreads();
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = l >> 4, col = l & 15;
    // gradient accumulators (D layout), this wave owns row tiles 2w, 2w+1
    f4 gW2[2][9], gW1[2], gW3[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) {
#pragma unroll
        for (int b = 0; b < 9; ++b)
            gW2[a][b] = f4{0, 0, 0, 0};
        gW1[a] = f4{0, 0, 0, 0};
        gW3[a] = f4{0, 0, 0, 0};
    }
    float gb3 = 0.0f, sqsum = 0.0f;

    for (int64_t chunk = (int64_t)blockIdx.x * 64; chunk < n; chunk += (int64_t)gridDim.x * 64) {
        const int64_t row = chunk + w * 16 + col;
        const bool live = row < n;
        float f[kIn];
#pragma unroll
        for (int k = 0; k < kIn; ++k)
            f[k] = live ? X[row * kIn + k] : 0.0f;
        FwdState st;
        st.h1t = s.H1T[w];
        st.h2t = s.H2T[w];
        float z = net_forward<true>(s.net, feature_operand(f), st);
        float res = live ? z - y[row] : 0.0f;
        float dz = live ? scale * res : 0.0f;
        if (l < 16)
            sqsum += res * res;
        gb3 += (l < 16) ? dz : 0.0f;
        // dA2^T = W3 dz silu'(A2^T), also written (bf16) for the products
        s4 da2[8];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int j = mt * 16 + 4 * g + r;
                v[r] = s.net.W3[j] * dz * silu_grad(st.a2[mt][r]);
            }
            da2[mt] = pack4(v[0], v[1], v[2], v[3]);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                s.dA2T[w][(mt * 16 + 4 * g + r) * 16 + col] = (unsigned short)da2[mt][r];
        }
        // dH1^T = W2^T dA2^T (K = the 128 units of layer 2, slot order);
        // dA1^T = dH1^T silu'(A1^T)
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            f4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int kt = 0; kt < 4; ++kt) {
                s8 a = lds_s8(&s.W2T[(mt * 16 + col) * kW2S + kt * 32 + 8 * g]);
                acc = mfma32(a, cat(da2[2 * kt], da2[2 * kt + 1]), acc);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int j = mt * 16 + 4 * g + r;
                s.dA1T[w][j * 16 + col] = bf16_bits(acc[r] * silu_grad(st.a1[mt][r]));
            }
        }
        // [X | 1]^T and [dz | 0]^T of this wave's 16 rows
        for (int k = 4 * g; k < 4 * g + 4; ++k) {
            float xv = k < kIn ? f[k] : (k == kIn && live ? 1.0f : 0.0f);
            s.XeT[w][k * 16 + col] = bf16_bits(xv);
            s.dzT[w][k * 16 + col] = bf16_bits(k == 0 ? dz : 0.0f);
        }
        __syncthreads();
        // weight gradients over the block's 64 rows (K = rows, two waves'
        // 16-row tiles per 32-deep step: slot r < 4 is row 4 g + r of the
        // first, r >= 4 row 4 g + r - 4 of the second, in A and B alike)
#pragma unroll
        for (int pr = 0; pr < 2; ++pr) {
            const int w0 = 2 * pr, w1 = 2 * pr + 1;
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int mt = 2 * w + a;
                // A: dA2^T rows j, K = rows i;  B: [H1 | 1] rows i, N = units k
                const int ra = (mt * 16 + col) * 16 + 4 * g;
                s8 A2 = cat(lds_s4(&s.dA2T[w0][ra]), lds_s4(&s.dA2T[w1][ra]));
#pragma unroll
                for (int nt = 0; nt < 8; ++nt) {
                    const int rb = (nt * 16 + col) * 16 + 4 * g;
                    gW2[a][nt] = mfma32(A2, cat(lds_s4(&s.H1T[w0][rb]), lds_s4(&s.H1T[w1][rb])), gW2[a][nt]);
                }
                // ones column (bias gradient): B[i][k] = 1 for k = 0
                const s4 one4 = (col == 0) ? pack4(1.0f, 1.0f, 1.0f, 1.0f) : s4{0, 0, 0, 0};
                gW2[a][8] = mfma32(A2, cat(one4, one4), gW2[a][8]);
                s8 A1 = cat(lds_s4(&s.dA1T[w0][ra]), lds_s4(&s.dA1T[w1][ra]));
                const int rx = col * 16 + 4 * g;
                gW1[a] = mfma32(A1, cat(lds_s4(&s.XeT[w0][rx]), lds_s4(&s.XeT[w1][rx])), gW1[a]);
                s8 H2 = cat(lds_s4(&s.H2T[w0][ra]), lds_s4(&s.H2T[w1][ra]));
                gW3[a] = mfma32(H2, cat(lds_s4(&s.dzT[w0][rx]), lds_s4(&s.dzT[w1][rx])), gW3[a]);
            }
        }
        __syncthreads();
    }
    // this block's partial gradient in the flat layout
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int mt = 2 * w + a;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = mt * 16 + 4 * g + r;
#pragma unroll
            for (int nt = 0; nt < 8; ++nt)
                store_shared(out[kOffW2 + j * kHid + nt * 16 + col], gW2[a][nt][r]);
            if (col == 0)
                store_shared(out[kOffB2 + j], gW2[a][8][r]);
            if (col < kIn)
                store_shared(out[kOffW1 + j * kIn + col], gW1[a][r]);
            if (col == kIn)
                store_shared(out[kOffB1 + j], gW1[a][r]);
            if (col == 0)
                store_shared(out[kOffW3 + j], gW3[a][r]);
        }
    }
    // b3 and the squared residuals: wave sums, then the block's
    for (int off = 32; off > 0; off >>= 1) {
        gb3 += __shfl_xor(gb3, off);
        sqsum += __shfl_xor(sqsum, off);
    }
    __shared__ float red_b3[4], red_sq[4];
    if (l == 0) {
        red_b3[w] = gb3;
        red_sq[w] = sqsum;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        store_shared(out[kOffB3], red_b3[0] + red_b3[1] + red_b3[2] + red_b3[3]);
        store_shared(out[kParams], red_sq[0] + red_sq[1] + red_sq[2] + red_sq[3]);
    }
}

// Grid-wide barrier of a cooperative launch.  sync[0] counts arrivals;
// the block that brings it to the target writes the target into every
// block's flag (sync[kSyncLine (b + 1)], one 128-byte line per block), and
// each other block waits on its own flag, so no line is polled by more than
// one block.  Thread 0 of a block carries the block's synchronisation: its
// arrival releases what the block wrote (the block's threads have finished
// their stores at the preceding __syncthreads) and acquires what the blocks
// before it released; the flags are polled with relaxed loads and one
// acquire fence follows the wait, so the XCD's L2 is invalidated once per
// barrier, not once per poll.  The wait is bounded (about a second); a block
// that gives up sets *fail, which the host reports, and goes on, so every
// wave still ends.
constexpr unsigned kSyncSpinLimit = 1u << 20;
__device__ void grid_barrier(unsigned long long *sync, unsigned long long target, unsigned int *fail)
{
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long seen =
            __hip_atomic_fetch_add(sync, 1ull, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1;
        if (seen == target) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            for (int b = 0; b < (int)gridDim.x; ++b)
                __hip_atomic_store(&sync[kSyncLine * (b + 1)], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            unsigned long long *flag = &sync[kSyncLine * (blockIdx.x + 1)];
            unsigned spins = 0;
            while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (++spins > kSyncSpinLimit) {
                    atomicOr(fail, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
    }
    __syncthreads();
}

// One parameter of the packed network from its FP32 master value.
__device__ __forceinline__ void pack_param(MlpPacked *net, int q, float x)
{
    if (q < kOffB1) {
        store_shared(net->W1[(q / kIn) * 16 + q % kIn], bf16_bits(x));
    } else if (q < kOffW2) {
        store_shared(net->b1[q - kOffB1], bf16_value(bf16_bits(x)));
    } else if (q < kOffB2) {
        const int j = (q - kOffW2) / kHid, k = (q - kOffW2) % kHid;
        const unsigned short h = bf16_bits(x);
        store_shared(net->W2[j * kHid + slot_of_col(k)], h);
        store_shared(net->W2T[k * kHid + slot_of_col(j)], h);
    } else if (q < kOffW3) {
        store_shared(net->b2[q - kOffB2], bf16_value(bf16_bits(x)));
    } else if (q < kOffB3) {
        store_shared(net->W3[q - kOffW3], bf16_value(bf16_bits(x)));
    } else {
        store_shared(net->b3, bf16_value(bf16_bits(x)));
    }
}

// Phase 2 for this block's slice [q0, q1) of the parameters (q0 a
// multiple of 4): column c of the slice's 16-byte units is summed over the
// block partials b = r, r + R, ... by thread (c, r), in FP64, and the R
// sums of a column are then added in order r = 0, 1, ...: a fixed order,
// whatever the scheduling.  Then the gradient, Adam (bias-corrected) on
// the FP32 masters and the packed network for those parameters.
__device__ void reduce_and_update(const TrainRun &p, double4 *red, int q0, int q1, int64_t gs, int it)
{
    const int nb = (int)gridDim.x;
    const double frac = p.total > 1 ? (double)gs / (double)(p.total - 1) : 1.0;
    const float lr = (float)(p.lr_final + 0.5 * (p.lr - p.lr_final) * (1.0 + cos(M_PI * frac)));
    const float step = (float)(p.adam0 + it + 1);
    const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(beta1, step), c2 = 1.0f - powf(beta2, step);
    const int ncol = (q1 - q0 + 3) / 4;
    const int cols = ncol < 64 ? ncol : 64;  // columns per pass
    const int R = kMlpThreads / cols;         // partial subsets per column
    const int c = threadIdx.x % cols, r = threadIdx.x / cols;
    for (int c0 = 0; c0 < ncol; c0 += cols) {
        const int col = c0 + c;
        double4 acc = make_double4(0.0, 0.0, 0.0, 0.0);
        if (r < R && col < ncol) {
            const float4 *src = reinterpret_cast<const float4 *>(p.part + q0) + col;
#pragma unroll 8
            for (int b = r; b < nb; b += R) {
                const float4 x = src[(int64_t)b * (kPartStride / 4)];
                acc.x += x.x;
                acc.y += x.y;
                acc.z += x.z;
                acc.w += x.w;
            }
        }
        if (r < R)
            red[r * cols + c] = acc;
        __syncthreads();
        if (r == 0 && col < ncol) {
            double4 t = red[c];
            for (int k = 1; k < R; ++k) {
                const double4 u = red[k * cols + c];
                t.x += u.x;
                t.y += u.y;
                t.z += u.z;
                t.w += u.w;
            }
            const double tv[4] = {t.x, t.y, t.z, t.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int q = q0 + 4 * col + e;
                if (q >= q1)
                    break;
                const float gr = (float)tv[e];
                p.grad[q] = gr;
                if (q == kParams && gs == 0)
                    *p.loss_first = gr;
                if (p.apply && q < kParams) {
                    const float mm = beta1 * p.m[q] + (1.0f - beta1) * gr;
                    const float vv = beta2 * p.v[q] + (1.0f - beta2) * gr * gr;
                    p.m[q] = mm;
                    p.v[q] = vv;
                    const float x = p.master[q] - lr * (mm / c1) / (sqrtf(vv / c2) + eps);
                    p.master[q] = x;
                    pack_param(p.net, q, x);
                }
            }
        }
        __syncthreads();
    }
}

// Training: p.steps optimizer steps in one launch.  Per step: phase 1 on
// the step's batch (consecutive rows, wrapping to the start when a batch
// would run past the end), a grid barrier, phase 2 on this block's slice
// of the parameters, and a second barrier before the next step reads the
// packed network.
__global__ __launch_bounds__(kMlpThreads) void mlp_train_kernel(const TrainRun *run)
{
    // The run's parameters are read from device memory where they are used
    // (the empty asm statements below mark memory as changed, so they are
    // not held in registers across the step loop, which would spill).
    const TrainRun &p = *run;
    extern __shared__ unsigned char tls_raw[];
    TrainLds &s = *reinterpret_cast<TrainLds *>(tls_raw);
    // phase 2's column sums reuse the H1^T tiles (16 KiB, 512 double4)
    static_assert(sizeof(s.H1T) >= kMlpThreads * sizeof(double4), "phase-2 sums fit the H1^T tiles");
    double4 *red = reinterpret_cast<double4 *>(&s.H1T[0][0]);
    const int nb = (int)gridDim.x;
    const int slice = ((kParams + 1 + nb - 1) / nb + 3) & ~3;
    const int q0 = min((int)blockIdx.x * slice, kParams + 1);
    const int q1 = min(q0 + slice, kParams + 1);
    unsigned long long target = p.sync_base;
    for (int it = 0; it < p.steps; ++it) {
        asm volatile("" ::: "memory");
        const int64_t gs = p.step0 + it;
        int64_t start = (gs * p.batch) % p.count;
        if (start + p.batch > p.count)
            start = 0;
        block_gradient(s, p.net, p.X + start * kIn, p.y + start, p.batch, 2.0f / (float)p.batch,
                       p.part + (int64_t)blockIdx.x * kPartStride);
        target += nb;
        grid_barrier(p.sync, target, p.fail);
        asm volatile("" ::: "memory");
        if (q0 < q1)
            reduce_and_update(p, red, q0, q1, gs, it);
        if (it + 1 < p.steps) {
            target += nb;
            grid_barrier(p.sync, target, p.fail);
        }
    }
}

// Clears the barrier counter, the flags of up to kSyncMaxBlocks blocks and
// the failure word (one block of kMlpThreads threads).
__global__ void mlp_sync_clear_kernel(unsigned long long *sync, unsigned int *fail)
{
    for (int i = threadIdx.x; i < kSyncLine * (kSyncMaxBlocks + 1); i += blockDim.x)
        sync[i] = 0;
    if (threadIdx.x == 0)
        *fail = 0;
}

// FP32 masters -> packed network (bf16 matrices, bf16-rounded vectors;
// the padding columns of W1 are zero).
__global__ void mlp_pack_kernel(const float *master, MlpPacked *net)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kHid * 16 && p % 16 >= kIn)
        net->W1[p] = 0;
    if (p < kParams)
        pack_param(net, p, master[p]);
}

// ---------------------------------------------------------------------------
// Pair features and exact targets from the stored histories.
//   features: (r - w_n)/sigma_ref, v_n/c, (w_n - w_{n-4})/(c (T_n - T_{n-4})),
//             log1p((t - T_n)/dt);  target: log(c (t - t_r) / s_line), s_line
//             the look-back of a source coasting with its newest velocity.
// Pairs are given (target particle, source) or drawn with a counter-based
// generator (splitmix64 of seed + pair counter).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

__device__ void pair_features(const SampleParams &p, int64_t i, int64_t j, float *Xrow, float *yrow)
{
    const int D = p.D;
    const int h = p.head;
    double4 r = p.ring_w[i * D + h];
    double4 wn = p.ring_w[j * D + h];
    double4 vn = p.ring_v[j * D + h];
    int h4 = h - 4;
    h4 += h4 < 0 ? D : 0;
    double4 w4 = p.ring_w[j * D + h4];
    const double c = kC_LIGHT;
    double Rx = r.x - wn.x, Ry = r.y - wn.y, Rz = r.z - wn.z;
    double span = c * (p.T[h] - p.T[h4]);
    Xrow[0] = (float)(Rx * p.inv_sigma);
    Xrow[1] = (float)(Ry * p.inv_sigma);
    Xrow[2] = (float)(Rz * p.inv_sigma);
    Xrow[3] = (float)(vn.x / c);
    Xrow[4] = (float)(vn.y / c);
    Xrow[5] = (float)(vn.z / c);
    Xrow[6] = (float)((wn.x - w4.x) / span);
    Xrow[7] = (float)((wn.y - w4.y) / span);
    Xrow[8] = (float)((wn.z - w4.z) / span);
    Xrow[9] = 0.0f;  // log1p((t - T_n)/dt) with t = T_n
    // exact bracket (FP64 sign tests on the history in HBM) and root
    const double R0sq = offset_sq(Rx, Ry, Rz);
    auto test = [&](int b) {
        int ph = h - b;
        ph += ph < 0 ? D : 0;
        const double L = c * (p.t - p.T[ph]);
        return lightcone_positive(lightcone_record(wn, p.ring_w[j * D + ph], L), Rx, Ry, Rz, R0sq);
    };
    int probes = 0;
    int b = search_bisect(test, D, probes);
    const bool before = b < 0;
    const int bb = before ? D - 1 : b;
    int ph1 = h - bb;
    ph1 += ph1 < 0 ? D : 0;
    double4 w1 = p.ring_w[j * D + ph1];
    double4 v1 = p.ring_v[j * D + ph1];
    double L1 = c * (p.t - p.T[ph1]);
    double dx = r.x - w1.x, dy = r.y - w1.y, dz = r.z - w1.z;
    double C2 = c * c - (v1.x * v1.x + v1.y * v1.y + v1.z * v1.z);
    double C1h = (dx * v1.x + dy * v1.y + dz * v1.z) - c * L1;
    double C0 = L1 * L1 - (dx * dx + dy * dy + dz * dz);
    double sq = sqrt(fmax(C1h * C1h - C2 * C0, 0.0));
    double dtr = C1h <= 0.0 ? C0 / (sq - C1h) : -(C1h + sq) / C2;
    double look = L1 - c * dtr;  // c (t - t_r)
    // the model's fixed term: the look-back of a source coasting with its
    // newest velocity, s solving (1 - beta^2) s^2 - 2 (R.beta) s - R^2 = 0
    double bx = vn.x / c, by = vn.y / c, bz = vn.z / c;
    double rb = Rx * bx + Ry * by + Rz * bz, R2 = Rx * Rx + Ry * Ry + Rz * Rz;
    double g2 = 1.0 - (bx * bx + by * by + bz * bz);
    double s_line = (rb + sqrt(rb * rb + g2 * R2)) / g2;
    yrow[0] = (float)log(look / s_line);
}

__global__ void mlp_sample_kernel(SampleParams p, const int64_t *tgt, const int64_t *src, int64_t count, float *X,
                                  float *y)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= count)
        return;
    int64_t i, j;
    if (tgt) {
        i = tgt[q];
        j = src[q];
    } else {
        uint64_t h1 = splitmix64(p.seed + 2 * (uint64_t)q);
        uint64_t h2 = splitmix64(p.seed + 2 * (uint64_t)q + 1);
        i = (int64_t)(h1 % (uint64_t)p.N);
        j = (int64_t)(h2 % (uint64_t)(p.N - 1));
        j += j >= i ? 1 : 0;  // never the self pair
    }
    pair_features(p, i, j, X + q * kIn, y + q);
}

// ---------------------------------------------------------------------------
// Surrogate guesses for a step: one network evaluation per (group of 64
// consecutive targets in the spatial order, source) with the group's
// centroid as target, written as the predicted g; the pair kernel scales
// it by each target's own distance to the source's newest position.
#ifndef EMPP_GUESS_TILES
#define EMPP_GUESS_TILES 2
#endif
__global__ __launch_bounds__(256) void mlp_group_guess_kernel(const MlpPacked *net, GuessParams p, float *G)
{
    constexpr int kTiles = EMPP_GUESS_TILES;  // row tiles per wavefront and pass
    __shared__ NetLds s;
    load_net(s, net);
    __syncthreads();
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t rows = p.ngroups * p.N;
    const int D = p.D, h = p.head;
    int h4 = h - 4;
    h4 += h4 < 0 ? D : 0;
    const double inv_c = 1.0 / kC_LIGHT;
    const double inv_span = 1.0 / (kC_LIGHT * (p.T[h] - p.T[h4]));
    const float sig = (float)(1.0 / p.inv_sigma);
    for (int64_t base = ((int64_t)blockIdx.x * 4 + w) * 16 * kTiles; base < rows;
         base += (int64_t)gridDim.x * 64 * kTiles) {
        s4 xb[kTiles];
        float gb[kTiles];  // straight-line normalised delay s_line / |R| (per-pair mode)
#pragma unroll
        for (int t = 0; t < kTiles; ++t) {
            const int64_t row = base + t * 16 + (l & 15);
            float f[kIn];
#pragma unroll
            for (int k = 0; k < kIn; ++k)
                f[k] = 0.0f;
            if (row < rows) {
                // source-major rows: a tile of 16 rows shares one source
                int64_t j = row / p.ngroups, grp = row - j * p.ngroups;
                double3 cen = p.centroid[grp];
                double4 wn = p.ring_w[j * D + h];
                double4 vn = p.ring_v[j * D + h];
                double4 w4 = p.ring_w[j * D + h4];
                f[0] = (float)((cen.x - wn.x) * p.inv_sigma);
                f[1] = (float)((cen.y - wn.y) * p.inv_sigma);
                f[2] = (float)((cen.z - wn.z) * p.inv_sigma);
                f[3] = (float)(vn.x * inv_c);
                f[4] = (float)(vn.y * inv_c);
                f[5] = (float)(vn.z * inv_c);
                f[6] = (float)((wn.x - w4.x) * inv_span);
                f[7] = (float)((wn.y - w4.y) * inv_span);
                f[8] = (float)((wn.z - w4.z) * inv_span);
            }
            xb[t] = feature_operand(f);
            gb[t] = 1.0f;
            if (!p.ratio) {
                // straight-line look-back in units of |r - w_n|
                const float Rx = f[0] * sig, Ry = f[1] * sig, Rz = f[2] * sig;
                const float R2 = Rx * Rx + Ry * Ry + Rz * Rz;
                const float rb = Rx * f[3] + Ry * f[4] + Rz * f[5];
                const float g2 = 1.0f - (f[3] * f[3] + f[4] * f[4] + f[5] * f[5]);
                const float sb = (rb + sqrtf(rb * rb + g2 * R2)) / g2;
                const float b = sb * __builtin_amdgcn_rsqf(R2);
                gb[t] = R2 > 0.0f && b > 0.0f ? b : 0.0f;
            }
        }
        float zz[kTiles];
        net_forward_tiles<kTiles>(s, xb, zz);
#pragma unroll
        for (int t = 0; t < kTiles; ++t) {
            const int64_t row = base + t * 16 + (l & 15);
            if (l < 16 && row < rows) {
                // the network corrects the straight-line delay by exp(z):
                // ratio mode stores the correction, per-pair mode the
                // normalised delay
                float g = __expf(zz[t]);
                if (!p.ratio)
                    g *= gb[t];
                G[row] = g;
            }
        }
    }
}

// Group centroids of the spatially ordered targets (64 per group).
__global__ void group_centroid_kernel(const double4 *ring_w, const int32_t *order, int64_t N, int D, int head,
                                      double3 *centroid)
{
    int64_t grp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t ngroups = (N + 63) / 64;
    if (grp >= ngroups)
        return;
    double sx = 0, sy = 0, sz = 0;
    int cnt = 0;
    for (int k = 0; k < 64; ++k) {
        int64_t a = grp * 64 + k;
        if (a >= N)
            break;
        int64_t i = order ? order[a] : a;
        double4 w = ring_w[i * D + head];
        sx += w.x;
        sy += w.y;
        sz += w.z;
        ++cnt;
    }
    centroid[grp] = make_double3(sx / cnt, sy / cnt, sz / cnt);
}

// Group centroids of external targets x[3][m] (`group` consecutive per
// group; group 1 gives each target its own row).
__global__ void group_centroid_x_kernel(const double *x, int64_t m, int group, double3 *centroid)
{
    int64_t grp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t ngroups = (m + group - 1) / group;
    if (grp >= ngroups)
        return;
    double sx = 0, sy = 0, sz = 0;
    int cnt = 0;
    for (int k = 0; k < group; ++k) {
        int64_t a = grp * group + k;
        if (a >= m)
            break;
        sx += x[a];
        sy += x[m + a];
        sz += x[2 * m + a];
        ++cnt;
    }
    centroid[grp] = make_double3(sx / cnt, sy / cnt, sz / cnt);
}

// ---------------------------------------------------------------------------
hipError_t launch_mlp_forward(const MlpPacked *net, const float *X, int64_t n, float *z, hipStream_t s)
{
    int64_t blocks = (n + 63) / 64;
    if (blocks > 4096)
        blocks = 4096;
    if (blocks < 1)
        blocks = 1;
    hipLaunchKernelGGL(mlp_forward_kernel, dim3((unsigned)blocks), dim3(256), 0, s, net, X, n, z);
    return hipGetLastError();
}

size_t mlp_train_lds_bytes() { return sizeof(TrainLds); }

// Blocks of the training kernel that fit on the device at once (the
// cooperative launch needs every block resident).
hipError_t mlp_train_max_blocks(int device, int *out)
{
    const size_t lds = sizeof(TrainLds);
    hipError_t e =
        hipFuncSetAttribute((const void *)mlp_train_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    int per_cu = 0, cus = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mlp_train_kernel, kMlpThreads, lds)) !=
        hipSuccess)
        return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device)) != hipSuccess)
        return e;
    *out = per_cu * cus;
    return hipSuccess;
}

hipError_t launch_mlp_sync_clear(unsigned long long *sync, unsigned int *fail, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_sync_clear_kernel, dim3(1), dim3(kMlpThreads), 0, s, sync, fail);
    return hipGetLastError();
}

// run->steps optimizer steps (or, with apply = 0, one gradient evaluation)
// on nblocks resident blocks; run is in device memory; *run->sync must hold
// run->sync_base arrivals when the launch starts, and holds sync_base +
// nblocks (2 steps - 1) after it.
hipError_t launch_mlp_train(const TrainRun *run, int nblocks, hipStream_t s)
{
    const TrainRun *arg = run;
    void *args[] = {&arg};
    return hipLaunchCooperativeKernel((const void *)mlp_train_kernel, dim3((unsigned)nblocks), dim3(kMlpThreads),
                                      args, (unsigned)sizeof(TrainLds), s);
}

hipError_t launch_mlp_pack(const float *master, MlpPacked *net, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_pack_kernel, dim3((kParams + kMlpThreads - 1) / kMlpThreads), dim3(kMlpThreads), 0, s,
                       master, net);
    return hipGetLastError();
}

hipError_t launch_mlp_sample(const SampleParams &p, const int64_t *tgt, const int64_t *src, int64_t count, float *X,
                             float *y, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_sample_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, tgt, src, count,
                       X, y);
    return hipGetLastError();
}

hipError_t launch_mlp_group_guess(const MlpPacked *net, const GuessParams &p, float *G, hipStream_t s)
{
    int64_t rows = p.ngroups * p.N;
    int64_t blocks = (rows + 255) / 256;
    if (blocks > 8192)
        blocks = 8192;
    hipLaunchKernelGGL(mlp_group_guess_kernel, dim3((unsigned)blocks), dim3(256), 0, s, net, p, G);
    return hipGetLastError();
}

hipError_t launch_group_centroid(const double4 *ring_w, const int32_t *order, int64_t N, int D, int head,
                                 double3 *centroid, hipStream_t s)
{
    int64_t ng = (N + 63) / 64;
    hipLaunchKernelGGL(group_centroid_kernel, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, ring_w, order, N,
                       D, head, centroid);
    return hipGetLastError();
}

// Centroids of groups of `ratio` consecutive 64-target groups (the last
// ones may be short), weighted by their target counts.
__global__ void merge_centroids_kernel(const double3 *cent64, int64_t m, int ratio, double3 *out)
{
    const int64_t n64 = (m + 63) / 64;
    const int64_t grp = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (grp * ratio >= n64)
        return;
    double sx = 0, sy = 0, sz = 0, wsum = 0;
    for (int k = 0; k < ratio && grp * ratio + k < n64; ++k) {
        const int64_t g = grp * ratio + k;
        const double w = (double)(g + 1 < n64 ? 64 : m - 64 * g);
        const double3 c = cent64[g];
        sx += w * c.x;
        sy += w * c.y;
        sz += w * c.z;
        wsum += w;
    }
    out[grp] = make_double3(sx / wsum, sy / wsum, sz / wsum);
}

hipError_t launch_merge_centroids(const double3 *cent64, int64_t m, int ratio, double3 *out, hipStream_t s)
{
    const int64_t ng = ((m + 63) / 64 + ratio - 1) / ratio;
    hipLaunchKernelGGL(merge_centroids_kernel, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, cent64, m, ratio,
                       out);
    return hipGetLastError();
}

hipError_t launch_group_centroid_x(const double *x, int64_t m, int group, double3 *centroid, hipStream_t s)
{
    int64_t ng = (m + group - 1) / group;
    hipLaunchKernelGGL(group_centroid_x_kernel, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, s, x, m, group,
                       centroid);
    return hipGetLastError();
}

}  // namespace empp
