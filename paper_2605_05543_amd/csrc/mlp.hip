// mlp.hip -- the retarded-delay surrogate network 10 -> 128 -> 128 -> 1
// (SiLU hidden layers) with BF16 weights and activations on the matrix
// cores (v_mfma_f32_16x16x16_bf16, FP32 accumulation): inference, training
// (forward + backward + Adam) and the sampling of training pairs from the
// stored histories.
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
// Matrix-core layout used throughout (checked on gfx950): for
// D = A B with A 16x16 (M x K), B 16x16 (K x N), lane l holds
//   A[l % 16][4 (l / 16) + r], B[4 (l / 16) + r][l % 16],
//   D[4 (l / 16) + r][l % 16],  r = 0..3.
// Layers are evaluated transposed, H^T = W X^T, so the D layout of one
// layer is exactly the B layout the next layer needs: activations stay in
// registers between layers.
#include "empp_dev.h"
#include "mlp_dev.h"
#include "pair_common.h"

namespace empp {

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma16(s4 a, s4 b, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0); }

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
// W2 [128][128], the bf16-rounded biases and W3 as floats.  Rows are padded
// (to 20 and 132 halfwords) so that the 16 rows one A-fragment read touches
// start on distinct banks.
constexpr int kW1S = 20, kW2S = 132;
struct NetLds {
    unsigned short W1[kHid * kW1S];
    unsigned short W2[kHid * kW2S];
    float b1[kHid], b2[kHid], W3[kHid], b3;
};

__device__ void load_net(NetLds &s, const MlpPacked *net)
{
    // two halfwords per copy; rows keep their padded stride
    const uint32_t *src1 = reinterpret_cast<const uint32_t *>(net->W1);
    uint32_t *dst1 = reinterpret_cast<uint32_t *>(s.W1);
    for (int i = threadIdx.x; i < kHid * 16 / 2; i += blockDim.x)
        dst1[(i / 8) * (kW1S / 2) + i % 8] = src1[i];
    const uint32_t *src2 = reinterpret_cast<const uint32_t *>(net->W2);
    uint32_t *dst2 = reinterpret_cast<uint32_t *>(s.W2);
    for (int i = threadIdx.x; i < kHid * kHid / 2; i += blockDim.x)
        dst2[(i / (kHid / 2)) * (kW2S / 2) + i % (kHid / 2)] = src2[i];
    for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
        s.b1[i] = net->b1[i];
        s.b2[i] = net->b2[i];
        s.W3[i] = net->W3[i];
    }
    if (threadIdx.x == 0)
        s.b3 = net->b3;
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
// row l % 16 (valid in every lane).  Optionally keeps the pre-activations
// and bf16 activations for the backward pass.
struct FwdState {
    f4 a1[8], a2[8];  // pre-activations (D layout)
    s4 h1[8];         // bf16 H1^T tiles (B layout of layer 2)
    f4 h2[8];         // H2^T (float)
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
        if (KEEP)
            st.h1[mt] = h1[mt];
    }
    // layer 2: H2^T = W2 H1^T
    float z = 0.0f;
    auto tile2 = [&](int mt) {
        f4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int kt = 0; kt < 8; ++kt) {
            s4 a = lds_s4(&s.W2[(mt * 16 + col) * kW2S + kt * 16 + 4 * g]);
            acc = mfma16(a, h1[kt], acc);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            int j = mt * 16 + 4 * g + r;
            float pre = acc[r] + s.b2[j];
            float h = KEEP ? silu(pre) : silu_fast(pre);
            if (KEEP) {
                st.a2[mt][r] = pre;
                st.h2[mt][r] = h;
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
        for (int kt = 0; kt < 8; ++kt) {
            s4 a = lds_s4(&s.W2[(mt * 16 + col) * kW2S + kt * 16 + 4 * g]);
#pragma unroll
            for (int t = 0; t < T; ++t)
                acc[t] = mfma16(a, h1[t][kt], acc[t]);
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
// Training step part 1: forward + backward of every row, gradients of the
// mean squared error of z against y accumulated per block (matrix cores for
// every product, biases through an appended column of ones), written as
// one partial gradient per block.  part[block][kParams + 1]: the flat
// gradient and the block's sum of squared residuals.
struct TrainLds {
    NetLds net;
    unsigned short W2T[kHid * kHid];       // W2 transposed
    unsigned short H1T[4][kHid * 16];      // per wave: H1^T [j][i]
    unsigned short dA2T[4][kHid * 16];     // dA2^T [j][i]
    unsigned short dA1T[4][kHid * 16];     // dA1^T [j][i]
    unsigned short H2T[4][kHid * 16];      // H2^T [j][i]
    unsigned short XeT[4][16 * 16];        // [X | 1]^T [k][i] (column 10 of X is 1)
    unsigned short dzT[4][16 * 16];        // [dz | 0]^T [k][i] (k = 0: dz_i)
};
static_assert(sizeof(TrainLds) <= 160 * 1024, "training tile exceeds the 160 KiB of LDS");

__global__ __launch_bounds__(256) void mlp_train_kernel(const MlpPacked *net, const float *X, const float *y,
                                                        int64_t n, float scale, float *part)
{
    extern __shared__ unsigned char tls_raw[];
    TrainLds &s = *reinterpret_cast<TrainLds *>(tls_raw);
    load_net(s.net, net);
    __syncthreads();
    for (int i = threadIdx.x; i < kHid * kHid; i += blockDim.x) {
        int m = i / kHid, k = i % kHid;
        s.W2T[m * kHid + k] = s.net.W2[k * kW2S + m];
    }
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
        float z = net_forward<true>(s.net, feature_operand(f), st);
        float res = live ? z - y[row] : 0.0f;
        float dz = live ? scale * res : 0.0f;
        if (l < 16)
            sqsum += res * res;
        gb3 += (l < 16) ? dz : 0.0f;
        // dA2^T = W3 dz silu'(A2^T); also write H1^T, H2^T, dA2^T (bf16) for the products
        s4 da2[8];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            float v[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int j = mt * 16 + 4 * g + r;
                v[r] = s.net.W3[j] * dz * silu_grad(st.a2[mt][r]);
                s.H2T[w][j * 16 + col] = bf16_bits(st.h2[mt][r]);
                s.H1T[w][j * 16 + col] = (unsigned short)st.h1[mt][r];
            }
            da2[mt] = pack4(v[0], v[1], v[2], v[3]);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                s.dA2T[w][(mt * 16 + 4 * g + r) * 16 + col] = (unsigned short)da2[mt][r];
        }
        // dH1^T = W2^T dA2^T; dA1^T = dH1^T silu'(A1^T)
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            f4 acc = {0, 0, 0, 0};
#pragma unroll
            for (int kt = 0; kt < 8; ++kt) {
                s4 a = lds_s4(&s.W2T[(mt * 16 + col) * kHid + kt * 16 + 4 * g]);
                acc = mfma16(a, da2[kt], acc);
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
        // weight gradients over the block's 64 rows (K = rows)
#pragma unroll
        for (int ww = 0; ww < 4; ++ww) {
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int mt = 2 * w + a;
                // A: dA2^T rows j, K = rows i;  B: [H1 | 1] rows i, N = units k
                s4 A2 = lds_s4(&s.dA2T[ww][(mt * 16 + col) * 16 + 4 * g]);
#pragma unroll
                for (int nt = 0; nt < 8; ++nt) {
                    s4 Bh = lds_s4(&s.H1T[ww][(nt * 16 + col) * 16 + 4 * g]);
                    gW2[a][nt] = mfma16(A2, Bh, gW2[a][nt]);
                }
                // ones column (bias gradient): B[i][k] = 1 for k = 0
                s4 ones = (col == 0) ? pack4(1.0f, 1.0f, 1.0f, 1.0f) : s4{0, 0, 0, 0};
                gW2[a][8] = mfma16(A2, ones, gW2[a][8]);
                s4 A1 = lds_s4(&s.dA1T[ww][(mt * 16 + col) * 16 + 4 * g]);
                gW1[a] = mfma16(A1, lds_s4(&s.XeT[ww][col * 16 + 4 * g]), gW1[a]);
                s4 H2 = lds_s4(&s.H2T[ww][(mt * 16 + col) * 16 + 4 * g]);
                gW3[a] = mfma16(H2, lds_s4(&s.dzT[ww][col * 16 + 4 * g]), gW3[a]);
            }
        }
        __syncthreads();
    }
    // write this block's partial gradient in the flat layout
    float *out = part + (int64_t)blockIdx.x * (kParams + 1);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int mt = 2 * w + a;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = mt * 16 + 4 * g + r;
#pragma unroll
            for (int nt = 0; nt < 8; ++nt)
                out[kOffW2 + j * kHid + nt * 16 + col] = gW2[a][nt][r];
            if (col == 0)
                out[kOffB2 + j] = gW2[a][8][r];
            if (col < kIn)
                out[kOffW1 + j * kIn + col] = gW1[a][r];
            if (col == kIn)
                out[kOffB1 + j] = gW1[a][r];
            if (col == 0)
                out[kOffW3 + j] = gW3[a][r];
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
        out[kOffB3] = red_b3[0] + red_b3[1] + red_b3[2] + red_b3[3];
        out[kParams] = red_sq[0] + red_sq[1] + red_sq[2] + red_sq[3];
    }
}

// Part 2: sum the block partials in a fixed order.
__global__ void mlp_reduce_kernel(const float *part, int nblocks, float *grad)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kParams)
        return;
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b)
        s += part[(int64_t)b * (kParams + 1) + p];
    grad[p] = (float)s;
}

// Part 3: Adam (bias-corrected) on the FP32 masters, then the bf16 copies.
__global__ void mlp_adam_kernel(float *master, float *m, float *v, const float *grad, int64_t step, float lr,
                                float beta1, float beta2, float eps)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kParams)
        return;
    float gr = grad[p];
    float mm = beta1 * m[p] + (1.0f - beta1) * gr;
    float vv = beta2 * v[p] + (1.0f - beta2) * gr * gr;
    m[p] = mm;
    v[p] = vv;
    float mh = mm / (1.0f - powf(beta1, (float)step));
    float vh = vv / (1.0f - powf(beta2, (float)step));
    master[p] -= lr * mh / (sqrtf(vh) + eps);
}

// FP32 masters -> packed network (bf16 matrices, bf16-rounded vectors).
__global__ void mlp_pack_kernel(const float *master, MlpPacked *net)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kHid * 16) {
        int j = p / 16, k = p % 16;
        net->W1[p] = k < kIn ? bf16_bits(master[kOffW1 + j * kIn + k]) : (unsigned short)0;
    }
    if (p < kHid * kHid)
        net->W2[p] = bf16_bits(master[kOffW2 + p]);
    if (p < kHid) {
        net->b1[p] = bf16_value(bf16_bits(master[kOffB1 + p]));
        net->b2[p] = bf16_value(bf16_bits(master[kOffB2 + p]));
        net->W3[p] = bf16_value(bf16_bits(master[kOffW3 + p]));
    }
    if (p == 0)
        net->b3 = bf16_value(bf16_bits(master[kOffB3]));
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

hipError_t launch_mlp_train(const MlpPacked *net, const float *X, const float *y, int64_t n, float scale,
                            float *part, int nblocks, hipStream_t s)
{
    size_t lds = sizeof(TrainLds);
    (void)hipFuncSetAttribute((const void *)mlp_train_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(mlp_train_kernel, dim3((unsigned)nblocks), dim3(256), lds, s, net, X, y, n, scale, part);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce(const float *part, int nblocks, float *grad, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((kParams + 1 + 255) / 256), dim3(256), 0, s, part, nblocks, grad);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *master, float *m, float *v, const float *grad, int64_t step, float lr,
                           hipStream_t s)
{
    hipLaunchKernelGGL(mlp_adam_kernel, dim3((kParams + 255) / 256), dim3(256), 0, s, master, m, v, grad, step, lr,
                       0.9f, 0.999f, 1e-8f);
    return hipGetLastError();
}

hipError_t launch_mlp_pack(const float *master, MlpPacked *net, hipStream_t s)
{
    hipLaunchKernelGGL(mlp_pack_kernel, dim3((kHid * kHid + 255) / 256), dim3(256), 0, s, master, net);
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
