// pair_mixed.hip -- mixed-precision all-pairs Lienard-Wiechert evaluation.
//
// Same method and bracket as the FP64 kernel (Secs. 2.1-2.2 of arXiv
// 2605.05543), with the precision split:
//  * FP64: absolute positions and times (the history in HBM), the offset
//    r - w_1 of the bracket sample, the light-cone residual at the root
//    C0 = L1^2 - |r - w_1|^2 and the other coefficients of the quadratic,
//    the velocity at the root, the vector eta - |eta| v/c whose length is
//    the cancellation-prone 1 - eta_hat.beta, every sign test that falls
//    inside the FP32 rounding band, and the root whenever the FP32 root
//    fails its residual test.
//  * FP32: history offsets relative to each source's newest position (the
//    LDS tile, 16 bytes per slot instead of 32), the sign tests, the
//    quadratic, the reconstruction and the LW terms; the field sum is
//    accumulated with Knuth's two-sum into an FP32 (sum, error) pair.
// The bracket index is identical to the FP64 path: an FP32 sign test is
// trusted only outside a band that bounds its rounding error; inside it
// the sample is re-tested in FP64 exactly as the FP64 path does.
#include "pair_common.h"

namespace empp {

extern const bool kHaveMixed = true;

namespace {

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
    double4 w1, v1, v2;  // FP64 records of the bracket (global memory)
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
__device__ __forceinline__ bool lw_pair_mixed(double rx, double ry, double rz, double L1d, MixedPair q, bool before,
                                              float kq, float f[6], bool &rescued)
{
    const double c = kC_LIGHT;
    const double ic = 1.0 / kC_LIGHT;
    const float cf = (float)kC_LIGHT;
    // FP64: offset to the bracket sample and the quadratic's coefficients
    double dxd = rx - q.w1.x, dyd = ry - q.w1.y, dzd = rz - q.w1.z;
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
        double sqd = sqrt(ok ? discd : 0.0);
        double rd = C1hd <= 0.0 ? C0d / (sqd - C1hd) : -(C1hd + sqd) / C2d;
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
    float hx = ex * ien, hy = ey * ien, hz = ez * ien;
    // c^2 - |v_r|^2 from the FP64 value at v_1 plus the small correction
    float cv = C2 - df * (2.0f * (vx * gx + vy * gy + vz * gz) + df * (gx * gx + gy * gy + gz * gz));
    float qx = py * az - pz * ay, qy = pz * ax - px * az, qz = px * ay - py * ax;
    float rdx = ey * qz - ez * qy, rdy = ez * qx - ex * qz, rdz = ex * qy - ey * qx;
    float pref = kq * en * (iev * iev * iev);
    float Ex = pref * (cv * px + rdx);
    float Ey = pref * (cv * py + rdy);
    float Ez = pref * (cv * pz + rdz);
    const float icf = (float)ic;
    f[0] = Ex;
    f[1] = Ey;
    f[2] = Ez;
    f[3] = (hy * Ez - hz * Ey) * icf;
    f[4] = (hz * Ex - hx * Ez) * icf;
    f[5] = (hx * Ey - hy * Ex) * icf;
    return ok;
}

}  // namespace

// LDS tile: S sources x D slots of float4 {x', y', z', L^2} with
// x' = x - (newest x of the source), then the FP64 light distances Ls[D]
// and the FP64 anchors (newest positions) of the tile's sources.
template <bool KSTAR, bool COUNT, int GUESS, int S>
__global__ __launch_bounds__(kBlock) void pair_mixed_kernel(PairParams p)
{
    extern __shared__ float4 ldsf[];
    const int D = p.D;
    float4 *recs = ldsf;
    double *Ls = reinterpret_cast<double *>(ldsf + S * D);
    double4 *anchor = reinterpret_cast<double4 *>(Ls + D);
    const int tid = threadIdx.x;
    const int nbx = (int)((p.m + kBlock - 1) / kBlock);
    int bxi, split;
    pair_block_coords(nbx, p.nsplit, bxi, split);
    const int64_t a = (int64_t)bxi * kBlock + tid;
    const bool active = a < p.m;
    const int64_t j0 = (int64_t)split * p.src_per_split;
    int64_t j1 = j0 + p.src_per_split;
    if (j1 > p.n_src)
        j1 = p.n_src;

    double rx = 0, ry = 0, rz = 0;
    int64_t self = -1, tgt = a;
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
        }
    }
    // the present time is the newest slot's (the clock lives in T)
    const double tnow = p.T[p.head];
    for (int b = tid; b < D; b += kBlock) {
        int ph = p.head - b;
        ph += ph < 0 ? D : 0;
        Ls[b] = kC_LIGHT * (tnow - p.T[ph]);
    }
    __syncthreads();
    const double Lmax = Ls[D - 1];
    const float kq = (float)p.kq;
    float sum[6] = {0, 0, 0, 0, 0, 0}, err[6] = {0, 0, 0, 0, 0, 0};
    int probes = 0, nbefore = 0, npairs = 0, nfall = 0, nresc = 0;
    bool failed = false;
    int64_t fail_j = 0;
    const float inv_cdt = (float)(1.0 / (kC_LIGHT * p.dt));

    for (int64_t jt = j0; jt < j1; jt += S) {
        const int ns = (int)((j1 - jt) < S ? (j1 - jt) : S);
        __syncthreads();
        if (tid < ns)
            anchor[tid] = p.ring_w[(jt + tid) * D + p.head];
        for (int s = 0; s < ns; ++s) {
            const double4 *src = p.ring_w + (jt + s) * D;
            const double4 an = src[p.head];
            for (int b = tid; b < D; b += kBlock) {
                int ph = p.head - b;
                ph += ph < 0 ? D : 0;
                double4 w = src[ph];
                double L = Ls[b];
                recs[s * D + b] = make_float4((float)(w.x - an.x), (float)(w.y - an.y), (float)(w.z - an.z),
                                              (float)(L * L));
            }
        }
        __syncthreads();
        if (!active)
            continue;

        bool valid[S];
        int64_t jj[S];
        int bk[S];
        float Rx[S], Ry[S], Rz[S], band[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            jj[s] = jt + (s < ns ? s : 0);
            valid[s] = s < ns && jj[s] != self;
            if (KSTAR && s < ns && jj[s] == self)
                p.kstar[a * p.n_src + jj[s]] = 0;
            double4 an = anchor[s < ns ? s : 0];
            double Rxd = rx - an.x, Ryd = ry - an.y, Rzd = rz - an.z;
            if (valid[s] && Rxd == 0.0 && Ryd == 0.0 && Rzd == 0.0) {
                // a target on the source's present position: eta = 0
                if (!failed)
                    fail_j = jj[s];
                failed = true;
                valid[s] = false;
            }
            Rx[s] = (float)Rxd;
            Ry[s] = (float)Ryd;
            Rz[s] = (float)Rzd;
            // |f32 - f| <= 8u (L^2 + M^2) with M >= |r - a| + |w - a|; |w - a| <= Lmax
            // because no stored segment moves faster than light; twice that.
            float M = fabsf(Rx[s]) + fabsf(Ry[s]) + fabsf(Rz[s]) + (float)Lmax;
            band[s] = 16.0f * 5.9604645e-8f * ((float)(Lmax * Lmax) + M * M);
        }
        // sign test of logical slot b of tile source s: FP32 outside the
        // rounding band, FP64 (the FP64 path's exact test) inside it
        auto test = [&](int s, int b) -> bool {
            float4 w = recs[s * D + b];
            float dx = Rx[s] - w.x, dy = Ry[s] - w.y, dz = Rz[s] - w.z;
            float fm = w.w - (dx * dx + dy * dy + dz * dz);
            if (fabsf(fm) > band[s])
                return fm > 0.0f;
            if (COUNT)
                nresc += 1;
            int ph = p.head - b;
            ph += ph < 0 ? D : 0;
            double4 rec = p.ring_w[jj[s] * D + ph];
            double L = Ls[b];
            rec.w = L * L;
            return lightcone_positive(rec, rx, ry, rz);
        };

        if (GUESS == 0) {
            bool inside[S];
            int xb[S];
#pragma unroll
            for (int s = 0; s < S; ++s) {
                inside[s] = test(s, D - 1);
                xb[s] = 0;
            }
            bool any = false;
#pragma unroll
            for (int s = 0; s < S; ++s)
                any = any || (inside[s] && valid[s]);
            if (__any(any)) {
                for (int n = D - 1; n > 1;) {
                    const int half = n >> 1;
#pragma unroll
                    for (int s = 0; s < S; ++s) {
                        int m = xb[s] + half;
                        bool fpos = test(s, m);
                        xb[s] = fpos ? xb[s] : m;
                    }
                    n -= half;
                }
            }
#pragma unroll
            for (int s = 0; s < S; ++s) {
                bk[s] = inside[s] ? xb[s] + 1 : -1;
                if (COUNT && valid[s])
                    probes += inside[s] ? 1 + p.nit : 1;
            }
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                bk[s] = -1;
                if (!valid[s])
                    continue;
                auto t1 = [&](int b) { return test(s, b); };
                float g;
                if (GUESS == 2) {
                    double4 vn = p.ring_v[jj[s] * D + p.head];
                    g = ballistic_steps((double)Rx[s], (double)Ry[s], (double)Rz[s], vn, inv_cdt);
                } else if (p.g_ratio) {
                    // surrogate, one evaluation per group: the group's
                    // correction factor to straight-line motion times this
                    // target's straight-line look-back
                    double4 vn = p.ring_v[jj[s] * D + p.head];
                    float gh = p.G[jj[s] * p.g_groups + (a >> p.g_shift)];
                    g = gh * ballistic_steps((double)Rx[s], (double)Ry[s], (double)Rz[s], vn, inv_cdt);
                } else {
                    // surrogate per pair: predicted c (t - t_r) / |r - w_n| times the distance
                    float gh = p.G[jj[s] * p.g_groups + (a >> p.g_shift)];
                    g = gh * __builtin_amdgcn_sqrtf(Rx[s] * Rx[s] + Ry[s] * Ry[s] + Rz[s] * Rz[s]) * inv_cdt;
                }
                int fb = 0;
                bk[s] = search_guided(t1, D, g, 6, probes, fb);
                nfall += fb;
            }
        }

        MixedPair q[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bool before = bk[s] < 0;
            const int bb = before ? D - 1 : bk[s];
            int ph1 = p.head - bb;
            ph1 += ph1 < 0 ? D : 0;
            int ph2 = ph1 + 1 == D ? 0 : ph1 + 1;
            q[s].w1 = p.ring_w[jj[s] * D + ph1];
            q[s].v1 = p.ring_v[jj[s] * D + ph1];
            q[s].v2 = p.ring_v[jj[s] * D + ph2];  // unused (inv_h = 0) out of history
        }
        float acc[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int s = 0; s < S; ++s) {
            const bool before = bk[s] < 0;
            const int bb = before ? D - 1 : bk[s];
            float f[6];
            bool resc = false;
            bool ok = lw_pair_mixed(rx, ry, rz, Ls[bb], q[s], before, kq, f, resc);
            if (valid[s]) {
                if (ok) {
#pragma unroll
                    for (int k = 0; k < 6; ++k)
                        acc[k] += f[k];
                } else {
                    if (!failed)
                        fail_j = jj[s];
                    failed = true;
                }
                if (KSTAR)
                    p.kstar[a * p.n_src + jj[s]] = before ? -1 : bk[s];
                if (COUNT) {
                    npairs += 1;
                    nbefore += before ? 1 : 0;
                    nresc += resc ? 1 : 0;
                }
            }
        }
#pragma unroll
        for (int k = 0; k < 6; ++k)
            two_sum(sum[k], err[k], acc[k]);
    }
    if (active) {
        double *out = p.part + (int64_t)split * 12 * p.m + tgt;
        for (int k = 0; k < 6; ++k) {
            out[k * p.m] = (double)sum[k];
            out[(6 + k) * p.m] = (double)err[k];
        }
        if (failed)
            report_error(p.err, tgt, fail_j, kErrCoincident);
    }
    if (COUNT) {
        unsigned long long c0 = npairs, c1 = nbefore, c2 = probes, c3 = nresc, c4 = nfall;
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
            atomicAdd(&p.counters[3], c3);
            atomicAdd(&p.counters[4], c4);
        }
    }
}

// Sources per LDS tile (FP32 records, 16 bytes per slot).
int pair_mixed_tile(int D) { return D <= 2048 ? 2 : 1; }

hipError_t launch_pair_mixed(const PairParams &p0, hipStream_t stream, bool kstar, bool count)
{
    PairParams p = p0;
    p.tile = pair_mixed_tile(p.D);
    const int64_t nblocks = (p.m + kBlock - 1) / kBlock * p.nsplit;
    if (nblocks < 1 || nblocks > INT32_MAX)
        return hipErrorInvalidConfiguration;
    dim3 grid((unsigned)nblocks);
    size_t lds = (size_t)p.tile * p.D * sizeof(float4) + (size_t)p.D * sizeof(double) + 4 * sizeof(double4);
#define EMPP_LAUNCH(K, C, G, S)                                                                              \
    do {                                                                                                    \
        if (lds > 65536)                                                                                    \
            (void)hipFuncSetAttribute((const void *)pair_mixed_kernel<K, C, G, S>,                          \
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);                \
        hipLaunchKernelGGL((pair_mixed_kernel<K, C, G, S>), grid, dim3(kBlock), lds, stream, p);            \
    } while (0)
#define EMPP_BY_TILE(K, C, G)                                                                                \
    do {                                                                                                    \
        if (p.tile == 4) EMPP_LAUNCH(K, C, G, 4);                                                            \
        else if (p.tile == 2) EMPP_LAUNCH(K, C, G, 2);                                                       \
        else EMPP_LAUNCH(K, C, G, 1);                                                                        \
    } while (0)
#define EMPP_BY_GUESS(K, C)                                                                                  \
    do {                                                                                                    \
        if (p.guess == 2) EMPP_BY_TILE(K, C, 2);                                                             \
        else if (p.guess == 1) EMPP_BY_TILE(K, C, 1);                                                        \
        else EMPP_BY_TILE(K, C, 0);                                                                          \
    } while (0)
    if (kstar) {
        if (count) EMPP_BY_GUESS(true, true); else EMPP_BY_GUESS(true, false);
    } else {
        if (count) EMPP_BY_GUESS(false, true); else EMPP_BY_GUESS(false, false);
    }
#undef EMPP_BY_GUESS
#undef EMPP_BY_TILE
#undef EMPP_LAUNCH
    return hipGetLastError();
}

}  // namespace empp
