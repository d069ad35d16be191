// pair_fp64.hip -- all-pairs Lienard-Wiechert field evaluation in double
// precision (Secs. 2.1-2.2 of arXiv 2605.05543).
//
// One thread owns one target.  A block of 256 targets walks its chunk of
// sources in tiles: the tile's histories (positions plus the light
// distance c (t - T_k) of every slot) are staged once into LDS and every
// target of the block then searches them, so each history byte read from
// HBM serves 256 targets.  The bracket velocities v_1, v_2 are read from
// the (L2-resident) history in HBM after the search.  Sums are kept per
// target in registers: a plain partial sum per tile, merged into a
// Neumaier-compensated total after each tile; source chunks (grid.y) write
// (sum, compensation) partials that the push kernel merges in a fixed
// order, so results do not depend on scheduling.
#include "pair_common.h"

namespace empp {

namespace {

struct LdsRec {
    const double4 *base;
    __device__ double4 operator()(int b) const { return base[b]; }
};

// Retarded root, reconstruction and LW field of one pair (Eqs. dt,
// linear, linear2, LW_E, LW_B).  w1 = {x, y, z, L1} is the bracket's older
// sample with L1 = c (t - t_1); v1, v2 the velocities of the bracket ends;
// inv_h = 1/(t_2 - t_1).  Adds E and B into acc[0..5].  Returns false on a
// numerical failure (negative discriminant or eta = 0).
__device__ inline bool lw_pair(double rx, double ry, double rz, double4 w1, double4 v1, double4 v2,
                               double inv_h, bool before, double kq, double acc[6])
{
    const double c = kC_LIGHT;
    const double c2 = c * c;
    double dx = rx - w1.x, dy = ry - w1.y, dz = rz - w1.z;
    double L1 = w1.w;
    // C2 dt^2 + C1 dt + C0 = 0 (Eq. dt); physical root in Vieta's form.
    double C2 = c2 - (v1.x * v1.x + v1.y * v1.y + v1.z * v1.z);
    double dv = dx * v1.x + dy * v1.y + dz * v1.z;
    double C1 = 2.0 * (dv - c * L1);
    double C0 = L1 * L1 - (dx * dx + dy * dy + dz * dz);
    double disc = C1 * C1 - 4.0 * C2 * C0;
    bool ok = disc >= 0.0;
    double sq = sqrt(fmax(disc, 0.0));
    double dtr = 2.0 * C0 * rcp64(sq - C1);
    // reconstruction: w = w1 + v1 dt; v = v1 + (v2 - v1) df; a = (v2 - v1)/h
    double ax = 0.0, ay = 0.0, az = 0.0, df = 0.0;
    if (!before) {
        ax = (v2.x - v1.x) * inv_h;
        ay = (v2.y - v1.y) * inv_h;
        az = (v2.z - v1.z) * inv_h;
        df = dtr * inv_h;
    }
    double vrx = v1.x + (v2.x - v1.x) * df;
    double vry = v1.y + (v2.y - v1.y) * df;
    double vrz = v1.z + (v2.z - v1.z) * df;
    if (before) {
        vrx = v1.x;
        vry = v1.y;
        vrz = v1.z;
    }
    double ex = dx - v1.x * dtr, ey = dy - v1.y * dtr, ez = dz - v1.z * dtr;  // eta
    // |eta| = c (t - t_r) on the reconstructed segment
    double en = L1 - c * dtr;
    ok = ok && (en > 0.0);
    double ien = rcp64(en);
    double hx = ex * ien, hy = ey * ien, hz = ez * ien;
    double px = c * hx - vrx, py = c * hy - vry, pz = c * hz - vrz;  // v'
    double ev = c * en - (ex * vrx + ey * vry + ez * vrz);            // eta . v'
    double vv = vrx * vrx + vry * vry + vrz * vrz;
    // eta x (v' x a)
    double qx = py * az - pz * ay, qy = pz * ax - px * az, qz = px * ay - py * ax;
    double rdx = ey * qz - ez * qy, rdy = ez * qx - ex * qz, rdz = ex * qy - ey * qx;
    double iev = rcp64(ev);
    double pref = kq * en * (iev * iev * iev);
    double cv = c2 - vv;
    double Ex = pref * (cv * px + rdx);
    double Ey = pref * (cv * py + rdy);
    double Ez = pref * (cv * pz + rdz);
    const double ic = 1.0 / c;
    double Bx = (hy * Ez - hz * Ey) * ic;
    double By = (hz * Ex - hx * Ez) * ic;
    double Bz = (hx * Ey - hy * Ex) * ic;
    if (ok) {
        acc[0] += Ex;
        acc[1] += Ey;
        acc[2] += Ez;
        acc[3] += Bx;
        acc[4] += By;
        acc[5] += Bz;
    }
    return ok;
}

}  // namespace

template <bool KSTAR, bool COUNT, int GUESS>
__global__ __launch_bounds__(kBlock) void pair_fp64_kernel(PairParams p)
{
    extern __shared__ double4 lds[];
    const int D = p.D;
    const int tid = threadIdx.x;
    const int64_t a = (int64_t)blockIdx.x * kBlock + tid;
    const bool active = a < p.m;
    const int split = blockIdx.y;
    const int64_t j0 = (int64_t)split * p.src_per_split;
    int64_t j1 = j0 + p.src_per_split;
    if (j1 > p.n_src)
        j1 = p.n_src;

    double rx = 0, ry = 0, rz = 0;
    int64_t self = -1;
    if (active) {
        if (p.x) {
            rx = p.x[a];
            ry = p.x[p.m + a];
            rz = p.x[2 * p.m + a];
            self = p.self_index ? p.self_index[a] : -1;
        } else {
            double4 w = p.ring_w[a * D + p.head];
            rx = w.x;
            ry = w.y;
            rz = w.z;
            self = a;
        }
    }
    double sum[6] = {0, 0, 0, 0, 0, 0}, comp[6] = {0, 0, 0, 0, 0, 0};
    int probes = 0, nbefore = 0, npairs = 0, nfall = 0;
    bool failed = false;
    int64_t fail_j = 0;
    const float inv_cdt = (float)(1.0 / (kC_LIGHT * p.dt));

    for (int64_t jt = j0; jt < j1; jt += p.tile) {
        const int ns = (int)((j1 - jt) < p.tile ? (j1 - jt) : p.tile);
        __syncthreads();
        for (int s = 0; s < ns; ++s) {
            const double4 *src = p.ring_w + (jt + s) * D;
            for (int b = tid; b < D; b += kBlock) {
                int ph = p.head - b;
                ph += ph < 0 ? D : 0;
                double4 w = src[ph];
                w.w = kC_LIGHT * (p.t - p.T[ph]);
                lds[s * D + b] = w;
            }
        }
        __syncthreads();
        if (!active)
            continue;
        double acc[6] = {0, 0, 0, 0, 0, 0};
        for (int s = 0; s < ns; ++s) {
            const int64_t j = jt + s;
            if (j == self) {
                if (KSTAR)
                    p.kstar[a * p.n_src + j] = 0;
                continue;
            }
            LdsRec rec{lds + s * D};
            {
                // a target on the source's present position: eta = 0
                double4 wn = rec(0);
                if (rx == wn.x && ry == wn.y && rz == wn.z) {
                    if (!failed)
                        fail_j = j;
                    failed = true;
                    continue;
                }
            }
            int b;
            if (GUESS == 0) {
                b = search_bisect(rec, D, rx, ry, rz, probes);
            } else {
                double4 wn = rec(0);
                double4 vn = p.ring_v[j * D + p.head];
                float g = ballistic_steps(rx - wn.x, ry - wn.y, rz - wn.z, vn, inv_cdt);
                int fb = 0;
                b = search_guided(rec, D, rx, ry, rz, g, 6, probes, fb);
                nfall += fb;
            }
            const bool before = b < 0;
            const int bb = before ? D - 1 : b;
            int ph1 = p.head - bb;
            ph1 += ph1 < 0 ? D : 0;
            int ph2 = ph1 + 1 == D ? 0 : ph1 + 1;
            double4 w1 = rec(bb);
            double4 v1 = p.ring_v[j * D + ph1];
            double4 v2 = before ? v1 : p.ring_v[j * D + ph2];
            double inv_h = before ? 0.0 : rcp64(p.T[ph2] - p.T[ph1]);
            if (!lw_pair(rx, ry, rz, w1, v1, v2, inv_h, before, p.kq, acc)) {
                if (!failed)
                    fail_j = j;
                failed = true;
            }
            if (KSTAR)
                p.kstar[a * p.n_src + j] = before ? -1 : b;
            if (COUNT) {
                npairs += 1;
                nbefore += before ? 1 : 0;
            }
        }
        for (int k = 0; k < 6; ++k)
            neumaier(sum[k], comp[k], acc[k]);
    }
    if (active) {
        double *out = p.part + (int64_t)split * 12 * p.m + a;
        for (int k = 0; k < 6; ++k) {
            out[k * p.m] = sum[k];
            out[(6 + k) * p.m] = comp[k];
        }
        if (failed)
            report_error(p.err, a, fail_j, kErrCoincident);
    }
    if (COUNT) {
        // one atomic per wavefront
        unsigned long long v0 = npairs, v1 = nbefore, v2 = probes, v3 = nfall;
        for (int off = 32; off > 0; off >>= 1) {
            v0 += __shfl_down(v0, off);
            v1 += __shfl_down(v1, off);
            v2 += __shfl_down(v2, off);
            v3 += __shfl_down(v3, off);
        }
        if ((tid & 63) == 0) {
            atomicAdd(&p.counters[0], v0);
            atomicAdd(&p.counters[1], v1);
            atomicAdd(&p.counters[2], v2);
            atomicAdd(&p.counters[4], v3);
        }
    }
}

// Host-side launcher (called from the C ABI layer).
hipError_t launch_pair_fp64(const PairParams &p, hipStream_t stream, bool kstar, bool count)
{
    dim3 grid((unsigned)((p.m + kBlock - 1) / kBlock), (unsigned)p.nsplit);
    size_t lds = (size_t)p.tile * p.D * sizeof(double4);
#define EMPP_LAUNCH(K, C, G) \
    hipLaunchKernelGGL((pair_fp64_kernel<K, C, G>), grid, dim3(kBlock), lds, stream, p)
    if (p.guess == 2) {
        if (kstar) { if (count) EMPP_LAUNCH(true, true, 2); else EMPP_LAUNCH(true, false, 2); }
        else { if (count) EMPP_LAUNCH(false, true, 2); else EMPP_LAUNCH(false, false, 2); }
    } else {
        if (kstar) { if (count) EMPP_LAUNCH(true, true, 0); else EMPP_LAUNCH(true, false, 0); }
        else { if (count) EMPP_LAUNCH(false, true, 0); else EMPP_LAUNCH(false, false, 0); }
    }
#undef EMPP_LAUNCH
    return hipGetLastError();
}

}  // namespace empp
