// push.hip -- per-particle kernels: merge of the pair partials, centred
// dipole, Higuera-Cary push, drift and history update (Secs. 2.3, 2.6 of
// arXiv 2605.05543), the straight-line prior history, layout conversions
// and bunch diagnostics (Secs. 2.5, 2.7).
#include "empp_dev.h"
#include "pair_common.h"

namespace empp {

// Light-cone records of every (source j, slot b) at the present time T[head]
// (b = 0 the newest slot): rec[j D + b] = {-2 D, L^2 - |D|^2} with
// D = w_n - w_b and L = c (T[head] - T_b), the per-sample part of the split
// sign test (lightcone_record).  Written once per pair pass, so that the
// pair kernels' target blocks stage them instead of each recomputing them.
__global__ void lightcone_records_kernel(const double4 *ring_w, const double *T, int64_t N, int D, int head,
                                         double4 *rec)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= N * (int64_t)D)
        return;
    const int64_t j = q / D;
    const int b = (int)(q - j * D);
    int ph = head - b;
    ph += ph < 0 ? D : 0;
    const double L = kC_LIGHT * (T[head] - T[ph]);
    const double4 wn = ring_w[j * D + head];
    rec[q] = lightcone_record(make_double4(wn.x, wn.y, wn.z, 0.0), ring_w[j * D + ph], L);
}

hipError_t launch_lightcone_records(const double4 *ring_w, const double *T, int64_t N, int D, int head,
                                    double4 *rec, hipStream_t s)
{
    const int64_t n = N * (int64_t)D;
    hipLaunchKernelGGL(lightcone_records_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ring_w, T, N, D,
                       head, rec);
    return hipGetLastError();
}

// Merge nsplit (sum, comp) partials of one component in split order.
__device__ inline double merge_partials(const double *part, int nsplit, int64_t m, int k, int64_t a)
{
    double s = 0.0, c = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) {
        const double *base = part + (int64_t)sp * 12 * m;
        neumaier(s, c, base[k * m + a]);
        neumaier(s, c, base[(6 + k) * m + a]);
    }
    return s + c;
}

// One thread per (component, target): the six field components of a
// target are merged by six threads, which keeps enough loads in flight
// for the nsplit x 12 x m partials.  The partials are in the pair launch's
// target order; order[a] (null: the identity) is the particle index that
// target a's fields are written at.
__global__ void merge_fields_kernel(const double *part, int nsplit, int64_t m, const int32_t *order, double *E,
                                    double *B)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 6 * m)
        return;
    const int k = (int)(idx / m);
    const int64_t a = idx - (int64_t)k * m;
    const double v = merge_partials(part, nsplit, m, k, a);
    const int64_t t = order ? (int64_t)order[a] : a;
    if (k < 3)
        E[k * m + t] = v;
    else
        B[(k - 3) * m + t] = v;
}

// Sec. 2.6: B = (mu0/4pi)(3 (M.rhat) rhat - M)/r^3 with M = M0 e_z, written
// with dip_k = (mu0/4pi) M0 = b0 re^3.
__device__ inline void dipole_field(double x, double y, double z, double dip_k, double &bx, double &by,
                                    double &bz)
{
    double r2 = x * x + y * y + z * z;
    double ir = 1.0 / sqrt(r2);
    double ir3 = ir * ir * ir;
    double mr = z * ir;  // M_hat . r_hat
    double f = dip_k * ir3;
    bx = f * (3.0 * mr * x * ir);
    by = f * (3.0 * mr * y * ir);
    bz = f * (3.0 * mr * z * ir - 1.0);
}

// Sec. 2.3, Higuera-Cary: half electric kick, magnetic rotation with the
// time-centred Lorentz factor gamma+, second half kick (the rotation's
// last term uses u+).
__device__ inline void higuera_cary(double &ux, double &uy, double &uz, double Ex, double Ey, double Ez,
                                    double Bx, double By, double Bz, double eps)
{
    const double c = kC_LIGHT;
    const double ic2 = 1.0 / (c * c);
    double umx = ux + eps * Ex, umy = uy + eps * Ey, umz = uz + eps * Ez;
    double tx = eps * Bx, ty = eps * By, tz = eps * Bz;
    double gm2 = 1.0 + (umx * umx + umy * umy + umz * umz) * ic2;
    double ustar = (umx * tx + umy * ty + umz * tz) / c;
    double tau2 = tx * tx + ty * ty + tz * tz;
    double sig = gm2 - tau2;
    double gp = sqrt(0.5 * (sig + sqrt(sig * sig + 4.0 * (tau2 + ustar * ustar))));
    double igp = 1.0 / gp;
    tx *= igp;
    ty *= igp;
    tz *= igp;
    double s = 1.0 / (1.0 + tx * tx + ty * ty + tz * tz);
    double ut = umx * tx + umy * ty + umz * tz;
    double upx = s * (umx + ut * tx + (umy * tz - umz * ty));
    double upy = s * (umy + ut * ty + (umz * tx - umx * tz));
    double upz = s * (umz + ut * tz + (umx * ty - umy * tx));
    ux = upx + eps * Ex + (upy * tz - upz * ty);
    uy = upy + eps * Ey + (upz * tx - upx * tz);
    uz = upz + eps * Ez + (upx * ty - upy * tx);
}

// One push per particle: merge the self-field partials, add the dipole,
// Higuera-Cary, finalise the newest slot's velocity, drift, and write the
// new newest slot at physical index head+1.
__global__ void push_kernel(PushParams p)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p.ad) {
        // Sec. 2.4: this step's dt from the pair kernel's reductions (the
        // same value in every thread); the clock lives in T[head]
        const double eta_min = __longlong_as_double((long long)p.ad[0]);
        const double v_max = sqrt(__longlong_as_double((long long)p.ad[1]));
        double dt = p.dt_max;
        if (v_max > 0.0 && eta_min < __longlong_as_double((long long)kPosInfBits))
            dt = fmin(p.dt_max, fmax(p.dt_min, p.c_dt * eta_min / v_max));
        p.dt = dt;
        p.eps = p.q * dt / (2.0 * p.m);
        p.t_now = p.T[p.head];
        p.t_next = p.t_now + dt;
        if (i == 0) {
            p.ad_next[0] = kPosInfBits;
            p.ad_next[1] = 0ull;
            p.dt_out[0] = dt;
        }
    }
    if (i >= p.N)
        return;
    const int D = p.D;
    // self-fields merged from the pair partials by merge_fields_kernel
    double Ex = 0, Ey = 0, Ez = 0, Bx = 0, By = 0, Bz = 0;
    if (p.self_field) {
        Ex = p.E[i];
        Ey = p.E[p.N + i];
        Ez = p.E[2 * p.N + i];
        Bx = p.B[i];
        By = p.B[p.N + i];
        Bz = p.B[2 * p.N + i];
    }
    double4 y = p.ring_w[i * D + p.head];
    if (p.ext_field == 1) {
        double gx, gy, gz;
        dipole_field(y.x, y.y, y.z, p.dip_k, gx, gy, gz);
        Bx += gx;
        By += gy;
        Bz += gz;
    }
    double ux = p.u[i], uy = p.u[p.N + i], uz = p.u[2 * p.N + i];
    higuera_cary(ux, uy, uz, Ex, Ey, Ez, Bx, By, Bz, p.eps);
    p.u[i] = ux;
    p.u[p.N + i] = uy;
    p.u[2 * p.N + i] = uz;
    const double c = kC_LIGHT;
    double g = sqrt(1.0 + (ux * ux + uy * uy + uz * uz) / (c * c));
    double ig = 1.0 / g;
    // velocity records carry 1/(T_{k+1} - T_k) of their segment in .w
    // (0 for the newest slot, which has no segment yet)
    double4 vn = make_double4(ux * ig, uy * ig, uz * ig, 1.0 / (p.t_next - p.t_now));
    p.ring_v[i * D + p.head] = vn;
    int nh = p.head + 1 == D ? 0 : p.head + 1;
    p.ring_w[i * D + nh] = make_double4(y.x + vn.x * p.dt, y.y + vn.y * p.dt, y.z + vn.z * p.dt, 0.0);
    vn.w = 0.0;
    p.ring_v[i * D + nh] = vn;
    if (i == 0)
        p.T[nh] = p.t_next;
}

// Straight-line prior history: logical slot k = -(D-1)..0 (physical
// index k + D - 1) at T_k = t0 + k dt, w_k = r + v0 (k dt), v_k = v0.
__global__ void init_straight_kernel(double4 *ring_w, double4 *ring_v, double *T, const double *r,
                                     const double *u, int64_t N, int D, double t0, double dt)
{
    // Rounded exactly as a plain IEEE evaluation (no fused multiply-add),
    // so that the stored history is reproducible bit for bit on any host.
#pragma clang fp contract(off)
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * D)
        return;
    int64_t i = idx / D;
    int s = (int)(idx - i * D);
    const double c = kC_LIGHT;
    double ux = u[i], uy = u[N + i], uz = u[2 * N + i];
    double g = sqrt(1.0 + ((ux * ux + uy * uy) + uz * uz) / (c * c));
    double vx = ux / g, vy = uy / g, vz = uz / g;
    int64_t k = (int64_t)s - (D - 1);
    double kdt = (double)k * dt;
    ring_w[idx] = make_double4(r[i] + vx * kdt, r[N + i] + vy * kdt, r[2 * N + i] + vz * kdt, 0.0);
    double inv_h = s + 1 < D ? 1.0 / ((t0 + (double)(k + 1) * dt) - (t0 + kdt)) : 0.0;
    ring_v[idx] = make_double4(vx, vy, vz, inv_h);
    if (i == 0)
        T[s] = t0 + kdt;
}

// [ns][3][N] component-major history (oldest first) -> ring layout with
// logical slot s at physical slot s (head = D - 1).
__global__ void history_to_ring_kernel(const double *w, const double *v, const double *T, double4 *ring_w,
                                       double4 *ring_v, int64_t N, int D)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * D)
        return;
    int64_t i = idx / D;
    int64_t s = idx - i * D;
    const double *ws = w + s * 3 * N;
    const double *vs = v + s * 3 * N;
    ring_w[idx] = make_double4(ws[i], ws[N + i], ws[2 * N + i], 0.0);
    double inv_h = s + 1 < D ? 1.0 / (T[s + 1] - T[s]) : 0.0;
    ring_v[idx] = make_double4(vs[i], vs[N + i], vs[2 * N + i], inv_h);
}

// Ring -> [D][3][N] oldest first (logical order).
__global__ void ring_to_history_kernel(const double4 *ring_w, const double4 *ring_v, double *w, double *v,
                                       int64_t N, int D, int head)
{
    int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * D)
        return;
    int64_t i = idx / D;
    int s = (int)(idx - i * D);          // logical slot, 0 = oldest
    int ph = head - (D - 1 - s);
    ph += ph < 0 ? D : 0;
    double4 a = ring_w[i * D + ph];
    double4 b = ring_v[i * D + ph];
    double *ws = w + (int64_t)s * 3 * N;
    double *vs = v + (int64_t)s * 3 * N;
    ws[i] = a.x;
    ws[N + i] = a.y;
    ws[2 * N + i] = a.z;
    vs[i] = b.x;
    vs[N + i] = b.y;
    vs[2 * N + i] = b.z;
}

__global__ void newest_positions_kernel(const double4 *ring_w, double *r, int64_t N, int D, int head)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N)
        return;
    double4 a = ring_w[i * D + head];
    r[i] = a.x;
    r[N + i] = a.y;
    r[2 * N + i] = a.z;
}

// Diagnostics partial sums per block: positions relative to particle 0's
// (so that offsets of Earth radii do not swamp millimetre spreads), their
// squares, and gamma - 1.  out[block][7] = {sx, sy, sz, sxx, syy, szz, sg}.
__global__ void diag_kernel(const double4 *ring_w, const double *u, int64_t N, int D, int head, double *out)
{
    __shared__ double red[7][kBlock];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    double4 ref = ring_w[head];
    if (i < N) {
        double4 y = ring_w[i * D + head];
        double dx = y.x - ref.x, dy = y.y - ref.y, dz = y.z - ref.z;
        v[0] = dx;
        v[1] = dy;
        v[2] = dz;
        v[3] = dx * dx;
        v[4] = dy * dy;
        v[5] = dz * dz;
        const double c = kC_LIGHT;
        double u2 = (u[i] * u[i] + u[N + i] * u[N + i] + u[2 * N + i] * u[2 * N + i]) / (c * c);
        v[6] = u2 / (sqrt(1.0 + u2) + 1.0);  // gamma - 1 without cancellation
    }
    for (int k = 0; k < 7; ++k)
        red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int k = 0; k < 7; ++k)
                red[k][threadIdx.x] += red[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int k = 0; k < 7; ++k)
            out[blockIdx.x * 7 + k] = red[k][0];
}

// ---- Stage II: prescribed field only (Sec. 2.7) ---------------------------

// gamma / |B| of one particle, +inf where it sees no field.
__device__ inline double gyro_key(double4 y, double ux, double uy, double uz, double dip_k, int ext_field)
{
    if (ext_field != 1)
        return __longlong_as_double((long long)kPosInfBits);
    double bx, by, bz;
    dipole_field(y.x, y.y, y.z, dip_k, bx, by, bz);
    const double c = kC_LIGHT;
    double g = sqrt(1.0 + (ux * ux + uy * uy + uz * uz) / (c * c));
    double bm = sqrt(bx * bx + by * by + bz * bz);
    return bm > 0.0 ? g / bm : __longlong_as_double((long long)kPosInfBits);
}

// Block minimum of a positive double, folded into *slot with one atomic.
__device__ inline void block_min_to(double v, unsigned long long *slot)
{
    __shared__ double wmin[16];
    for (int off = 32; off > 0; off >>= 1)
        v = fmin(v, __shfl_xor(v, off));
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        wmin[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = wmin[0];
        for (int k = 1; k < (int)(blockDim.x >> 6); ++k)
            m = fmin(m, wmin[k]);
        atomicMin(slot, (unsigned long long)__double_as_longlong(m));
    }
}

// Positions of the newest slot -> compact Stage-II array; clears the three
// step slots and sets the clock.
__global__ void handoff_kernel(const double4 *ring_w, int D, int head, double4 *pos, int64_t N,
                               unsigned long long *key, double *t, double t_now)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) {
        double4 y = ring_w[i * D + head];
        pos[i] = make_double4(y.x, y.y, y.z, 0.0);
    }
    if (i == 0) {
        key[0] = key[1] = key[2] = kPosInfBits;
        t[0] = t_now;
    }
}

// The first step's minimum (slot 0) from the handed-off state.
__global__ void transport_key_kernel(const double4 *pos, const double *u, int64_t N, double dip_k, int ext_field,
                                     unsigned long long *key)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double k = __longlong_as_double((long long)kPosInfBits);
    if (i < N)
        k = gyro_key(pos[i], u[i], u[N + i], u[2 * N + i], dip_k, ext_field);
    block_min_to(k, key);
}

// One Stage-II step: E = 0, B = B_geo, Higuera-Cary, drift with the new
// velocity; then the next step's gamma / |B| at the new state.
__global__ void transport_kernel(TransportParams p)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s0 = (int)(p.step % 3);
    const int s1 = s0 == 2 ? 0 : s0 + 1;
    const int s2 = s1 == 2 ? 0 : s1 + 1;
    const double kmin = __longlong_as_double((long long)p.key[s0]);
    double dt = p.dt_max;
    const double d = p.gyro_k * kmin;
    if (d < dt)
        dt = d;
    double knext = __longlong_as_double((long long)kPosInfBits);
    if (i < p.N) {
        double4 y = p.pos[i];
        double bx = 0.0, by = 0.0, bz = 0.0;
        if (p.ext_field == 1)
            dipole_field(y.x, y.y, y.z, p.dip_k, bx, by, bz);
        double ux = p.u[i], uy = p.u[p.N + i], uz = p.u[2 * p.N + i];
        higuera_cary(ux, uy, uz, 0.0, 0.0, 0.0, bx, by, bz, p.q_over_2m * dt);
        const double c = kC_LIGHT;
        double ig = 1.0 / sqrt(1.0 + (ux * ux + uy * uy + uz * uz) / (c * c));
        y = make_double4(y.x + ux * ig * dt, y.y + uy * ig * dt, y.z + uz * ig * dt, 0.0);
        p.pos[i] = y;
        p.u[i] = ux;
        p.u[p.N + i] = uy;
        p.u[2 * p.N + i] = uz;
        knext = gyro_key(y, ux, uy, uz, p.dip_k, p.ext_field);
    }
    block_min_to(knext, p.key + s1);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        p.key[s2] = kPosInfBits;
        p.t[0] += dt;
    }
}

hipError_t launch_handoff(const double4 *ring_w, int D, int head, double4 *pos, const double *u, int64_t N,
                          double dip_k, int ext_field, unsigned long long *key, double *t, double t_now,
                          hipStream_t s)
{
    const unsigned nb = (unsigned)((N + 255) / 256);
    hipLaunchKernelGGL(handoff_kernel, dim3(nb), dim3(256), 0, s, ring_w, D, head, pos, N, key, t, t_now);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(transport_key_kernel, dim3(nb), dim3(256), 0, s, (const double4 *)pos, u, N, dip_k,
                       ext_field, key);
    return hipGetLastError();
}

hipError_t launch_transport(const TransportParams &p, hipStream_t s)
{
    hipLaunchKernelGGL(transport_kernel, dim3((unsigned)((p.N + 255) / 256)), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_merge_fields(const double *part, int nsplit, int64_t m, const int32_t *order, double *E,
                               double *B, hipStream_t s)
{
    hipLaunchKernelGGL(merge_fields_kernel, dim3((unsigned)((6 * m + 255) / 256)), dim3(256), 0, s, part, nsplit,
                       m, order, E, B);
    return hipGetLastError();
}

// Merge of the self-field partials into E, B, then the push.
hipError_t launch_push(const PushParams &p, hipStream_t s)
{
    if (p.self_field) {
        hipError_t e = launch_merge_fields(p.part, p.nsplit, p.N, p.order, p.E, p.B, s);
        if (e != hipSuccess)
            return e;
    }
    hipLaunchKernelGGL(push_kernel, dim3((unsigned)((p.N + 255) / 256)), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_init_straight(double4 *rw, double4 *rv, double *T, const double *r, const double *u, int64_t N,
                                int D, double t0, double dt, hipStream_t s)
{
    int64_t tot = N * D;
    hipLaunchKernelGGL(init_straight_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, rw, rv, T, r, u,
                       N, D, t0, dt);
    return hipGetLastError();
}

hipError_t launch_history_to_ring(const double *w, const double *v, const double *T, double4 *rw, double4 *rv,
                                  int64_t N, int D, hipStream_t s)
{
    int64_t tot = N * D;
    hipLaunchKernelGGL(history_to_ring_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, w, v, T, rw,
                       rv, N, D);
    return hipGetLastError();
}

hipError_t launch_ring_to_history(const double4 *rw, const double4 *rv, double *w, double *v, int64_t N, int D,
                                  int head, hipStream_t s)
{
    int64_t tot = N * D;
    hipLaunchKernelGGL(ring_to_history_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, s, rw, rv, w, v,
                       N, D, head);
    return hipGetLastError();
}

hipError_t launch_newest_positions(const double4 *rw, double *r, int64_t N, int D, int head, hipStream_t s)
{
    hipLaunchKernelGGL(newest_positions_kernel, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, rw, r, N, D,
                       head);
    return hipGetLastError();
}

hipError_t launch_diag(const double4 *rw, const double *u, int64_t N, int D, int head, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(diag_kernel, dim3((unsigned)((N + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, rw, u, N, D,
                       head, out);
    return hipGetLastError();
}

}  // namespace empp
