/*
 * empp_oracle.c -- plain FP64 CPU oracle of the EM-PP hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the HIP path is checked against.  It shares no code,
 * header, table or helper with the GPU library; only the test suite, the
 * package smoke check and the CPU-baseline leg of the benchmark may load it.
 *
 * Everything is IEEE double.  Build with -ffp-contract=off so that no
 * multiply-add is fused behind our back: the light-cone sign test that
 * decides the bracket index must round exactly as written.
 *
 * Paper sections followed (arXiv 2605.05543):
 *   Sec. 2.1  Lienard-Wiechert fields, Eqs. (LW_E), (LW_B); superposition.
 *   Sec. 2.2  retarded time: history bracket, bisection, linear
 *             reconstruction (Eq. dt, Eq. linear), out-of-history
 *             extrapolation (Eq. linear2).
 *   Sec. 2.3  Higuera-Cary pusher.
 *   Sec. 2.5  RMS sizes; Sec. 2.7 mean kinetic energy.
 *   Sec. 2.6  centred dipole field.
 *
 * Conventions (shared with the test-side Python wrapper only):
 *   history  T[ns], w[ns][3][N], v[ns][3][N]; slot 0 is the oldest, slot
 *            ns-1 the newest (the present time).
 *   targets  x[3][m];   fields E[3][m], B[3][m].
 *   kstar    [m][N] int32: slots back from the newest of the bracket's
 *            left end (1..ns-1), -1 when the retarded time is older than
 *            the history, 0 for the excluded self pair.
 *
 * Mutation hooks: compiling with -DMUT_<NAME> plants one deliberate
 * mistake (see the MUT_ blocks).  The test suite builds such variants to
 * show that its closed-form pins catch each of them.  The default build
 * defines none.
 */
#define _GNU_SOURCE
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- physical constants: CODATA 2018 exact/recommended values ---------- */
static const double C_LIGHT = 299792458.0;          /* m/s (exact)          */
static const double E_CHARGE = 1.602176634e-19;     /* C (exact)            */
static const double M_ELECTRON = 9.1093837015e-31;  /* kg                   */
static const double MU0 = 1.25663706212e-6;         /* N/A^2                */

static double eps0(void) { return 1.0 / (MU0 * C_LIGHT * C_LIGHT); }
static double coulomb_k(void) { return 1.0 / (4.0 * M_PI * eps0()); }

enum { OR_OK = 0, OR_EINVAL = 1, OR_ENUMERIC = 2, OR_ECHECK = 3 };

void oracle_constants(double out[6])
{
    out[0] = C_LIGHT;
    out[1] = E_CHARGE;
    out[2] = M_ELECTRON;
    out[3] = MU0;
    out[4] = eps0();
    out[5] = coulomb_k();
}

/* ---- small vector helpers (plain, no fusion) ---------------------------- */
static double dot3(const double a[3], const double b[3])
{
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

static void cross3(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

/* Neumaier's improved Kahan summation, one component. */
static void neumaier_add(double *sum, double *comp, double x)
{
    double t = *sum + x;
#ifdef MUT_NEUMAIER_SIGN
    if (fabs(*sum) >= fabs(x))
        *comp -= (*sum - t) + x;
    else
        *comp -= (x - t) + *sum;
#else
    if (fabs(*sum) >= fabs(x))
        *comp += (*sum - t) + x;
    else
        *comp += (x - t) + *sum;
#endif
    *sum = t;
}

/* ---- Sec. 2.2: light-cone sign of a stored sample --------------------------
 * f_k = c (t - T_k) - |r - w_k|.  Only its sign is needed, and both terms are
 * non-negative, so it is taken on squares: f_k > 0 <=> L^2 > |d|^2 with
 * L = c (t - T_k) and d = r - w_k.  Plain evaluation in the written order,
 * no fusion (the build forbids contraction):
 *     LL = L * L,   dd = (d_x d_x + d_y d_y) + d_z d_z,   positive: LL > dd.
 * An exact tie (LL == dd) goes to the older side, as the paper's bisection
 * sends c dt <= |r - w(t_m)| to the older half.
 *
 * Rounding.  On the stored doubles (t, T_k, r, w_k) the exact value is
 * F = L^2 - |d|^2.  L carries two roundings (the subtraction and the product
 * with c) and LL one more; each d_c^2 carries two and the sum two more, so
 * |(LL - dd) - F| <= gamma_5 (L^2 + |d|^2) with gamma_5 ~ 5 u, u = 2^-53.
 * Hence LL - dd has the sign of F whenever |LL - dd| > 2^-50 (LL + dd): the
 * decision is certified there.  Decisions with |LL - dd| <= NEAR_TIE (LL + dd),
 * NEAR_TIE = 2^-44, are reported as near ties: the band is 64 times the
 * certified bound, wide enough that any other FP64 evaluation order of the
 * same test may decide them either way, and every consumer of the bracket
 * accepts either neighbouring bracket there.                                */
#define NEAR_TIE 0x1p-44

typedef struct {
    int positive; /* decided f_k > 0                                    */
    int near;     /* |LL - dd| within the near-tie band                  */
} lc_sign_t;

static lc_sign_t lightcone_sign(const double r[3], const double wk[3], double t, double Tk)
{
    double L = C_LIGHT * (t - Tk);
    double dx = r[0] - wk[0];
    double dy = r[1] - wk[1];
    double dz = r[2] - wk[2];
    double LL = L * L;
    double dd = (dx * dx + dy * dy) + dz * dz;
    lc_sign_t s;
#ifdef MUT_TIE_NEWER
    s.positive = LL >= dd;
#else
    s.positive = LL > dd;
#endif
#ifdef MUT_NO_NEAR_TIE
    s.near = LL == dd;
#else
    s.near = fabs(LL - dd) <= NEAR_TIE * (LL + dd);
#endif
    return s;
}

static void load_sample(const double *a, int64_t N, int32_t s, int64_t j, double out[3])
{
    out[0] = a[((int64_t)s * 3 + 0) * N + j];
    out[1] = a[((int64_t)s * 3 + 1) * N + j];
    out[2] = a[((int64_t)s * 3 + 2) * N + j];
}

/* Reconstruction inside the bracket: 0 = the local linear one of Sec. 2.2
 * (Eq. linear, the method), 1 = the earlier midpoint values (Eq. mid),
 * kept as an accuracy ablation.  Set before a call, read-only during it. */
static int g_recon = 0;

void oracle_set_reconstruction(int mode) { g_recon = mode == 1 ? 1 : 0; }

/* Retarded quantities of one (target, source) pair.                         */
typedef struct {
    int32_t slot;     /* left end of the bracket (logical slot, 0 = oldest) */
    int before;       /* 1: retarded time older than the stored history     */
    double dt_root;   /* delta t = t_r - t_1 (Eq. dt)                       */
    double tr;        /* t_r = t_1 + delta t                                */
    double wr[3];     /* w(t_r) (Eq. linear / linear2)                      */
    double vr[3];     /* v(t_r)                                             */
    double ar[3];     /* a(t_r)                                             */
    double eta[3];    /* r - w(t_r), formed as (r - w_1) - v_1 dt           */
    int near_tie;     /* 1: a sign decision of the scan was a near tie      */
    int32_t alt_slot; /* near tie: the bracket the other decision gives
                         (logical slot, -1 before the history)             */
} retarded_t;

/* Sec. 2.2 retarded-time determination for target position r at time t
 * against source j's history.
 *
 * Bracket.  The paper's search (start from [t_0, t]; near-field shortcut
 * |r - w(t - dt)| < c dt; then bisection comparing c*delta with
 * |r - w(t_m)|, ties sent to the older half) stops at the unique stored
 * step k* whose sample lies inside the past light cone while the next
 * one does not.  Because every stored segment moves slower than light,
 * f_k decreases strictly with k, so that step is simply
 *      k* = max { k : f_k > 0 }.
 * The oracle evaluates this definition directly with a scan from the
 * newest sample backwards.  If no stored sample has f_k > 0 the retarded
 * time precedes the history (t_r < t_0) and the oldest sample is used
 * with the extrapolation of Eq. (linear2).
 *
 * Near ties (see lightcone_sign).  When a decision of the scan falls in
 * the near-tie band the pair is flagged and alt_slot names the bracket of
 * the other decision: the flagged sample itself if it was decided outside
 * the cone, the next older sample (or the before-history branch) if it was
 * decided inside.
 *
 * Root.  With t_1, w_1, v_1 the bracket's left sample the linear
 * reconstruction w(t_r) ~ w_1 + v_1 delta t turns the retardation
 * condition into C2 dt^2 + C1 dt + C0 = 0 with
 *      C2 = c^2 - v_1^2,
 *      C1 = 2 [ (r - w_1).v_1 - c^2 (t - t_1) ],
 *      C0 = c^2 (t - t_1)^2 - |r - w_1|^2,
 * and the physical root is (-C1 - sqrt(C1^2 - 4 C2 C0)) / (2 C2).  The
 * oracle evaluates the same root in Vieta's form 2 C0 / (-C1 + sqrt(.)),
 * which avoids the cancellation of the printed form, and checks that the
 * printed form agrees.
 *
 * Reconstruction (Eq. linear): t_r = t_1 + dt, w = w_1 + v_1 dt,
 * v = v_1 (1 - df) + v_2 df, a = (v_2 - v_1)/(t_2 - t_1), df = dt/(t_2-t_1).
 * Out of history (Eq. linear2): w = w_1 + v_1 dt, v = v_1, a = 0.            */
static int solve_retarded(int64_t N, int32_t ns, const double *T, const double *w,
                          const double *v, int64_t j, const double r[3], double t,
                          retarded_t *out)
{
    int32_t ks = -1;
    int near = 0;
    int32_t alt = -1;
    for (int32_t s = ns - 2; s >= 0; --s) {
        double wk[3];
        load_sample(w, N, s, j, wk);
        lc_sign_t g = lightcone_sign(r, wk, t, T[s]);
        if (g.near && !near) {
            near = 1;
            alt = g.positive ? s - 1 : s;
        }
        if (g.positive) {
            ks = s;
            break;
        }
    }
#ifdef MUT_KSTAR_OLDER
    if (ks > 0)
        ks -= 1;
#endif
    int before = (ks < 0);
    int32_t s1 = before ? 0 : ks;

    double w1[3], v1[3];
    load_sample(w, N, s1, j, w1);
    load_sample(v, N, s1, j, v1);
    double d[3] = {r[0] - w1[0], r[1] - w1[1], r[2] - w1[2]};
    double tau1 = t - T[s1];
    double c2 = C_LIGHT * C_LIGHT;

    double C2 = c2 - dot3(v1, v1);
    double C1 = 2.0 * (dot3(d, v1) - c2 * tau1);
    double C0 = c2 * tau1 * tau1 - dot3(d, d);
    double disc = C1 * C1 - 4.0 * C2 * C0;
    if (!(disc >= 0.0) || !(C2 > 0.0))
        return OR_ENUMERIC;
    double sq = sqrt(disc);
#ifdef MUT_ROOT_PLUS
    double dtr = (-C1 + sq) / (2.0 * C2);
#else
    double dtr = 2.0 * C0 / (-C1 + sq);
    /* The printed form of Eq. (dt) must agree with Vieta's form.  Its own
     * rounding error is of order eps * |C1| / C2, i.e. a few eps times the
     * look-back time t - t_1, so the check is scaled by that time.        */
    double literal = (-C1 - sq) / (2.0 * C2);
    double scale = fabs(tau1) + fabs(dtr);
    if (fabs(literal - dtr) > 1e-10 * scale)
        return OR_ECHECK;
#endif

    out->slot = s1;
    out->before = before;
    out->near_tie = near;
    out->alt_slot = alt;
    out->dt_root = dtr;
    out->tr = T[s1] + dtr;
    /* eta = r - w(t_r) with w(t_r) = w_1 + v_1 dt.  It is formed as
     * (r - w_1) - v_1 dt: r - w_1 is exact for nearby points, whereas the
     * absolute w(t_r) would be rounded to the spacing of doubles at its
     * coordinates (3.7 nm at three Earth radii), a relative error of ~1e-6
     * of a millimetre separation.                                         */
    for (int c = 0; c < 3; ++c) {
        out->wr[c] = w1[c] + v1[c] * dtr;
#ifdef MUT_ETA_ABSOLUTE
        out->eta[c] = r[c] - out->wr[c];
#else
        out->eta[c] = d[c] - v1[c] * dtr;
#endif
    }
    if (before) {
        for (int c = 0; c < 3; ++c) {
            out->vr[c] = v1[c];
#ifdef MUT_ACCEL_BEFORE_RING
            double v2[3];
            load_sample(v, N, s1 + 1, j, v2);
            out->ar[c] = (v2[c] - v1[c]) / (T[s1 + 1] - T[s1]);
#else
            out->ar[c] = 0.0;
#endif
        }
    } else if (g_recon == 1) {
        /* Eq. (mid): t_r, w, v at the bracket's midpoint, a from the
         * velocity difference; eta = r - (w_1 + w_2)/2 formed relative to
         * w_1 as above.                                                    */
        double w2[3], v2[3];
        load_sample(w, N, s1 + 1, j, w2);
        load_sample(v, N, s1 + 1, j, v2);
        double h = T[s1 + 1] - T[s1];
        out->dt_root = 0.5 * h;
        out->tr = 0.5 * (T[s1] + T[s1 + 1]);
        for (int c = 0; c < 3; ++c) {
            out->wr[c] = 0.5 * (w1[c] + w2[c]);
            out->eta[c] = d[c] - 0.5 * (w2[c] - w1[c]);
            out->vr[c] = 0.5 * (v1[c] + v2[c]);
            out->ar[c] = (v2[c] - v1[c]) / h;
        }
    } else {
        double v2[3];
        load_sample(v, N, s1 + 1, j, v2);
        double h = T[s1 + 1] - T[s1];
        double df = dtr / h;
        for (int c = 0; c < 3; ++c) {
#ifdef MUT_NO_VINTERP
            out->vr[c] = v1[c];
#else
            out->vr[c] = v1[c] * (1.0 - df) + v2[c] * df;
#endif
            out->ar[c] = (v2[c] - v1[c]) / h;
        }
    }
    return OR_OK;
}

/* Sec. 2.1, Eqs. (LW_E), (LW_B): field of one source at the target r,
 * given its retarded position, velocity and acceleration:
 *   eta = r - w(t_r),  v' = c eta_hat - v,
 *   E = q |eta| [ (c^2 - v^2) v' + eta x (v' x a) ] / (4 pi eps0 (eta.v')^3),
 *   B = eta_hat x E / c.                                                    */
static int lw_field(const double r[3], const retarded_t *rt, double q, double E[3], double B[3])
{
    const double *eta = rt->eta;
    (void)r;
    double en = sqrt(dot3(eta, eta));
    if (!(en > 0.0))
        return OR_ENUMERIC;
    double eh[3] = {eta[0] / en, eta[1] / en, eta[2] / en};
    double vp[3];
    for (int c = 0; c < 3; ++c) {
#ifdef MUT_VPRIME_NOHAT
        vp[c] = C_LIGHT * eta[c] - rt->vr[c];
#else
        vp[c] = C_LIGHT * eh[c] - rt->vr[c];
#endif
    }
    double ev = dot3(eta, vp);
    double vv = dot3(rt->vr, rt->vr);
    double vpxa[3], rad[3];
    cross3(vp, rt->ar, vpxa);
    cross3(eta, vpxa, rad);
    double pref = coulomb_k() * q * en / (ev * ev * ev);
    for (int c = 0; c < 3; ++c) {
#ifdef MUT_DROP_ACCEL
        E[c] = pref * ((C_LIGHT * C_LIGHT - vv) * vp[c]);
#else
        E[c] = pref * ((C_LIGHT * C_LIGHT - vv) * vp[c] + rad[c]);
#endif
    }
    double exE[3];
#ifdef MUT_B_SIGN
    cross3(E, eh, exE);
#else
    cross3(eh, E, exE);
#endif
    for (int c = 0; c < 3; ++c)
        B[c] = exE[c] / C_LIGHT;
    return OR_OK;
}

/* A bracket as slots back from the newest (1..ns-1), -1 before the history. */
static int32_t back_offset(int32_t ns, int32_t slot) { return slot < 0 ? -1 : (ns - 1) - slot; }

/* Per-pair inspection: retarded quantities for every (target, source).
 * Arrays [m][N] (scalars) or [m][N][3] (vectors); kstar as documented
 * above, kalt the same except on near ties, where it holds the bracket of
 * the other decision.  Pairs with j == self_index[a] are skipped (0).    */
int oracle_retarded(int64_t N, int32_t ns, const double *T, const double *w, const double *v,
                    double t, int64_t m, const double *x, const int64_t *self_index,
                    int32_t *kstar, int32_t *kalt, double *dt_root, double *tr, double *wr,
                    double *vr, double *ar)
{
    if (N < 1 || ns < 2 || m < 0)
        return OR_EINVAL;
    for (int64_t a = 0; a < m; ++a) {
        double r[3] = {x[a], x[m + a], x[2 * m + a]};
        for (int64_t j = 0; j < N; ++j) {
            int64_t p = a * N + j;
            if (self_index && self_index[a] == j) {
                if (kstar) kstar[p] = 0;
                if (kalt) kalt[p] = 0;
                continue;
            }
            retarded_t rt;
            int st = solve_retarded(N, ns, T, w, v, j, r, t, &rt);
            if (st != OR_OK)
                return st;
            if (kstar) kstar[p] = back_offset(ns, rt.before ? -1 : rt.slot);
            if (kalt) kalt[p] = back_offset(ns, rt.near_tie ? rt.alt_slot : (rt.before ? -1 : rt.slot));
            if (dt_root) dt_root[p] = rt.dt_root;
            if (tr) tr[p] = rt.tr;
            for (int c = 0; c < 3; ++c) {
                if (wr) wr[p * 3 + c] = rt.wr[c];
                if (vr) vr[p * 3 + c] = rt.vr[c];
                if (ar) ar[p * 3 + c] = rt.ar[c];
            }
        }
    }
    return OR_OK;
}

int oracle_fields_abs(int64_t N, int32_t ns, const double *T, const double *w, const double *v,
                      double q, double t, int64_t m, const double *x, const int64_t *self_index,
                      double *E, double *B, int32_t *kstar, int32_t *kalt, double *SE, double *SB,
                      int nthreads, int64_t *bad);

/* Sec. 2.1 superposition: E_i = sum_{j != i} E_ij and the same for B,
 * each sum Neumaier-compensated over j in index order.  q is the charge
 * of every source (all macro-particles carry the same charge and weight).
 * On a numerical failure the first failing (target, source) is reported
 * in bad[0], bad[1] (lowest target index wins).                          */
int oracle_fields(int64_t N, int32_t ns, const double *T, const double *w, const double *v,
                  double q, double t, int64_t m, const double *x, const int64_t *self_index,
                  double *E, double *B, int32_t *kstar, int nthreads, int64_t *bad)
{
    return oracle_fields_abs(N, ns, T, w, v, q, t, m, x, self_index, E, B, kstar, NULL, NULL, NULL,
                             nthreads, bad);
}

/* As oracle_fields, and also S_E[a] = sum_j |E_aj|, S_B[a] = sum_j |B_aj|
 * (either may be NULL): the scale against which a sum's rounding error
 * is judged; kalt (or NULL) as in oracle_retarded.                      */
int oracle_fields_abs(int64_t N, int32_t ns, const double *T, const double *w, const double *v,
                      double q, double t, int64_t m, const double *x, const int64_t *self_index,
                      double *E, double *B, int32_t *kstar, int32_t *kalt, double *SE, double *SB,
                      int nthreads, int64_t *bad)
{
    if (N < 1 || ns < 2 || m < 0 || !T || !w || !v || !x || !E || !B)
        return OR_EINVAL;
    if (t != T[ns - 1])
        return OR_EINVAL;
    int status = OR_OK;
    int64_t bad_i = -1, bad_j = -1;
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
    for (int64_t a = 0; a < m; ++a) {
        double r[3] = {x[a], x[m + a], x[2 * m + a]};
        double sE[3] = {0, 0, 0}, cE[3] = {0, 0, 0};
        double sB[3] = {0, 0, 0}, cB[3] = {0, 0, 0};
        double aE = 0.0, aB = 0.0;
        int st = OR_OK;
        int64_t jfail = -1;
#ifdef MUT_SUM_SKIP_LAST
        for (int64_t j = 0; j < N - 1; ++j) {
#else
        for (int64_t j = 0; j < N; ++j) {
#endif
#ifndef MUT_SELF_INDEX_IGNORED
            if (self_index && self_index[a] == j) {
                if (kstar) kstar[a * N + j] = 0;
                if (kalt) kalt[a * N + j] = 0;
                continue;
            }
#endif
            /* A target on a source's present position has eta = 0 at
             * t_r = t: the field is undefined (Sec. 2.1 divides by eta). */
            double wn[3];
            load_sample(w, N, ns - 1, j, wn);
            if (r[0] == wn[0] && r[1] == wn[1] && r[2] == wn[2]) {
                st = OR_ENUMERIC;
                jfail = j;
                break;
            }
            retarded_t rt;
            st = solve_retarded(N, ns, T, w, v, j, r, t, &rt);
            double Eij[3], Bij[3];
            if (st == OR_OK)
                st = lw_field(r, &rt, q, Eij, Bij);
            if (st != OR_OK) {
                jfail = j;
                break;
            }
            if (kstar)
                kstar[a * N + j] = back_offset(ns, rt.before ? -1 : rt.slot);
            if (kalt)
                kalt[a * N + j] = back_offset(ns, rt.near_tie ? rt.alt_slot : (rt.before ? -1 : rt.slot));
            for (int c = 0; c < 3; ++c) {
                neumaier_add(&sE[c], &cE[c], Eij[c]);
                neumaier_add(&sB[c], &cB[c], Bij[c]);
            }
            aE += sqrt(dot3(Eij, Eij));
            aB += sqrt(dot3(Bij, Bij));
        }
        if (SE) SE[a] = aE;
        if (SB) SB[a] = aB;
        for (int c = 0; c < 3; ++c) {
            E[c * m + a] = sE[c] + cE[c];
            B[c * m + a] = sB[c] + cB[c];
        }
        if (st != OR_OK) {
#pragma omp critical(oracle_fail)
            {
                if (bad_i < 0 || a < bad_i) {
                    bad_i = a;
                    bad_j = jfail;
                    status = st;
                }
            }
        }
    }
    if (bad) {
        bad[0] = bad_i;
        bad[1] = bad_j;
    }
    return status;
}

/* Sec. 2.6: centred dipole B = (mu0/4pi) (3 (M.rhat) rhat - M) / r^3 with
 * M = M0 e_z.  M0 is fixed by the equatorial surface field b0 at radius
 * re: |B(re, equator)| = (mu0/4pi) M0 / re^3 = b0.                        */
void oracle_dipole(double b0, double re, int64_t m, const double *x, double *B)
{
    double M0 = 4.0 * M_PI * b0 * re * re * re / MU0;
    double Mv[3] = {0.0, 0.0, M0};
    for (int64_t a = 0; a < m; ++a) {
        double r[3] = {x[a], x[m + a], x[2 * m + a]};
        double rn = sqrt(dot3(r, r));
        double rh[3] = {r[0] / rn, r[1] / rn, r[2] / rn};
        double mr = dot3(Mv, rh);
        double f = MU0 / (4.0 * M_PI) / (rn * rn * rn);
        for (int c = 0; c < 3; ++c) {
#ifdef MUT_DIPOLE_SIGN
            B[c * m + a] = f * (-3.0 * mr * rh[c] - Mv[c]);
#else
            B[c * m + a] = f * (3.0 * mr * rh[c] - Mv[c]);
#endif
        }
    }
}

/* Sec. 2.3: one Higuera-Cary update of the proper velocity u (in place)
 * for particles of charge q and mass mass in fields E, B over dt:
 *   u-  = u + (q dt/2m) E
 *   g-  = sqrt(1 + u-^2/c^2),  tau = (q dt/2m) B,  u* = u-.tau / c,
 *   sig = g-^2 - tau^2,  g+ = sqrt((sig + sqrt(sig^2 + 4(tau^2 + u*^2)))/2)
 *   t = tau/g+,  s = 1/(1 + t^2),
 *   u+  = s [ u- + (u-.t) t + u- x t ]
 *   u^{n+1} = u+ + (q dt/2m) E + u+ x t.
 * The last cross product takes u+, not u-; the paper flags the latter as
 * a typo in its source.                                                   */
static void hc_one(double q, double mass, double dt, double u[3], const double E[3],
                   const double B[3])
{
    double eps = q * dt / (2.0 * mass);
    double c = C_LIGHT;
    double um[3], tau[3];
    for (int k = 0; k < 3; ++k) {
        um[k] = u[k] + eps * E[k];
        tau[k] = eps * B[k];
    }
    double gm = sqrt(1.0 + dot3(um, um) / (c * c));
    double ustar = dot3(um, tau) / c;
    double tau2 = dot3(tau, tau);
    double sig = gm * gm - tau2;
    double gp = sqrt((sig + sqrt(sig * sig + 4.0 * (tau2 + ustar * ustar))) / 2.0);
    double tv[3] = {tau[0] / gp, tau[1] / gp, tau[2] / gp};
    double s = 1.0 / (1.0 + dot3(tv, tv));
    double umt = dot3(um, tv);
    double umxt[3];
    cross3(um, tv, umxt);
    double up[3];
    for (int k = 0; k < 3; ++k)
        up[k] = s * (um[k] + umt * tv[k] + umxt[k]);
    double upxt[3];
#ifdef MUT_HC_TYPO
    cross3(um, tv, upxt);
#else
    cross3(up, tv, upxt);
#endif
    for (int k = 0; k < 3; ++k)
        u[k] = up[k] + eps * E[k] + upxt[k];
}

void oracle_hc(double q, double mass, double dt, int64_t m, double *u, const double *E,
               const double *B)
{
    for (int64_t a = 0; a < m; ++a) {
        double ua[3] = {u[a], u[m + a], u[2 * m + a]};
        double Ea[3] = {E[a], E[m + a], E[2 * m + a]};
        double Ba[3] = {B[a], B[m + a], B[2 * m + a]};
        hc_one(q, mass, dt, ua, Ea, Ba);
        u[a] = ua[0];
        u[m + a] = ua[1];
        u[2 * m + a] = ua[2];
    }
}

static void velocity_of(const double u[3], double vel[3])
{
    double g = sqrt(1.0 + dot3(u, u) / (C_LIGHT * C_LIGHT));
    for (int c = 0; c < 3; ++c)
        vel[c] = u[c] / g;
}

/* Straight-line prior history (Sec. 2.2 needs a stored past; before the
 * first step the bunch is taken to have coasted with its initial
 * velocity).  Slots k = -(D-1) .. 0 at T_k = t0 + k dt hold
 * w_k = y0 + v0 (k dt) and v_k = v0 = u0 / gamma0.                        */
int oracle_init_straight(int64_t N, int32_t D, double dt, double t0, const double *r,
                         const double *u, double *T, double *w, double *v)
{
    if (N < 1 || D < 2 || !(dt > 0.0))
        return OR_EINVAL;
    for (int32_t s = 0; s < D; ++s) {
        int64_t k = (int64_t)s - (D - 1);
        double kdt = (double)k * dt;
        T[s] = t0 + kdt;
        for (int64_t i = 0; i < N; ++i) {
            double ui[3] = {u[i], u[N + i], u[2 * N + i]}, vi[3];
#ifdef MUT_INIT_NO_GAMMA
            vi[0] = ui[0], vi[1] = ui[1], vi[2] = ui[2];
#else
            velocity_of(ui, vi);
#endif
            for (int c = 0; c < 3; ++c) {
#ifdef MUT_INIT_FORWARD
                w[((int64_t)s * 3 + c) * N + i] = r[c * N + i] - vi[c] * kdt;
#else
                w[((int64_t)s * 3 + c) * N + i] = r[c * N + i] + vi[c] * kdt;
#endif
                v[((int64_t)s * 3 + c) * N + i] = vi[c];
            }
        }
    }
    return OR_OK;
}

/* One or more fixed-dt EM-PP steps (Secs. 2.1-2.3).
 *
 * State: the history (T, w, v) with the newest slot at the present time
 * T_n = t0 + n dt, the proper velocities u^n (before the kick at T_n) and
 * the step index *n.  The newest slot holds w_n = y^n and a provisional
 * v_n = v^n.  A stored v_k is the velocity that carries the particle from
 * T_k to T_{k+1}, so w_{k+1} = w_k + v_k dt holds for every slot.
 *
 * Each step:
 *   1. self-fields E_i, B_i at (y_i^n, T_n) from every other source;
 *   2. B_i += B_geo(y_i^n) when ext_field == 1;
 *   3. Higuera-Cary: u^{n+1};  v^{n+1} = u^{n+1}/gamma^{n+1};
 *   4. the newest slot's velocity becomes v^{n+1};
 *   5. y^{n+1} = y^n + v^{n+1} dt; the oldest slot is dropped and a new
 *      newest slot (T_{n+1}, y^{n+1}, v^{n+1}) is appended.
 * Fields of the last step are returned in E_last, B_last (self part only).
 * The history shift is a plain memmove: slow and obviously right.        */
int oracle_step(int64_t N, int32_t D, double q, double mass, double dt, double t0,
                int64_t *n, int32_t ext_field, double b0, double re, double *T, double *w,
                double *v, double *u, double *E_last, double *B_last, int64_t nsteps,
                int nthreads, int64_t *bad)
{
    if (N < 2 || D < 2 || !(dt > 0.0) || nsteps < 0)
        return OR_EINVAL;
    double *y = (double *)malloc(sizeof(double) * 3 * N);
    double *E = (double *)malloc(sizeof(double) * 3 * N);
    double *B = (double *)malloc(sizeof(double) * 3 * N);
    double *Bg = (double *)malloc(sizeof(double) * 3 * N);
    int64_t *self = (int64_t *)malloc(sizeof(int64_t) * N);
    if (!y || !E || !B || !Bg || !self) {
        free(y); free(E); free(B); free(Bg); free(self);
        return OR_EINVAL;
    }
    for (int64_t i = 0; i < N; ++i)
        self[i] = i;
    int st = OR_OK;
    for (int64_t step = 0; step < nsteps; ++step) {
        double t = T[D - 1];
        memcpy(y, w + (int64_t)(D - 1) * 3 * N, sizeof(double) * 3 * N);
        st = oracle_fields(N, D, T, w, v, q, t, N, y, self, E, B, NULL, nthreads, bad);
        if (st != OR_OK)
            break;
        if (E_last) memcpy(E_last, E, sizeof(double) * 3 * N);
        if (B_last) memcpy(B_last, B, sizeof(double) * 3 * N);
        if (ext_field == 1) {
            oracle_dipole(b0, re, N, y, Bg);
            for (int64_t p = 0; p < 3 * N; ++p)
                B[p] += Bg[p];
        }
        oracle_hc(q, mass, dt, N, u, E, B);
        /* finalise the newest slot's velocity, then drift */
        double *vnew = (double *)malloc(sizeof(double) * 3 * N);
        for (int64_t i = 0; i < N; ++i) {
            double ui[3] = {u[i], u[N + i], u[2 * N + i]}, vi[3];
            velocity_of(ui, vi);
            for (int c = 0; c < 3; ++c)
                vnew[c * N + i] = vi[c];
        }
#ifndef MUT_NO_FINALISE
        memcpy(v + (int64_t)(D - 1) * 3 * N, vnew, sizeof(double) * 3 * N);
#endif
        memmove(T, T + 1, sizeof(double) * (D - 1));
        memmove(w, w + 3 * N, sizeof(double) * 3 * N * (D - 1));
        memmove(v, v + 3 * N, sizeof(double) * 3 * N * (D - 1));
        *n += 1;
        T[D - 1] = t0 + (double)(*n) * dt;
        for (int64_t p = 0; p < 3 * N; ++p) {
            w[(int64_t)(D - 1) * 3 * N + p] = y[p] + vnew[p] * dt;
            v[(int64_t)(D - 1) * 3 * N + p] = vnew[p];
        }
        free(vnew);
    }
    free(y); free(E); free(B); free(Bg); free(self);
    return st;
}

/* Sec. 2.4 adaptive step.  From the same per-pair retarded quantities as
 * the field sum, over the pairs i != j with |eta_ij| >= eta_allow:
 *   eta_min = min |eta_ij|,   v_max = max |v_i(t) - v_j(t_r,ij)|,
 * with v_i(t) the target's present velocity vt[3][m] and v_j(t_r) the
 * reconstructed retarded velocity.  out = {eta_min, v_max}; eta_min = +inf
 * and v_max = 0 when no pair qualifies.                                    */
int oracle_adaptive_scan(int64_t N, int32_t ns, const double *T, const double *w, const double *v,
                         double t, int64_t m, const double *x, const int64_t *self_index,
                         const double *vt, double eta_allow, double out[2])
{
    if (N < 1 || ns < 2 || m < 0 || t != T[ns - 1])
        return OR_EINVAL;
    double emin = INFINITY, vmax = 0.0;
    for (int64_t a = 0; a < m; ++a) {
        double r[3] = {x[a], x[m + a], x[2 * m + a]};
        double va[3] = {vt[a], vt[m + a], vt[2 * m + a]};
        for (int64_t j = 0; j < N; ++j) {
            if (self_index && self_index[a] == j)
                continue;
            retarded_t rt;
            int st = solve_retarded(N, ns, T, w, v, j, r, t, &rt);
            if (st != OR_OK)
                return st;
            double en = sqrt(dot3(rt.eta, rt.eta));
#ifdef MUT_ADAPT_ETA_PRESENT
            double wn[3];
            load_sample(w, N, ns - 1, j, wn);
            double dn[3] = {r[0] - wn[0], r[1] - wn[1], r[2] - wn[2]};
            en = sqrt(dot3(dn, dn));
#endif
#ifndef MUT_ADAPT_NO_ALLOW
            if (en < eta_allow)
                continue;
#endif
            double dv[3] = {va[0] - rt.vr[0], va[1] - rt.vr[1], va[2] - rt.vr[2]};
            double sp = sqrt(dot3(dv, dv));
            if (en < emin)
                emin = en;
            if (sp > vmax)
                vmax = sp;
        }
    }
    out[0] = emin;
    out[1] = vmax;
    return OR_OK;
}

/* dt = C_dt eta_min / v_max, then clamped to [dt_min, dt_max]; dt_max when
 * no pair qualified or nothing moves relative to anything.               */
double oracle_adaptive_dt(double eta_min, double v_max, double c_dt, double dt_min, double dt_max)
{
    if (!(v_max > 0.0) || !(eta_min < INFINITY))
        return dt_max;
    double dt = c_dt * eta_min / v_max;
    return fmin(dt_max, fmax(dt_min, dt));
}

/* EM-PP steps with the adaptive step of Sec. 2.4: as oracle_step, with the
 * step of every pass taken from oracle_adaptive_scan at the present state
 * (targets: the particles, present velocities: the newest slot's) and the
 * new slot at T_{n+1} = T_n + dt.  dts[k] receives the k-th step.          */
int oracle_step_adaptive(int64_t N, int32_t D, double q, double mass, double c_dt, double dt_min,
                         double dt_max, double eta_allow, int32_t ext_field, double b0, double re,
                         double *T, double *w, double *v, double *u, double *dts, int64_t nsteps,
                         int nthreads, int64_t *bad)
{
    if (N < 2 || D < 2 || nsteps < 0 || !(dt_min > 0.0) || !(dt_max >= dt_min))
        return OR_EINVAL;
    double *y = (double *)malloc(sizeof(double) * 3 * N);
    double *E = (double *)malloc(sizeof(double) * 3 * N);
    double *B = (double *)malloc(sizeof(double) * 3 * N);
    double *Bg = (double *)malloc(sizeof(double) * 3 * N);
    double *vt = (double *)malloc(sizeof(double) * 3 * N);
    double *vnew = (double *)malloc(sizeof(double) * 3 * N);
    int64_t *self = (int64_t *)malloc(sizeof(int64_t) * N);
    int st = OR_OK;
    if (!y || !E || !B || !Bg || !vt || !vnew || !self)
        st = OR_EINVAL;
    for (int64_t i = 0; st == OR_OK && i < N; ++i)
        self[i] = i;
    for (int64_t step = 0; st == OR_OK && step < nsteps; ++step) {
        double t = T[D - 1];
        memcpy(y, w + (int64_t)(D - 1) * 3 * N, sizeof(double) * 3 * N);
        memcpy(vt, v + (int64_t)(D - 1) * 3 * N, sizeof(double) * 3 * N);
        st = oracle_fields(N, D, T, w, v, q, t, N, y, self, E, B, NULL, nthreads, bad);
        if (st != OR_OK)
            break;
        double ev[2];
        st = oracle_adaptive_scan(N, D, T, w, v, t, N, y, self, vt, eta_allow, ev);
        if (st != OR_OK)
            break;
        double dt = oracle_adaptive_dt(ev[0], ev[1], c_dt, dt_min, dt_max);
        if (dts)
            dts[step] = dt;
        if (ext_field == 1) {
            oracle_dipole(b0, re, N, y, Bg);
            for (int64_t p = 0; p < 3 * N; ++p)
                B[p] += Bg[p];
        }
        oracle_hc(q, mass, dt, N, u, E, B);
        for (int64_t i = 0; i < N; ++i) {
            double ui[3] = {u[i], u[N + i], u[2 * N + i]}, vi[3];
            velocity_of(ui, vi);
            for (int c = 0; c < 3; ++c)
                vnew[c * N + i] = vi[c];
        }
        memcpy(v + (int64_t)(D - 1) * 3 * N, vnew, sizeof(double) * 3 * N);
        memmove(T, T + 1, sizeof(double) * (D - 1));
        memmove(w, w + 3 * N, sizeof(double) * 3 * N * (D - 1));
        memmove(v, v + 3 * N, sizeof(double) * 3 * N * (D - 1));
        T[D - 1] = t + dt;
        for (int64_t p = 0; p < 3 * N; ++p) {
            w[(int64_t)(D - 1) * 3 * N + p] = y[p] + vnew[p] * dt;
            v[(int64_t)(D - 1) * 3 * N + p] = vnew[p];
        }
    }
    free(y); free(E); free(B); free(Bg); free(vt); free(vnew); free(self);
    return st;
}

/* Stage II of Sec. 2.7: after the switch the self-field is dropped and the
 * particles move in the prescribed field alone, E = 0 and B = B_geo(y)
 * (Sec. 2.6; B = 0 without an external field), advanced by the same
 * Higuera-Cary update and drift y += v dt as in Stage I.  The paper lets the
 * step grow but gives no rule; the reading taken here is a fixed fraction
 * of the shortest gyro-period in the bunch, evaluated before every step,
 *   dt = min(dt_max, gyro_k * min_i gamma_i / |B(y_i)|),
 *   gyro_k = frac * 2 pi m / |q|   (the period is 2 pi gamma m / (|q| B)),
 * and dt = dt_max when no particle sees a field.  *t advances by each dt;
 * dt_last returns the last step's dt.                                      */
int oracle_transport(int64_t N, double q, double mass, int32_t ext_field, double b0, double re,
                     double dt_max, double frac, double *y, double *u, double *t, int64_t nsteps,
                     double *dt_last)
{
    if (N < 1 || !(dt_max > 0.0) || !(frac > 0.0) || nsteps < 0 || q == 0.0)
        return OR_EINVAL;
    double *Bg = (double *)calloc((size_t)(3 * N), sizeof(double));
    if (!Bg)
        return OR_EINVAL;
    const double gyro_k = frac * 2.0 * M_PI * mass / fabs(q);
    const double zero[3] = {0.0, 0.0, 0.0};
    for (int64_t step = 0; step < nsteps; ++step) {
        if (ext_field == 1)
            oracle_dipole(b0, re, N, y, Bg);
        double key_min = INFINITY;
        for (int64_t i = 0; i < N; ++i) {
            double ui[3] = {u[i], u[N + i], u[2 * N + i]};
            double Bi[3] = {Bg[i], Bg[N + i], Bg[2 * N + i]};
            double g = sqrt(1.0 + dot3(ui, ui) / (C_LIGHT * C_LIGHT));
            double bm = sqrt(dot3(Bi, Bi));
#ifdef MUT_TRANSPORT_DT_NO_GAMMA
            g = 1.0;
#endif
            double key = bm > 0.0 ? g / bm : INFINITY;
            if (key < key_min)
                key_min = key;
        }
        double dt = dt_max;
        double d = gyro_k * key_min;
        if (d < dt)
            dt = d;
        for (int64_t i = 0; i < N; ++i) {
            double ui[3] = {u[i], u[N + i], u[2 * N + i]};
            double Bi[3] = {Bg[i], Bg[N + i], Bg[2 * N + i]};
            double vi[3];
#ifdef MUT_TRANSPORT_OLD_V
            velocity_of(ui, vi);
            hc_one(q, mass, dt, ui, zero, Bi);
#else
            hc_one(q, mass, dt, ui, zero, Bi);
            velocity_of(ui, vi);
#endif
            for (int c = 0; c < 3; ++c) {
                u[c * N + i] = ui[c];
                y[c * N + i] += vi[c] * dt;
            }
        }
        *t += dt;
        if (dt_last)
            *dt_last = dt;
    }
    free(Bg);
    return OR_OK;
}

/* Diagnostics (Sec. 2.5 RMS sizes, Sec. 2.7 mean kinetic energy, and the
 * weighted centroid), all weights 1:
 *   out = { sigma_x, sigma_y, sigma_z, sigma_xy, xbar, ybar, zbar, Ebar }
 * with Ebar the mean kinetic energy (gamma - 1) m c^2 in joules.          */
void oracle_diag(int64_t N, const double *y, const double *u, double mass, double out[8])
{
    double mean[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) {
        for (int64_t i = 0; i < N; ++i)
            mean[c] += y[c * N + i];
        mean[c] /= (double)N;
    }
    double var[3] = {0, 0, 0};
    for (int c = 0; c < 3; ++c) {
        for (int64_t i = 0; i < N; ++i) {
            double d = y[c * N + i] - mean[c];
            var[c] += d * d;
        }
        var[c] /= (double)N;
    }
    double ek = 0.0;
    for (int64_t i = 0; i < N; ++i) {
        double ui[3] = {u[i], u[N + i], u[2 * N + i]};
        double g = sqrt(1.0 + dot3(ui, ui) / (C_LIGHT * C_LIGHT));
        ek += (g - 1.0) * mass * C_LIGHT * C_LIGHT;
    }
    out[0] = sqrt(var[0]);
    out[1] = sqrt(var[1]);
    out[2] = sqrt(var[2]);
    out[3] = 0.5 * (out[0] + out[1]);
    out[4] = mean[0];
    out[5] = mean[1];
    out[6] = mean[2];
    out[7] = ek / (double)N;
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
