/*
 * empp.h -- C ABI of libempp.so, the MI355X (gfx950) implementation of the
 * hot path of the electromagnetic particle-particle (EM-PP) method for
 * relativistic electron bunches (arXiv 2605.05543).
 *
 * What one step computes (fixed time step dt, present time T_n):
 *   1. For every target particle i and every other source j, the retarded
 *      time on j's stored trajectory history: bracket by the light-cone
 *      sign test, then the segment quadratic and linear reconstruction
 *      (Sec. 2.2, Eqs. dt, linear, linear2).
 *   2. The Lienard-Wiechert velocity and acceleration fields of that pair
 *      (Sec. 2.1, Eqs. LW_E, LW_B), summed over j != i with compensated
 *      accumulation (superposition, Sec. 2.1).
 *   3. A Higuera-Cary push of every particle in its self-field plus the
 *      centred-dipole geomagnetic field (Secs. 2.3 and 2.6), the drift, and
 *      the history update.
 *
 * Units are SI throughout.  Host arrays are component-major: a [3][N]
 * array holds x[0..N), then y[0..N), then z[0..N).  A history is given
 * oldest slot first: T[ns], w[ns][3][N] (positions), v[ns][3][N]
 * (velocities).  Slot k's velocity is the one that carries the particle
 * from T_k to T_{k+1}; the newest slot's velocity is provisional until the
 * next push finalises it.
 *
 * Ownership: every pointer argument is borrowed for the duration of the
 * call.  Host inputs are copied; host outputs are written before return.
 * Device pointers (the *_dev entry points and the optional workspace) stay
 * owned by the caller; the library never frees them.  Memory the library
 * allocates itself is released by empp_destroy.
 *
 * Streams: all device work of a context is issued on the stream given in
 * its configuration (NULL: the device's null stream).  empp_step and the
 * *_dev calls only enqueue work; calls that return host data synchronise
 * the stream first.  Errors detected by kernels (coincident particles, a
 * negative discriminant: the pair's field is then left out of the sum)
 * are latched on the device and reported, with the first failing
 * (target, source), by the next call that synchronises: empp_sync,
 * empp_get_state, empp_get_history, empp_get_fields, empp_get_diag,
 * empp_step_until_switch, empp_handoff, empp_transport and empp_fields_at
 * (which reports an error left by an earlier step before its own launch).
 *
 * Threading: a context is bound to one device and must not be used by two
 * threads at once.  Different contexts are independent.
 *
 * Errors: every call returns an empp_status and never aborts or throws.
 * empp_last_error() returns a thread-local description of the last
 * failure on the calling thread.
 */
#ifndef EMPP_H
#define EMPP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct empp_ctx empp_ctx;

typedef enum {
    EMPP_OK = 0,
    EMPP_EINVAL = 1,       /* invalid argument or configuration            */
    EMPP_ENOMEM = 2,       /* device or host allocation failed             */
    EMPP_EDEVICE = 3,      /* HIP runtime error (message has its text)     */
    EMPP_ESTATE = 4,       /* call not valid in the context's state        */
    EMPP_ENUMERIC = 5,     /* coincident particles or negative discriminant */
    EMPP_EUNSUPPORTED = 6  /* option not available in this library         */
} empp_status;

typedef enum {
    EMPP_FP64 = 0,  /* everything in double precision                      */
    EMPP_MIXED = 1  /* FP64 absolute positions and times and every
                       light-cone sign test (the bracket is the FP64
                       path's); FP32 root, reconstruction and LW terms
                       around FP64 quadratic coefficients, with two-sum
                       accumulation; an FP32 root that fails its residual
                       test is recomputed in FP64 (a rescue)             */
} empp_precision;

typedef enum {
    EMPP_GUESS_BISECT = 0,    /* the paper's search: oldest-sample test, then
                                 bisection of the whole history            */
    EMPP_GUESS_MLP = 1,       /* start from the surrogate network's delay
                                 (modes 1 and 3 need depth >= 5: the
                                 network reads the slot 4 steps back;
                                 EUNSUPPORTED otherwise)                    */
    EMPP_GUESS_BALLISTIC = 2, /* start from the closed-form delay of a source
                                 coasting with its newest velocity          */
    EMPP_GUESS_MLP_PAIR = 3,  /* surrogate evaluated for every pair (fields_at
                                 only: measures the network's own accuracy
                                 at one evaluation per pair)                */
    EMPP_GUESS_PREVIOUS = 4   /* start from the pair's bracket of the previous
                                 step (FP64 path, empp_step only; fields_at
                                 bisects).  The workspace then holds N*N
                                 uint16 brackets (8 GiB at N = 65536); the
                                 first step after a history is set bisects.
                                 Set at creation: empp_set_mode cannot
                                 switch a context without the cache to it. */
} empp_guess;

typedef struct {
    int64_t n;             /* particles, >= 2                                */
    int32_t depth;         /* history slots D, 2 <= D <= 4064 (the deepest
                              history whose LDS tile fits a CU)             */
    int32_t ext_field;     /* 0: none; 1: centred dipole, moment along +z    */
    double q;              /* charge of every macro-particle (C); a weight w
                              is q = -w e with m = w m_e (q/m unchanged)     */
    double m;              /* mass of every macro-particle (kg), > 0         */
    double dt;             /* fixed time step (s), > 0                       */
    double dipole_b0;      /* dipole equatorial field at radius dipole_re (T) */
    double dipole_re;      /* reference radius of dipole_b0 (m)              */
    int32_t precision;     /* empp_precision                                 */
    int32_t guess;         /* empp_guess                                     */
    int32_t device;        /* HIP device ordinal                             */
    int32_t source_splits; /* 0: automatic; else number of source chunks     */
    void *stream;          /* hipStream_t or NULL                            */
    void *workspace;       /* caller-owned device memory, or NULL            */
    uint64_t workspace_bytes;
    /* Adaptive step (Sec. 2.4; FP64 path, guess modes other than MLP):
     * each step is c_dt * eta_min / v_max clamped to [dt_min, dt_max], where
     * eta_min = min |eta_ij| and v_max = max |v_i(t) - v_j(t_r)| over the
     * pairs with |eta_ij| >= eta_allow, reduced in the same pair pass that
     * sums the fields; dt then only spaces the straight-line prior history.
     * adaptive = 0: fixed dt (the remaining fields are ignored).          */
    int32_t adaptive;
    double c_dt;           /* safety factor (the paper: 0.05)                */
    double dt_min, dt_max; /* clamp (the paper: 1e-15 s and 1e-12 s)         */
    double eta_allow;      /* pairs closer than this are left out (m, >= 0)  */
    /* Reconstruction inside the bracket: 0 = the local linear one of
     * Sec. 2.2 (Eq. linear, the method); 1 = the earlier midpoint values of
     * Eq. (mid), an accuracy ablation (FP64 path, bisection, fixed step).  */
    int32_t recon;
    /* Targets per surrogate evaluation in guess mode EMPP_GUESS_MLP:
     * 2^guess_group_log2 consecutive targets (in the spatial order when
     * stepping) share one network evaluation at their centroid; 6 to 16,
     * 0 means 6 (64 targets, one wavefront).                              */
    int32_t guess_group_log2;
} empp_config;

typedef struct {
    double sigma[3];       /* RMS sizes sigma_x, sigma_y, sigma_z (Sec. 2.5)  */
    double sigma_xy;       /* (sigma_x + sigma_y)/2                          */
    double centroid[3];    /* mean position (weights 1)                      */
    double mean_kinetic;   /* mean kinetic energy (gamma-1) m c^2, J (Sec. 2.7) */
    double t;              /* present time                                   */
    int64_t step;          /* steps taken since the history was set          */
    double dt_last;        /* the last step's dt (adaptive), else cfg.dt     */
} empp_diag;

typedef struct {
    uint64_t pairs;        /* (target, source) pairs evaluated               */
    uint64_t before;       /* pairs whose retarded time precedes the history */
    uint64_t probes;       /* light-cone sign tests performed                */
    uint64_t rescues;      /* FP32 roots recomputed in FP64 (mixed precision) */
    uint64_t fallbacks;    /* guided searches that fell back to bisection    */
} empp_counters;

/* Device memory a context needs for cfg (bytes), so that a caller can
 * supply it through cfg->workspace.  EINVAL on a bad configuration.     */
empp_status empp_workspace_size(const empp_config *cfg, uint64_t *bytes);

/* Create a context on cfg->device.  With cfg->workspace NULL the library
 * allocates its device memory itself; otherwise the caller's buffer must
 * hold at least empp_workspace_size bytes, 256-byte aligned.            */
empp_status empp_create(const empp_config *cfg, empp_ctx **out);

/* Release the context and everything the library allocated.  NULL-safe. */
void empp_destroy(empp_ctx *ctx);

const char *empp_last_error(void);

/* Set the bunch (Sec. 2.5): positions r[3][N] and proper velocities
 * u[3][N] (u = gamma v, m/s) at time t0 (host arrays).  The history is
 * built by empp_init_history_straight.  EINVAL on non-finite values.    */
empp_status empp_init_bunch(empp_ctx *ctx, const double *r, const double *u, double t0);

/* Straight-line prior history (the stored past the retarded-time search of
 * Sec. 2.2 needs before the first step): slots k = -(D-1)..0 at
 * T_k = t0 + k dt with w_k = r + v0 (k dt), v_k = v0 = u / gamma (the
 * particle coasted with its initial velocity).  The present time becomes
 * t0, step index 0.  ESTATE before empp_init_bunch.                     */
empp_status empp_init_history_straight(empp_ctx *ctx);

/* Install an explicit history of Sec. 2.2's stored trajectories (host
 * arrays, nslots == D, oldest first, T strictly increasing) and the
 * present proper velocities u[3][N].  The present time is T[nslots-1];
 * later steps advance it by dt.  EINVAL when a stored speed is >= c or a
 * value is not finite.                                                    */
empp_status empp_set_history(empp_ctx *ctx, int32_t nslots, const double *T, const double *w,
                             const double *v, const double *u);

/* Advance nsteps steps (asynchronous): each is the pair pass of Secs.
 * 2.1-2.2 (bracket, Eq. dt root, Eqs. linear/linear2 reconstruction, Eqs.
 * LW_E/LW_B fields summed over j != i), the Higuera-Cary kick of Sec. 2.3
 * in the self-field plus the dipole of Sec. 2.6, the drift and the history
 * update; the step is cfg.dt, or the rule of Sec. 2.4 when cfg.adaptive.
 * ESTATE before a history exists or after the handoff.                  */
empp_status empp_step(empp_ctx *ctx, int64_t nsteps);

/* Lienard-Wiechert self-fields (Secs. 2.1-2.2, the same pass as a step's)
 * at m external points x[3][m] (host) at the present time t (t must
 * equal it exactly: EINVAL otherwise).  self_index[m] (or NULL) names a
 * source to leave out per target (-1: none).  Outputs E[3][m], B[3][m]
 * (self-fields only, no external field) and, if kstar is not NULL,
 * kstar[m][N]: for each pair the number of slots back from the newest of
 * the bracket's older end (1..D-1), -1 when the retarded time precedes the
 * history, 0 for a skipped pair.  Synchronous.                           */
empp_status empp_fields_at(empp_ctx *ctx, double t, int64_t m, const double *x,
                           const int64_t *self_index, double *E, double *B, int32_t *kstar);

/* Same with device pointers (same layouts); asynchronous on the context's
 * stream.  kstar_dev may be NULL.                                       */
empp_status empp_fields_at_dev(empp_ctx *ctx, double t, int64_t m, const double *x_dev,
                               const int64_t *self_index_dev, double *E_dev, double *B_dev,
                               int32_t *kstar_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * fields as empp_fields_at_dev, with the same arguments and layouts,
 * asynchronous on the context's stream, but the call allocates nothing.
 * The per-chunk field partials of its pass go to a fixed 128 MiB device
 * array the library holds on every GPU it runs on until the process ends
 * (its address is looked up once per device by empp_create), so at most
 * floor(128 MiB / (96 B x source chunks)) targets fit one call (10922 with
 * the 128 chunks of N = 65536): EINVAL beyond that.  Guess modes
 * EMPP_GUESS_MLP and EMPP_GUESS_MLP_PAIR are EUNSUPPORTED here.  Results
 * are bit-identical to empp_fields_at_dev's (same chunks, same merge
 * order).  All calls on one GPU share the array, which keeps the last
 * call's partials: calls that overlap on one GPU (two streams, two
 * threads) race and must be serialised by the caller.                    */
empp_status empp_fields_at_dev_noalloc(empp_ctx *ctx, double t, int64_t m, const double *x_dev,
                                       const int64_t *self_index_dev, double *E_dev, double *B_dev,
                                       int32_t *kstar_dev);

/* Present positions r[3][N], proper velocities u[3][N], time and step
 * index (host; any output may be NULL).                                  */
empp_status empp_get_state(empp_ctx *ctx, double *r, double *u, double *t, int64_t *step);

/* Whole history, oldest first: T[D], w[D][3][N], v[D][3][N] (host).      */
empp_status empp_get_history(empp_ctx *ctx, double *T, double *w, double *v);

/* Self-fields E[3][N], B[3][N] that the last step's push used (host).    */
empp_status empp_get_fields(empp_ctx *ctx, double *E, double *B);

/* Diagnostics of the present state (host): RMS sizes (Sec. 2.5), centroid,
 * mean kinetic energy (Sec. 2.7), time, step and last step size.        */
empp_status empp_get_diag(empp_ctx *ctx, empp_diag *out);

/* Counters accumulated since the last reset (the counting kernels run
 * only while counting is enabled).                                       */
empp_status empp_set_counting(empp_ctx *ctx, int32_t enable);
empp_status empp_get_counters(empp_ctx *ctx, empp_counters *out);

typedef struct {
    double pair_ms;        /* summed duration of pair-kernel launches (ms)   */
    int64_t pair_launches;
    double push_ms;        /* summed duration of push-kernel launches (ms)   */
    int64_t push_launches;
    double guess_ms;       /* summed duration of surrogate-guess launches    */
    int64_t guess_launches;
} empp_timing;

/* Kernel timing with HIP events recorded on the context's stream around
 * every pair and push launch while enabled.  empp_get_timing synchronises,
 * returns the sums since the last call (or enable) and resets them.      */
empp_status empp_set_timing(empp_ctx *ctx, int32_t enable);
empp_status empp_get_timing(empp_ctx *ctx, empp_timing *out);

/* ---- surrogate network (retarded-delay guess) ----------------------------
 * A 10 -> 128 -> 128 -> 1 SiLU network with BF16 weights on the matrix
 * cores (FP32 accumulation) corrects the straight-line retarded delay of a
 * (target, source) pair: the model's delay is s_line exp(z), s_line the
 * look-back c (t - t_r) of a source coasting with its newest velocity, and
 * the network output z is trained on log(c (t - t_r) / s_line).  Its 10
 * features: (r - w_n)/sigma_ref (3), the source's newest velocity / c (3),
 * its displacement over the last 4 steps / (c (T_n - T_{n-4})) (3) and
 * log1p((t - T_n)/dt) (1).  With guess mode EMPP_GUESS_MLP it is evaluated
 * once per (group of 64 consecutive targets -- in the spatial order when
 * stepping --, source) at the group centroid, and exp(z) there scales each
 * target's own straight-line look-back.  The exact search then finishes
 * every bracket, so the network changes cost, never results.  Not part of
 * the paper's method.  Parameters: the flat vector W1[128][10], b1[128], W2[128][128],
 * b2[128], W3[128], b3 (18049 floats, FP32 masters).                     */
typedef struct {
    int64_t steps;         /* optimizer steps                                */
    int32_t batch;         /* rows per step, a multiple of 64                */
    float lr;              /* initial Adam learning rate                     */
    float lr_final;        /* cosine decay to this rate at the last step     */
} empp_train_cfg;

typedef struct {
    double loss_first;     /* mean squared error of z at the first step      */
    double loss_last;      /* at the last step                               */
    int64_t steps;
    double seconds;        /* wall time of the loop (device work included)   */
} empp_train_report;

/* Install parameters (host, nparams == 18049) and sigma_ref (m).  Resets
 * the optimizer state.                                                    */
empp_status empp_surrogate_set(empp_ctx *ctx, const float *params, int64_t nparams, double sigma_ref);
/* Read the FP32 master parameters back (host).                            */
empp_status empp_surrogate_get(empp_ctx *ctx, float *params, int64_t nparams);
/* Features X[count][10] and exact targets y[count] (host outputs) of pairs
 * of the present state: given pairs (tgt[], src[] particle indices, host)
 * or, with tgt == NULL, pairs drawn by splitmix64(seed + counter).         */
empp_status empp_surrogate_samples(empp_ctx *ctx, int64_t count, uint64_t seed, const int64_t *tgt,
                                   const int64_t *src, float *X, float *y);
/* Drawn pairs written to caller-owned device buffers (asynchronous).      */
empp_status empp_surrogate_samples_dev(empp_ctx *ctx, int64_t count, uint64_t seed, float *X_dev, float *y_dev);
/* z for feature rows X[count][10] (host in, host out).                    */
empp_status empp_surrogate_forward(empp_ctx *ctx, const float *X, int64_t count, float *z);
/* Mean squared error of z against y and its gradient[18049] (host).       */
empp_status empp_surrogate_loss_grad(empp_ctx *ctx, const float *X, const float *y, int64_t count, double *loss,
                                     float *grad);
/* Adam training on device rows (X_dev[count][10], y_dev[count]), cycling
 * through them in order, batch rows per step.  Each optimizer step (forward
 * and backward on the matrix cores, the fixed-order sum of the block
 * partials, Adam, the packed bf16 copy) runs inside one cooperative launch
 * that takes up to 256 steps; results do not depend on scheduling.
 * Synchronous.  EMPP_EDEVICE if a grid-wide barrier of that launch timed
 * out (the parameters are then not to be trusted).                      */
empp_status empp_surrogate_train(empp_ctx *ctx, const float *X_dev, const float *y_dev, int64_t count,
                                 const empp_train_cfg *cfg, empp_train_report *out);

/* Wait for the context's stream and report latched device errors.        */
empp_status empp_sync(empp_ctx *ctx);

/* Change precision / search mode of an existing context.                 */
empp_status empp_set_mode(empp_ctx *ctx, int32_t precision, int32_t guess);

/* ---- two-stage strategy (Sec. 2.7) -----------------------------------------
 * Stage I (empp_step) until the mean kinetic energy settles, then Stage II:
 * no self-field, the particles move in the prescribed field alone.       */

/* Stage I steps in windows of check_every steps until the growth rate of
 * the mean kinetic energy over a window, |dE/dt| (J/s, from empp_diag's
 * mean_kinetic), falls below eps_E, or max_steps are taken.  Outputs (any
 * may be NULL): steps taken, the time reached, and whether the criterion
 * was met.  Errors as empp_step; EINVAL on eps_E < 0 or check_every < 1. */
empp_status empp_step_until_switch(empp_ctx *ctx, double eps_E, int64_t check_every, int64_t max_steps,
                                   int64_t *steps_done, double *t_sw, int32_t *switched);

/* Hand the present state over to Stage II: positions, proper velocities
 * and time are kept, the history ring and self-fields are no longer used
 * (empp_step, empp_fields_at and empp_get_history then return ESTATE;
 * setting a history again returns to Stage I).  ESTATE before a history
 * exists or after a handoff.                                              */
empp_status empp_handoff(empp_ctx *ctx);

/* Stage-II transport: nsteps steps with E = 0 and B = B_geo (the centred
 * dipole, or 0 without an external field), Higuera-Cary and drift as in
 * Stage I.  The step is
 *   dt = min(dt_max, gyro_fraction * 2 pi m / |q| * min_i gamma_i / |B(y_i)|),
 * a fraction of the shortest gyro-period in the bunch, re-evaluated on the
 * device before every step (dt_max when nothing sees a field).  Blocks
 * until done and advances the context's time.  ESTATE before the handoff;
 * EINVAL on dt_max <= 0, gyro_fraction <= 0 or nsteps < 0.               */
empp_status empp_transport(empp_ctx *ctx, double dt_max, double gyro_fraction, int64_t nsteps);

/* Checkpoint: write the whole state (history ring in Stage I, or the
 * Stage-II positions; proper velocities, slot times, the spatial order,
 * step counters and clock) to a binary file at path, and read it back into
 * a context created with the same n, depth, q, m and dt (EINVAL
 * otherwise, or on an unreadable or truncated file or a spatial order that
 * is not a permutation of 0..n-1, after which the context holds no
 * state).  Layout: an 88-byte header (magic "EMPPCKP1", n, depth, head,
 * step counters, clock, stage, q, m, dt), then T[depth], u[3][n] and the
 * order int32[n], then the two rings (Stage I) or the positions, step
 * keys and clock (Stage II).  Caches (warm-start brackets, surrogate
 * guesses) and the last step's fields are not saved.                     */
empp_status empp_save(empp_ctx *ctx, const char *path);
empp_status empp_load(empp_ctx *ctx, const char *path);

#ifdef __cplusplus
}
#endif

#endif /* EMPP_H */
