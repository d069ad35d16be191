// api.cpp -- the C ABI of libempp.so (declared in include/empp.h): context
// and workspace management, argument validation, kernel launches on the
// context's stream, and host read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cerrno>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include <chrono>

#include "empp.h"
#include "empp_dev.h"
#include "mlp_dev.h"

namespace empp {
int pair_fp64_tile(int D);
hipError_t launch_pair_fp64(const PairParams &p, hipStream_t stream, bool kstar, bool count);
hipError_t launch_pair_mixed(const PairParams &p, hipStream_t stream, bool kstar, bool count);
hipError_t launch_lightcone_records(const double4 *ring_w, const double *T, int64_t N, int D, int head,
                                    double4 *rec, hipStream_t s);
hipError_t launch_merge_fields(const double *part, int nsplit, int64_t m, const int32_t *order, double *E,
                               double *B, hipStream_t s);
hipError_t launch_push(const PushParams &p, hipStream_t s);
hipError_t launch_init_straight(double4 *rw, double4 *rv, double *T, const double *r, const double *u, int64_t N,
                                int D, double t0, double dt, hipStream_t s);
hipError_t launch_history_to_ring(const double *w, const double *v, const double *T, double4 *rw, double4 *rv,
                                  int64_t N, int D, hipStream_t s);
hipError_t launch_ring_to_history(const double4 *rw, const double4 *rv, double *w, double *v, int64_t N, int D,
                                  int head, hipStream_t s);
hipError_t launch_newest_positions(const double4 *rw, double *r, int64_t N, int D, int head, hipStream_t s);
hipError_t launch_diag(const double4 *rw, const double *u, int64_t N, int D, int head, double *out, hipStream_t s);
hipError_t launch_handoff(const double4 *ring_w, int D, int head, double4 *pos, const double *u, int64_t N,
                          double dip_k, int ext_field, unsigned long long *key, double *t, double t_now,
                          hipStream_t s);
hipError_t launch_transport(const TransportParams &p, hipStream_t s);
hipError_t launch_mlp_forward(const MlpPacked *net, const float *X, int64_t n, float *z, hipStream_t s);
hipError_t mlp_train_max_blocks(int device, int *out);
hipError_t launch_mlp_sync_clear(unsigned long long *sync, unsigned int *fail, hipStream_t s);
hipError_t launch_mlp_train(const TrainRun *run, int nblocks, hipStream_t s);
hipError_t launch_mlp_pack(const float *master, MlpPacked *net, hipStream_t s);
hipError_t launch_mlp_sample(const SampleParams &p, const int64_t *tgt, const int64_t *src, int64_t count, float *X,
                             float *y, hipStream_t s);
hipError_t launch_mlp_group_guess(const MlpPacked *net, const GuessParams &p, float *G, hipStream_t s);
hipError_t launch_group_centroid(const double4 *ring_w, const int32_t *order, int64_t N, int D, int head,
                                 double3 *centroid, hipStream_t s);
hipError_t launch_group_centroid_x(const double *x, int64_t m, int group, double3 *centroid, hipStream_t s);
hipError_t launch_merge_centroids(const double3 *cent64, int64_t m, int ratio, double3 *out, hipStream_t s);
size_t noalloc_scratch_bytes();
hipError_t noalloc_scratch(int device, void **out);
}  // namespace empp

using namespace empp;

namespace empp {
extern const bool kHaveMixed;
}

namespace {

thread_local std::string g_last_error;

empp_status fail(empp_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(EMPP_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));              \
    } while (0)

constexpr uint64_t kAlign = 256;

uint64_t align_up(uint64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
    uint64_t ring_w, ring_v, rec, T, u, E, B, part, err, counters, diag, order, pos, skey, st, ad, kc, kc_bytes, total;
};

int tile_for_depth(int D) { return pair_fp64_tile(D); }

int bisection_steps(int D)
{
    int nit = 0;
    while ((1 << nit) < D - 1)
        ++nit;
    return nit;
}

// Spatial (Morton, 21 bits per axis) order of points x[3][N]: the pair
// kernels visit targets in this order so that the lanes of a wavefront are
// neighbours and probe nearby history slots.  Only the mapping of targets
// to threads changes; every target's sum is unaffected.
std::vector<int32_t> morton_order(const double *x, int64_t N)
{
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) {
        lo[c] = hi[c] = x[c * N];
        for (int64_t i = 1; i < N; ++i) {
            lo[c] = std::min(lo[c], x[c * N + i]);
            hi[c] = std::max(hi[c], x[c * N + i]);
        }
    }
    auto spread = [](uint64_t v) {
        v &= 0x1fffff;
        v = (v | v << 32) & 0x1f00000000ffffull;
        v = (v | v << 16) & 0x1f0000ff0000ffull;
        v = (v | v << 8) & 0x100f00f00f00f00full;
        v = (v | v << 4) & 0x10c30c30c30c30c3ull;
        v = (v | v << 2) & 0x1249249249249249ull;
        return v;
    };
    std::vector<std::pair<uint64_t, int32_t>> key(N);
    for (int64_t i = 0; i < N; ++i) {
        uint64_t code = 0;
        for (int c = 0; c < 3; ++c) {
            double span = hi[c] - lo[c];
            double f = span > 0 ? (x[c * N + i] - lo[c]) / span : 0.0;
            uint64_t q = (uint64_t)std::min(2097151.0, std::max(0.0, f * 2097151.0));
            code |= spread(q) << c;
        }
        key[i] = {code, (int32_t)i};
    }
    std::sort(key.begin(), key.end());
    std::vector<int32_t> order(N);
    for (int64_t i = 0; i < N; ++i)
        order[i] = key[i].second;
    return order;
}

int splits_for(const empp_config &c)
{
    if (c.source_splits > 0)
        return std::min(c.source_splits, kMaxSplits);
    // About 8192 blocks of the FP64 pair kernel (32 rounds of one block per
    // CU) evens out blocks that finish early and keeps each chunk's
    // histories near its XCD's L2 (measured optimum at N = 65536: 128
    // chunks); the warm-started search, with less work per tile, does best
    // with half as many.
    int64_t bx = (c.n + kBlockFp64 - 1) / kBlockFp64;
    int tile = tile_for_depth(c.depth);
    const int64_t target = c.guess == EMPP_GUESS_PREVIOUS ? 4096 : 8192;
    int64_t want = (target + bx - 1) / bx;
    int64_t maxs = std::max<int64_t>(1, c.n / (4 * tile));
    int64_t s = std::min(want, maxs);
    return (int)std::max<int64_t>(1, std::min<int64_t>(s, kMaxSplits));
}

Layout layout_for(const empp_config &c)
{
    Layout L{};
    uint64_t N = (uint64_t)c.n, D = (uint64_t)c.depth;
    uint64_t o = 0;
    auto take = [&](uint64_t bytes) {
        uint64_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.ring_w = take(N * D * sizeof(double4));
    L.ring_v = take(N * D * sizeof(double4));
    // light-cone records of the present pass (lightcone_records_kernel)
    L.rec = take(N * D * sizeof(double4));
    L.T = take(D * sizeof(double));
    L.u = take(3 * N * sizeof(double));
    L.E = take(3 * N * sizeof(double));
    L.B = take(3 * N * sizeof(double));
    L.part = take((uint64_t)splits_for(c) * 12 * N * sizeof(double));
    L.err = take(2 * sizeof(unsigned long long));
    L.counters = take(8 * sizeof(unsigned long long));
    L.diag = take(((N + kBlock - 1) / kBlock) * 7 * sizeof(double));
    L.order = take(N * sizeof(int32_t));
    // Stage II: compact positions, the step-minimum slots and the clock
    L.pos = take(N * sizeof(double4));
    L.skey = take(4 * sizeof(unsigned long long));
    L.st = take(sizeof(double));
    // adaptive step: two {eta_min, v_max^2} slots and the last dt
    L.ad = take(8 * sizeof(unsigned long long));
    // previous-step brackets (warm start): uint16 per (source, target)
    L.kc_bytes = c.guess == EMPP_GUESS_PREVIOUS ? N * N * sizeof(uint16_t) : 0;
    L.kc = L.kc_bytes ? take(L.kc_bytes) : 0;
    L.total = o;
    return L;
}

empp_status validate(const empp_config *c)
{
    if (!c)
        return fail(EMPP_EINVAL, "config is NULL");
    if (c->n < 2)
        return fail(EMPP_EINVAL, "n = %lld: need at least 2 particles", (long long)c->n);
    if (c->n > (int64_t)1 << 31)
        return fail(EMPP_EINVAL, "n = %lld exceeds 2^31", (long long)c->n);
    if (c->depth < 2 || c->depth > kMaxDepth)
        return fail(EMPP_EINVAL, "depth = %d: need 2 <= D <= %d", c->depth, kMaxDepth);
    if (!(c->dt > 0.0) || !std::isfinite(c->dt))
        return fail(EMPP_EINVAL, "dt must be positive and finite");
    if (!(c->m > 0.0) || !std::isfinite(c->m) || !std::isfinite(c->q))
        return fail(EMPP_EINVAL, "mass must be positive, charge finite");
    if (c->ext_field != 0 && c->ext_field != 1)
        return fail(EMPP_EINVAL, "ext_field must be 0 or 1");
    if (c->ext_field == 1 && (!std::isfinite(c->dipole_b0) || !(c->dipole_re > 0.0)))
        return fail(EMPP_EINVAL, "dipole parameters invalid");
    if (c->precision != EMPP_FP64 && c->precision != EMPP_MIXED)
        return fail(EMPP_EINVAL, "unknown precision %d", c->precision);
    if (c->precision == EMPP_MIXED && !kHaveMixed)
        return fail(EMPP_EUNSUPPORTED, "mixed precision is not built");
    if (c->guess < 0 || c->guess > 4)
        return fail(EMPP_EINVAL, "unknown guess mode %d", c->guess);
    if (c->guess == EMPP_GUESS_PREVIOUS && c->precision == EMPP_MIXED)
        return fail(EMPP_EUNSUPPORTED, "warm-start brackets are implemented for the FP64 path");
    if (c->recon != 0 && c->recon != 1)
        return fail(EMPP_EINVAL, "recon must be 0 (linear) or 1 (midpoint)");
    if (c->guess_group_log2 != 0 && (c->guess_group_log2 < 6 || c->guess_group_log2 > 16))
        return fail(EMPP_EINVAL, "guess_group_log2 must be 0 or 6..16");
    // the network's history-slope input reads the slot four steps back
    if ((c->guess == EMPP_GUESS_MLP || c->guess == EMPP_GUESS_MLP_PAIR) && c->depth < 5)
        return fail(EMPP_EUNSUPPORTED, "the surrogate guess needs at least 5 history slots");
    if (c->recon == 1 && (c->precision != EMPP_FP64 || c->guess != EMPP_GUESS_BISECT || c->adaptive))
        return fail(EMPP_EUNSUPPORTED, "the midpoint ablation runs on the FP64 path with bisection and a fixed step");
    if (c->adaptive) {
        if (c->precision != EMPP_FP64 || c->guess == EMPP_GUESS_MLP || c->guess == EMPP_GUESS_MLP_PAIR)
            return fail(EMPP_EUNSUPPORTED, "the adaptive step is implemented for the FP64 path without the surrogate");
        if (!(c->c_dt > 0.0) || !(c->dt_min > 0.0) || !(c->dt_max >= c->dt_min) || !std::isfinite(c->dt_max) ||
            !(c->eta_allow >= 0.0))
            return fail(EMPP_EINVAL, "adaptive step needs c_dt > 0, 0 < dt_min <= dt_max finite, eta_allow >= 0");
    }
    return EMPP_OK;
}

bool all_finite(const double *a, uint64_t n)
{
    for (uint64_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i]))
            return false;
    return true;
}

}  // namespace

struct empp_ctx {
    empp_config cfg{};
    Layout L{};
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    bool owns_ws = false;
    void *scratch = nullptr;  // this device's copy of the allocation-free entry point's scratch
    int nsplit = 1;
    int tile = 1;
    // state
    bool have_bunch = false;
    bool have_history = false;
    bool handed_off = false;
    int64_t tr_step = 0;    // Stage-II steps since the handoff
    bool counting = false;
    bool kc_valid = false;  // the bracket cache holds the previous step's brackets
    int head = 0;
    int64_t step = 0;
    double t_origin = 0.0;  // T of step 0
    double t_now = 0.0;
    std::vector<double> r0, u0;  // bunch before the history is built
    // kernel timing (HIP events on the context's stream)
    bool timing = false;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<std::pair<size_t, int>> ev_marks;  // (start index, kind 0 pair / 1 push / 2 guess)
    // surrogate network (device buffers allocated by empp_surrogate_set)
    struct {
        float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr, *part = nullptr;
        MlpPacked *net = nullptr;
        float *G = nullptr;
        double3 *cent = nullptr, *cent_big = nullptr;
        unsigned long long *sync = nullptr;  // training barrier arrivals
        unsigned int *sync_fail = nullptr;
        float *loss_first = nullptr;
        int part_blocks = 512;
        int train_blocks = 0;  // resident blocks of the training step
        int64_t adam_step = 0;
        double sigma_ref = 0.0;
        bool ready = false;
    } sg;

    template <typename Tp>
    Tp *at(uint64_t off) const { return reinterpret_cast<Tp *>(ws + off); }
    double4 *ring_w() const { return at<double4>(L.ring_w); }
    double4 *ring_v() const { return at<double4>(L.ring_v); }
    double4 *rec() const { return at<double4>(L.rec); }
    double *T() const { return at<double>(L.T); }
    double *u() const { return at<double>(L.u); }
    double *E() const { return at<double>(L.E); }
    double *B() const { return at<double>(L.B); }
    double *part() const { return at<double>(L.part); }
    unsigned long long *err() const { return at<unsigned long long>(L.err); }
    unsigned long long *counters() const { return at<unsigned long long>(L.counters); }
    double *diag() const { return at<double>(L.diag); }
    int32_t *order() const { return at<int32_t>(L.order); }
    uint16_t *kc() const { return L.kc_bytes ? at<uint16_t>(L.kc) : nullptr; }
    double4 *pos() const { return at<double4>(L.pos); }
    unsigned long long *skey() const { return at<unsigned long long>(L.skey); }
    double *stime() const { return at<double>(L.st); }
    unsigned long long *ad() const { return at<unsigned long long>(L.ad); }
    // present positions: the ring's newest slot (Stage I) or the compact
    // array viewed as a one-slot ring (Stage II)
    const double4 *present_pos() const { return handed_off ? pos() : ring_w(); }
    int present_depth() const { return handed_off ? 1 : cfg.depth; }
    int present_head() const { return handed_off ? 0 : head; }
};

namespace {

empp_status set_device(empp_ctx *ctx)
{
    HIP_TRY(hipSetDevice(ctx->cfg.device));
    return EMPP_OK;
}

empp_status reset_err(empp_ctx *ctx)
{
    unsigned long long init[2] = {~0ull, 0ull};
    HIP_TRY(hipMemcpyAsync(ctx->err(), init, sizeof init, hipMemcpyHostToDevice, ctx->stream));
    return EMPP_OK;
}

empp_status check_err(empp_ctx *ctx)
{
    unsigned long long h[2];
    HIP_TRY(hipMemcpyAsync(h, ctx->err(), sizeof h, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    if (h[1] != 0) {
        long long a = (long long)(h[0] >> 32), j = (long long)(h[0] & 0xffffffffull);
        empp_status st = reset_err(ctx);
        if (st != EMPP_OK)
            return st;
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        return fail(EMPP_ENUMERIC, "%s at target %lld, source %lld",
                    (h[1] & kErrDiscriminant) ? "negative discriminant" : "coincident particles (eta = 0)", a, j);
    }
    return EMPP_OK;
}

// Both {eta_min, v_max^2} slots empty, last dt = cfg.dt.
empp_status reset_adaptive(empp_ctx *ctx)
{
    double dt = ctx->cfg.dt;
    unsigned long long init[8] = {kPosInfBits, 0ull, kPosInfBits, 0ull, 0ull, 0ull, 0ull, 0ull};
    memcpy(&init[4], &dt, sizeof dt);
    HIP_TRY(hipMemcpyAsync(ctx->ad(), init, sizeof init, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return EMPP_OK;
}

PairParams pair_params(empp_ctx *ctx)
{
    PairParams p{};
    p.ring_w = ctx->ring_w();
    p.ring_v = ctx->ring_v();
    p.rec = ctx->rec();
    p.T = ctx->T();
    p.n_src = ctx->cfg.n;
    p.D = ctx->cfg.depth;
    p.head = ctx->head;
    p.t = ctx->t_now;
    const double c = kC_LIGHT;
    const double eps0 = 1.0 / (kMU0 * c * c);
    p.kq = ctx->cfg.q / (4.0 * M_PI * eps0);
    p.nsplit = ctx->nsplit;
    p.src_per_split = (ctx->cfg.n + ctx->nsplit - 1) / ctx->nsplit;
    p.tile = ctx->tile;
    p.nit = bisection_steps(ctx->cfg.depth);
    p.order = nullptr;
    p.part = ctx->part();
    p.err = ctx->err();
    p.counters = ctx->counters();
    p.guess = ctx->cfg.guess;
    // the bracket cache serves the step's launch only
    if (p.guess == EMPP_GUESS_PREVIOUS)
        p.guess = EMPP_GUESS_BISECT;
    p.kc = nullptr;
    p.kc_cold = 1;
    p.ad = nullptr;
    p.eta_allow = ctx->cfg.eta_allow;
    p.recon = ctx->cfg.recon;
    p.dt = ctx->cfg.dt;
    return p;
}

// Record an event on the context's stream (timing mode only).  Events are
// created once and reused; a failure just disables timing.
hipError_t timing_event(empp_ctx *ctx)
{
    if (ctx->ev_used == ctx->ev_pool.size()) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess)
            return err;
        ctx->ev_pool.push_back(e);
    }
    return hipEventRecord(ctx->ev_pool[ctx->ev_used++], ctx->stream);
}

template <typename F>
hipError_t timed(empp_ctx *ctx, int kind, F &&launch)
{
    if (!ctx->timing)
        return launch();
    size_t at = ctx->ev_used;
    hipError_t e = timing_event(ctx);
    if (e != hipSuccess)
        return e;
    e = launch();
    if (e != hipSuccess)
        return e;
    e = timing_event(ctx);
    if (e == hipSuccess)
        ctx->ev_marks.push_back({at, kind});
    return e;
}

// Surrogate guesses for a launch of m targets (external x or the
// particles in spatial order): group centroids, then one network evaluation
// per (group, source).
hipError_t launch_guesses(empp_ctx *ctx, PairParams &p, float *G_pair = nullptr, double3 *cent_pair = nullptr)
{
    if (ctx->cfg.guess == EMPP_GUESS_MLP_PAIR) {
        // one evaluation per (target, source): the "group" is the target
        return timed(ctx, 2, [&]() {
            hipError_t e = launch_group_centroid_x(p.x, p.m, 1, cent_pair, ctx->stream);
            if (e != hipSuccess)
                return e;
            GuessParams gp{};
            gp.ring_w = ctx->ring_w();
            gp.ring_v = ctx->ring_v();
            gp.T = ctx->T();
            gp.centroid = cent_pair;
            gp.N = ctx->cfg.n;
            gp.ngroups = p.m;
            gp.D = ctx->cfg.depth;
            gp.head = ctx->head;
            gp.inv_sigma = 1.0 / ctx->sg.sigma_ref;
            gp.ratio = 0;
            p.G = G_pair;
            p.g_groups = p.m;
            p.g_shift = 0;
            return launch_mlp_group_guess(ctx->sg.net, gp, G_pair, ctx->stream);
        });
    }
    if (ctx->cfg.guess != EMPP_GUESS_MLP)
        return hipSuccess;
    return timed(ctx, 2, [&]() {
        const int shift = ctx->cfg.guess_group_log2 ? ctx->cfg.guess_group_log2 : 6;
        double3 *cent = shift > 6 ? ctx->sg.cent_big : ctx->sg.cent;
        hipError_t e = hipSuccess;
        if (p.x) {
            e = launch_group_centroid_x(p.x, p.m, 1 << shift, cent, ctx->stream);
        } else {
            // centroids of 64 targets, merged into the larger groups
            e = launch_group_centroid(ctx->ring_w(), p.order, p.m, ctx->cfg.depth, ctx->head, ctx->sg.cent,
                                      ctx->stream);
            if (e == hipSuccess && shift > 6)
                e = launch_merge_centroids(ctx->sg.cent, p.m, 1 << (shift - 6), cent, ctx->stream);
        }
        if (e != hipSuccess)
            return e;
        GuessParams gp{};
        gp.ring_w = ctx->ring_w();
        gp.ring_v = ctx->ring_v();
        gp.T = ctx->T();
        gp.centroid = cent;
        gp.N = ctx->cfg.n;
        gp.ngroups = (p.m + (1 << shift) - 1) >> shift;
        gp.D = ctx->cfg.depth;
        gp.head = ctx->head;
        gp.inv_sigma = 1.0 / ctx->sg.sigma_ref;
        gp.ratio = 1;
        p.G = ctx->sg.G;
        p.g_groups = gp.ngroups;
        p.g_shift = shift;
        return launch_mlp_group_guess(ctx->sg.net, gp, ctx->sg.G, ctx->stream);
    });
}

// Whether the pair launch for p runs a search mode that stages the
// precomputed light-cone records (the midpoint ablation and a cold warm
// start run the bisection).
bool pair_needs_records(const PairParams &p)
{
    if (p.recon == 1)
        return false;
    if (p.guess == EMPP_GUESS_PREVIOUS)
        return !p.kc_cold;
    return pass_uses_records(p.guess);
}

hipError_t launch_pair(empp_ctx *ctx, PairParams &p, bool kstar, float *G_pair = nullptr,
                       double3 *cent_pair = nullptr)
{
    hipError_t eg = launch_guesses(ctx, p, G_pair, cent_pair);
    if (eg != hipSuccess)
        return eg;
    // the pass's light-cone records (guided searches), then the pair kernel
    // (timed together)
    return timed(ctx, 0, [&]() {
        if (pair_needs_records(p)) {
            hipError_t e = launch_lightcone_records(p.ring_w, p.T, p.n_src, p.D, p.head,
                                                    const_cast<double4 *>(p.rec), ctx->stream);
            if (e != hipSuccess)
                return e;
        }
        if (ctx->cfg.precision == EMPP_MIXED)
            return launch_pair_mixed(p, ctx->stream, kstar, ctx->counting);
        return launch_pair_fp64(p, ctx->stream, kstar, ctx->counting);
    });
}

}  // namespace

extern "C" {

const char *empp_last_error(void) { return g_last_error.c_str(); }

empp_status empp_workspace_size(const empp_config *cfg, uint64_t *bytes)
{
    empp_status st = validate(cfg);
    if (st != EMPP_OK)
        return st;
    if (!bytes)
        return fail(EMPP_EINVAL, "bytes is NULL");
    *bytes = layout_for(*cfg).total;
    return EMPP_OK;
}

empp_status empp_create(const empp_config *cfg, empp_ctx **out)
{
    if (!out)
        return fail(EMPP_EINVAL, "out is NULL");
    *out = nullptr;
    empp_status st = validate(cfg);
    if (st != EMPP_OK)
        return st;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (cfg->device < 0 || cfg->device >= ndev)
        return fail(EMPP_EINVAL, "device %d not present (%d devices)", cfg->device, ndev);
    empp_ctx *ctx = new (std::nothrow) empp_ctx();
    if (!ctx)
        return fail(EMPP_ENOMEM, "host allocation failed");
    ctx->cfg = *cfg;
    ctx->L = layout_for(*cfg);
    ctx->nsplit = splits_for(*cfg);
    ctx->tile = tile_for_depth(cfg->depth);
    ctx->stream = (hipStream_t)cfg->stream;
    if ((st = set_device(ctx)) != EMPP_OK) {
        delete ctx;
        return st;
    }
    // set-up of the allocation-free entry point: the address of this
    // device's scratch array (looked up once per device)
    {
        hipError_t e = noalloc_scratch(cfg->device, &ctx->scratch);
        if (e != hipSuccess) {
            delete ctx;
            return fail(EMPP_EDEVICE, "scratch address on device %d: %s", cfg->device, hipGetErrorString(e));
        }
    }
    if (cfg->workspace) {
        if (cfg->workspace_bytes < ctx->L.total || ((uintptr_t)cfg->workspace % kAlign) != 0) {
            delete ctx;
            return fail(EMPP_EINVAL, "workspace too small (%llu < %llu) or not 256-byte aligned",
                        (unsigned long long)cfg->workspace_bytes, (unsigned long long)ctx->L.total);
        }
        ctx->ws = (char *)cfg->workspace;
    } else {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, ctx->L.total);
        if (e != hipSuccess) {
            delete ctx;
            return fail(EMPP_ENOMEM, "hipMalloc(%llu) failed: %s", (unsigned long long)ctx->L.total,
                        hipGetErrorString(e));
        }
        ctx->ws = (char *)p;
        ctx->owns_ws = true;
    }
    if ((st = reset_err(ctx)) != EMPP_OK || (st = empp_set_counting(ctx, 0)) != EMPP_OK) {
        empp_destroy(ctx);
        return st;
    }
    hipError_t e = hipStreamSynchronize(ctx->stream);
    if (e != hipSuccess) {
        empp_destroy(ctx);
        return fail(EMPP_EDEVICE, "stream synchronise failed: %s", hipGetErrorString(e));
    }
    *out = ctx;
    return EMPP_OK;
}

void empp_destroy(empp_ctx *ctx)
{
    if (!ctx)
        return;
    (void)hipSetDevice(ctx->cfg.device);
    (void)hipStreamSynchronize(ctx->stream);
    for (hipEvent_t e : ctx->ev_pool)
        (void)hipEventDestroy(e);
    for (void *p : {(void *)ctx->sg.master, (void *)ctx->sg.m, (void *)ctx->sg.v, (void *)ctx->sg.grad,
                    (void *)ctx->sg.part, (void *)ctx->sg.net, (void *)ctx->sg.G, (void *)ctx->sg.cent,
                    (void *)ctx->sg.cent_big, (void *)ctx->sg.sync, (void *)ctx->sg.sync_fail,
                    (void *)ctx->sg.loss_first})
        if (p)
            (void)hipFree(p);
    if (ctx->owns_ws && ctx->ws)
        (void)hipFree(ctx->ws);
    delete ctx;
}

empp_status empp_init_bunch(empp_ctx *ctx, const double *r, const double *u, double t0)
{
    if (!ctx || !r || !u)
        return fail(EMPP_EINVAL, "NULL argument");
    const uint64_t n3 = 3 * (uint64_t)ctx->cfg.n;
    if (!all_finite(r, n3) || !all_finite(u, n3) || !std::isfinite(t0))
        return fail(EMPP_EINVAL, "non-finite bunch value");
    ctx->r0.assign(r, r + n3);
    ctx->u0.assign(u, u + n3);
    ctx->t_origin = t0;
    ctx->have_bunch = true;
    ctx->have_history = false;
    ctx->handed_off = false;
    return EMPP_OK;
}

empp_status empp_init_history_straight(empp_ctx *ctx)
{
    if (!ctx)
        return fail(EMPP_EINVAL, "NULL context");
    if (!ctx->have_bunch)
        return fail(EMPP_ESTATE, "init_history_straight before init_bunch");
    empp_status st = set_device(ctx);
    if (st != EMPP_OK)
        return st;
    const int64_t N = ctx->cfg.n;
    const int D = ctx->cfg.depth;
    // r is staged in the partials buffer (>= 12 N doubles), u goes to u.
    double *r_dev = ctx->part();
    HIP_TRY(hipMemcpyAsync(r_dev, ctx->r0.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipMemcpyAsync(ctx->u(), ctx->u0.data(), 3 * N * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(launch_init_straight(ctx->ring_w(), ctx->ring_v(), ctx->T(), r_dev, ctx->u(), N, D, ctx->t_origin,
                                 ctx->cfg.dt, ctx->stream));
    std::vector<int32_t> ord = morton_order(ctx->r0.data(), N);
    HIP_TRY(hipMemcpyAsync(ctx->order(), ord.data(), N * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipMemsetAsync(ctx->E(), 0, 3 * N * sizeof(double), ctx->stream));
    HIP_TRY(hipMemsetAsync(ctx->B(), 0, 3 * N * sizeof(double), ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->head = D - 1;
    ctx->step = 0;
    ctx->t_now = ctx->t_origin;  // t0 + 0 * dt
    ctx->have_history = true;
    ctx->handed_off = false;
    ctx->kc_valid = false;
    if ((st = reset_adaptive(ctx)) != EMPP_OK)
        return st;
    ctx->handed_off = false;
    return EMPP_OK;
}

empp_status empp_set_history(empp_ctx *ctx, int32_t nslots, const double *T, const double *w, const double *v,
                             const double *u)
{
    if (!ctx || !T || !w || !v || !u)
        return fail(EMPP_EINVAL, "NULL argument");
    const int64_t N = ctx->cfg.n;
    const int D = ctx->cfg.depth;
    if (nslots != D)
        return fail(EMPP_EINVAL, "nslots %d != depth %d", nslots, D);
    const uint64_t tot = 3 * (uint64_t)N * D;
    if (!all_finite(T, D) || !all_finite(w, tot) || !all_finite(v, tot) || !all_finite(u, 3 * (uint64_t)N))
        return fail(EMPP_EINVAL, "non-finite history value");
    for (int s = 1; s < D; ++s)
        if (!(T[s] > T[s - 1]))
            return fail(EMPP_EINVAL, "slot times not strictly increasing at slot %d", s);
    const double c2 = kC_LIGHT * kC_LIGHT;
    for (int s = 0; s < D; ++s)
        for (int64_t i = 0; i < N; ++i) {
            const double *vs = v + (uint64_t)s * 3 * N;
            double v2 = vs[i] * vs[i] + vs[N + i] * vs[N + i] + vs[2 * N + i] * vs[2 * N + i];
            if (!(v2 < c2))
                return fail(EMPP_EINVAL, "stored speed >= c (slot %d, particle %lld)", s, (long long)i);
        }
    empp_status st = set_device(ctx);
    if (st != EMPP_OK)
        return st;
    double *tmp = nullptr;
    hipError_t e = hipMalloc((void **)&tmp, 2 * tot * sizeof(double));
    if (e != hipSuccess)
        return fail(EMPP_ENOMEM, "hipMalloc for history upload failed: %s", hipGetErrorString(e));
    auto body = [&]() -> empp_status {
        HIP_TRY(hipMemcpyAsync(tmp, w, tot * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(hipMemcpyAsync(tmp + tot, v, tot * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(hipMemcpyAsync(ctx->T(), T, D * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(launch_history_to_ring(tmp, tmp + tot, ctx->T(), ctx->ring_w(), ctx->ring_v(), N, D, ctx->stream));
        HIP_TRY(hipMemcpyAsync(ctx->u(), u, 3 * N * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        std::vector<int32_t> ord = morton_order(w + (uint64_t)(D - 1) * 3 * N, N);
        HIP_TRY(hipMemcpyAsync(ctx->order(), ord.data(), N * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        HIP_TRY(hipMemsetAsync(ctx->E(), 0, 3 * N * sizeof(double), ctx->stream));
        HIP_TRY(hipMemsetAsync(ctx->B(), 0, 3 * N * sizeof(double), ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        return EMPP_OK;
    };
    st = body();
    (void)hipFree(tmp);
    if (st != EMPP_OK)
        return st;
    ctx->head = D - 1;
    ctx->step = 0;
    ctx->t_origin = T[D - 1];
    ctx->t_now = T[D - 1];
    ctx->have_bunch = true;
    ctx->have_history = true;
    ctx->handed_off = false;
    ctx->kc_valid = false;
    if ((st = reset_adaptive(ctx)) != EMPP_OK)
        return st;
    ctx->handed_off = false;
    return EMPP_OK;
}

empp_status empp_step(empp_ctx *ctx, int64_t nsteps)
{
    if (!ctx)
        return fail(EMPP_EINVAL, "NULL context");
    if (nsteps < 0)
        return fail(EMPP_EINVAL, "nsteps < 0");
    if (!ctx->have_history)
        return fail(EMPP_ESTATE, "step before the history is initialised");
    if (ctx->handed_off)
        return fail(EMPP_ESTATE, "step after handoff (use transport)");
    if (ctx->cfg.guess == EMPP_GUESS_MLP && !ctx->sg.ready)
        return fail(EMPP_ESTATE, "guess mode MLP without a surrogate network (empp_surrogate_set)");
    if (ctx->cfg.guess == EMPP_GUESS_MLP_PAIR)
        return fail(EMPP_EUNSUPPORTED, "per-pair surrogate guesses are available in fields_at only");
    empp_status st = set_device(ctx);
    if (st != EMPP_OK)
        return st;
    const int64_t N = ctx->cfg.n;
    const double c = kC_LIGHT;
    (void)c;
    for (int64_t s = 0; s < nsteps; ++s) {
        PairParams p = pair_params(ctx);
        p.x = nullptr;
        p.self_index = nullptr;
        p.order = ctx->order();
        p.m = N;
        p.kstar = nullptr;
        if (ctx->cfg.guess == EMPP_GUESS_PREVIOUS) {
            p.guess = EMPP_GUESS_PREVIOUS;
            p.kc = ctx->kc();
            p.kc_cold = ctx->kc_valid ? 0 : 1;
        }
        unsigned long long *slot = ctx->ad() + 2 * (ctx->step & 1);
        unsigned long long *other = ctx->ad() + 2 * ((ctx->step + 1) & 1);
        if (ctx->cfg.adaptive)
            p.ad = slot;
        HIP_TRY(launch_pair(ctx, p, false));
        ctx->kc_valid = p.kc != nullptr;
        PushParams q{};
        q.ring_w = ctx->ring_w();
        q.ring_v = ctx->ring_v();
        q.T = ctx->T();
        q.u = ctx->u();
        q.E = ctx->E();
        q.B = ctx->B();
        q.part = ctx->part();
        q.order = p.order;
        q.nsplit = ctx->nsplit;
        q.N = N;
        q.D = ctx->cfg.depth;
        q.head = ctx->head;
        q.dt = ctx->cfg.dt;
        q.t_now = ctx->t_now;
        q.t_next = ctx->t_origin + (double)(ctx->step + 1) * ctx->cfg.dt;
        q.eps = ctx->cfg.q * ctx->cfg.dt / (2.0 * ctx->cfg.m);
        q.ext_field = ctx->cfg.ext_field;
        q.dip_k = ctx->cfg.dipole_b0 * ctx->cfg.dipole_re * ctx->cfg.dipole_re * ctx->cfg.dipole_re;
        q.self_field = 1;
        if (ctx->cfg.adaptive) {
            q.ad = slot;
            q.ad_next = other;
            q.dt_out = reinterpret_cast<double *>(ctx->ad() + 4);
            q.c_dt = ctx->cfg.c_dt;
            q.dt_min = ctx->cfg.dt_min;
            q.dt_max = ctx->cfg.dt_max;
            q.q = ctx->cfg.q;
            q.m = ctx->cfg.m;
        }
        HIP_TRY(timed(ctx, 1, [&]() { return launch_push(q, ctx->stream); }));
        ctx->head = ctx->head + 1 == ctx->cfg.depth ? 0 : ctx->head + 1;
        ctx->step += 1;
        ctx->t_now = q.t_next;
    }
    if (ctx->cfg.adaptive && nsteps > 0) {
        // the steps were chosen on the device: bring the clock back
        double tn = 0.0;
        HIP_TRY(hipMemcpyAsync(&tn, ctx->T() + ctx->head, sizeof tn, hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        ctx->t_now = tn;
    }
    return EMPP_OK;
}

// Device scratch of one call, freed on every return path once the stream
// has drained.
struct StreamScratch {
    hipStream_t stream;
    void *ptr = nullptr;
    explicit StreamScratch(hipStream_t s) : stream(s) {}
    StreamScratch(const StreamScratch &) = delete;
    StreamScratch &operator=(const StreamScratch &) = delete;
    ~StreamScratch()
    {
        if (ptr) {
            (void)hipStreamSynchronize(stream);
            (void)hipFree(ptr);
        }
    }
};

static empp_status fields_dev_impl(empp_ctx *ctx, int64_t m, const double *x_dev, const int64_t *self_dev,
                                   double *E_dev, double *B_dev, int32_t *kstar_dev)
{
    const int64_t N = ctx->cfg.n;
    // targets go through in chunks of at most N (the partials buffer's size)
    for (int64_t a0 = 0; a0 < m; a0 += N) {
        const int64_t mc = std::min<int64_t>(N, m - a0);
        StreamScratch xbuf(ctx->stream), obuf(ctx->stream), gbuf(ctx->stream);
        // x for the chunk must be a [3][mc] array: chunking needs a copy
        const double *xc = x_dev;
        if (m > N) {
            HIP_TRY(hipMalloc(&xbuf.ptr, 3 * mc * sizeof(double)));
            double *tmpx = (double *)xbuf.ptr;
            for (int k = 0; k < 3; ++k)
                HIP_TRY(hipMemcpyAsync(tmpx + k * mc, x_dev + k * m + a0, mc * sizeof(double),
                                       hipMemcpyDeviceToDevice, ctx->stream));
            xc = tmpx;
        }
        PairParams p = pair_params(ctx);
        p.x = xc;
        p.self_index = self_dev ? self_dev + a0 : nullptr;
        p.m = mc;
        p.kstar = kstar_dev ? kstar_dev + a0 * N : nullptr;
        float *G_pair = nullptr;
        double3 *cent_pair = nullptr;
        if (ctx->cfg.guess == EMPP_GUESS_MLP_PAIR) {
            HIP_TRY(hipMalloc(&gbuf.ptr, (size_t)mc * N * sizeof(float) + (size_t)mc * sizeof(double3) + 256));
            G_pair = (float *)gbuf.ptr;
            cent_pair = (double3 *)((char *)G_pair + align_up((size_t)mc * N * sizeof(float)));
        }
        HIP_TRY(launch_pair(ctx, p, kstar_dev != nullptr, G_pair, cent_pair));
        double *Ec = E_dev, *Bc = B_dev;
        if (m > N) {
            HIP_TRY(hipMalloc(&obuf.ptr, 6 * mc * sizeof(double)));
            Ec = (double *)obuf.ptr;
            Bc = Ec + 3 * mc;
        }
        HIP_TRY(launch_merge_fields(ctx->part(), ctx->nsplit, mc, nullptr, Ec, Bc, ctx->stream));
        if (m > N) {
            for (int k = 0; k < 3; ++k) {
                HIP_TRY(hipMemcpyAsync(E_dev + k * m + a0, Ec + k * mc, mc * sizeof(double), hipMemcpyDeviceToDevice,
                                       ctx->stream));
                HIP_TRY(hipMemcpyAsync(B_dev + k * m + a0, Bc + k * mc, mc * sizeof(double), hipMemcpyDeviceToDevice,
                                       ctx->stream));
            }
        }
    }
    return EMPP_OK;
}

static empp_status fields_precheck(empp_ctx *ctx, double t, int64_t m)
{
    if (!ctx)
        return fail(EMPP_EINVAL, "NULL context");
    if (!ctx->have_history)
        return fail(EMPP_ESTATE, "fields_at before the history is initialised");
    if (ctx->handed_off)
        return fail(EMPP_ESTATE, "fields_at after handoff");
    if (m < 0)
        return fail(EMPP_EINVAL, "m < 0");
    if (t != ctx->t_now)
        return fail(EMPP_EINVAL, "t = %.17g is not the present time %.17g", t, ctx->t_now);
    if ((ctx->cfg.guess == EMPP_GUESS_MLP || ctx->cfg.guess == EMPP_GUESS_MLP_PAIR) && !ctx->sg.ready)
        return fail(EMPP_ESTATE, "guess mode MLP without a surrogate network (empp_surrogate_set)");
    return set_device(ctx);
}

empp_status empp_fields_at_dev(empp_ctx *ctx, double t, int64_t m, const double *x_dev, const int64_t *self_dev,
                               double *E_dev, double *B_dev, int32_t *kstar_dev)
{
    empp_status st = fields_precheck(ctx, t, m);
    if (st != EMPP_OK)
        return st;
    if (m == 0)
        return EMPP_OK;
    if (!x_dev || !E_dev || !B_dev)
        return fail(EMPP_EINVAL, "NULL argument");
    return fields_dev_impl(ctx, m, x_dev, self_dev, E_dev, B_dev, kstar_dev);
}

empp_status empp_fields_at_dev_noalloc(empp_ctx *ctx, double t, int64_t m, const double *x_dev,
                                       const int64_t *self_dev, double *E_dev, double *B_dev, int32_t *kstar_dev)
{
    empp_status st = fields_precheck(ctx, t, m);
    if (st != EMPP_OK)
        return st;
    if (m == 0)
        return EMPP_OK;
    if (!x_dev || !E_dev || !B_dev)
        return fail(EMPP_EINVAL, "NULL argument");
    if (ctx->cfg.guess == EMPP_GUESS_MLP || ctx->cfg.guess == EMPP_GUESS_MLP_PAIR)
        return fail(EMPP_EUNSUPPORTED, "the allocation-free fields call runs the bisection or the straight-line guess");
    // the chunk partials, nsplit x 12 doubles per target, live in the scratch array
    const uint64_t per_target = (uint64_t)ctx->nsplit * 12 * sizeof(double);
    const int64_t m_max = (int64_t)(noalloc_scratch_bytes() / per_target);
    if (m > m_max)
        return fail(EMPP_EINVAL, "m = %lld targets exceed the allocation-free call's maximum of %lld (%llu-byte scratch, "
                    "%d source chunks)", (long long)m, (long long)m_max, (unsigned long long)noalloc_scratch_bytes(),
                    ctx->nsplit);
    if (!ctx->scratch)
        return fail(EMPP_ESTATE, "no scratch address for device %d", ctx->cfg.device);
    PairParams p = pair_params(ctx);
    p.x = x_dev;
    p.self_index = self_dev;
    p.m = m;
    p.kstar = kstar_dev;
    p.part = reinterpret_cast<double *>(ctx->scratch);
    // launched directly: no timing events, no guess buffers; the records
    // live in the context's workspace
    hipError_t e = hipSuccess;
    if (pair_needs_records(p))
        e = launch_lightcone_records(p.ring_w, p.T, p.n_src, p.D, p.head, const_cast<double4 *>(p.rec), ctx->stream);
    if (e == hipSuccess)
        e = ctx->cfg.precision == EMPP_MIXED ? launch_pair_mixed(p, ctx->stream, kstar_dev != nullptr, ctx->counting)
                                             : launch_pair_fp64(p, ctx->stream, kstar_dev != nullptr, ctx->counting);
    if (e != hipSuccess)
        return fail(EMPP_EDEVICE, "pair pass: %s", hipGetErrorString(e));
    HIP_TRY(launch_merge_fields(p.part, ctx->nsplit, m, nullptr, E_dev, B_dev, ctx->stream));
    return EMPP_OK;
}

empp_status empp_fields_at(empp_ctx *ctx, double t, int64_t m, const double *x, const int64_t *self_index,
                           double *E, double *B, int32_t *kstar)
{
    empp_status st = fields_precheck(ctx, t, m);
    if (st != EMPP_OK)
        return st;
    if (m == 0)
        return EMPP_OK;
    if (!x || !E || !B)
        return fail(EMPP_EINVAL, "NULL argument");
    if (!all_finite(x, 3 * (uint64_t)m))
        return fail(EMPP_EINVAL, "non-finite target position");
    // an error latched by earlier asynchronous work (a step) is reported
    // here as that work's, before this call's own pairs can latch one
    if ((st = check_err(ctx)) != EMPP_OK)
        return fail(st, "an earlier step: %s", std::string(g_last_error).c_str());
    const int64_t N = ctx->cfg.n;
    if (self_index)
        for (int64_t a = 0; a < m; ++a)
            if (self_index[a] < -1 || self_index[a] >= N)
                return fail(EMPP_EINVAL, "self_index[%lld] out of range", (long long)a);
    uint64_t bytes = 3 * m * sizeof(double) * 3 + (self_index ? m * sizeof(int64_t) : 0) +
                     (kstar ? (uint64_t)m * N * sizeof(int32_t) : 0) + 4 * kAlign;
    char *tmp = nullptr;
    hipError_t e = hipMalloc((void **)&tmp, bytes);
    if (e != hipSuccess)
        return fail(EMPP_ENOMEM, "hipMalloc(%llu) for fields_at failed", (unsigned long long)bytes);
    uint64_t o = 0;
    auto take = [&](uint64_t b) {
        char *p = tmp + o;
        o = align_up(o + b);
        return p;
    };
    double *xd = (double *)take(3 * m * sizeof(double));
    double *Ed = (double *)take(3 * m * sizeof(double));
    double *Bd = (double *)take(3 * m * sizeof(double));
    int64_t *sd = self_index ? (int64_t *)take(m * sizeof(int64_t)) : nullptr;
    int32_t *kd = kstar ? (int32_t *)take((uint64_t)m * N * sizeof(int32_t)) : nullptr;
    auto body = [&]() -> empp_status {
        HIP_TRY(hipMemcpyAsync(xd, x, 3 * m * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
        if (sd)
            HIP_TRY(hipMemcpyAsync(sd, self_index, m * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
        empp_status s2 = fields_dev_impl(ctx, m, xd, sd, Ed, Bd, kd);
        if (s2 != EMPP_OK)
            return s2;
        HIP_TRY(hipMemcpyAsync(E, Ed, 3 * m * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipMemcpyAsync(B, Bd, 3 * m * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        if (kd)
            HIP_TRY(hipMemcpyAsync(kstar, kd, (uint64_t)m * N * sizeof(int32_t), hipMemcpyDeviceToHost,
                                   ctx->stream));
        return check_err(ctx);
    };
    st = body();
    (void)hipStreamSynchronize(ctx->stream);
    (void)hipFree(tmp);
    return st;
}

empp_status empp_sync(empp_ctx *ctx)
{
    if (!ctx)
        return fail(EMPP_EINVAL, "NULL context");
    empp_status st = set_device(ctx);
    if (st != EMPP_OK)
        return st;
    return check_err(ctx);
}

empp_status empp_get_state(empp_ctx *ctx, double *r, double *u, double *t, int64_t *step)
{
    if (!ctx)
        return fail(EMPP_EINVAL, "NULL context");
    if (!ctx->have_history)
        return fail(EMPP_ESTATE, "no state yet");
    empp_status st = empp_sync(ctx);
    if (st != EMPP_OK)
        return st;
    const int64_t N = ctx->cfg.n;
    if (r) {
        double *tmp = nullptr;
        HIP_TRY(hipMalloc((void **)&tmp, 3 * N * sizeof(double)));
        hipError_t e = launch_newest_positions(ctx->present_pos(), tmp, N, ctx->present_depth(), ctx->present_head(),
                                               ctx->stream);
        if (e == hipSuccess)
            e = hipMemcpyAsync(r, tmp, 3 * N * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(ctx->stream);
        (void)hipFree(tmp);
        if (e != hipSuccess)
            return fail(EMPP_EDEVICE, "get_state: %s", hipGetErrorString(e));
    }
    if (u) {
        HIP_TRY(hipMemcpyAsync(u, ctx->u(), 3 * N * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    }
    if (t)
        *t = ctx->t_now;
    if (step)
        *step = ctx->step;
    return EMPP_OK;
}

empp_status empp_get_history(empp_ctx *ctx, double *T, double *w, double *v)
{
    if (!ctx || !T || !w || !v)
        return fail(EMPP_EINVAL, "NULL argument");
    if (!ctx->have_history || ctx->handed_off)
        return fail(EMPP_ESTATE, "no history");
    empp_status st = empp_sync(ctx);
    if (st != EMPP_OK)
        return st;
    const int64_t N = ctx->cfg.n;
    const int D = ctx->cfg.depth;
    const uint64_t tot = 3 * (uint64_t)N * D;
    double *tmp = nullptr;
    HIP_TRY(hipMalloc((void **)&tmp, 2 * tot * sizeof(double)));
    hipError_t e = launch_ring_to_history(ctx->ring_w(), ctx->ring_v(), tmp, tmp + tot, N, D, ctx->head, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(w, tmp, tot * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(v, tmp + tot, tot * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    std::vector<double> Tp(D);
    if (e == hipSuccess)
        e = hipMemcpyAsync(Tp.data(), ctx->T(), D * sizeof(double), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(ctx->stream);
    (void)hipFree(tmp);
    if (e != hipSuccess)
        return fail(EMPP_EDEVICE, "get_history: %s", hipGetErrorString(e));
    for (int s = 0; s < D; ++s) {
        int ph = ctx->head - (D - 1 - s);
        ph += ph < 0 ? D : 0;
        T[s] = Tp[ph];
    }
    return EMPP_OK;
}

empp_status empp_get_fields(empp_ctx *ctx, double *E, double *B)
{
    if (!ctx || !E || !B)
        return fail(EMPP_EINVAL, "NULL argument");
    if (!ctx->have_history)
        return fail(EMPP_ESTATE, "no state yet");
    empp_status st = empp_sync(ctx);
    if (st != EMPP_OK)
        return st;
    const int64_t N = ctx->cfg.n;
    HIP_TRY(hipMemcpyAsync(E, ctx->E(), 3 * N * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipMemcpyAsync(B, ctx->B(), 3 * N * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return EMPP_OK;
}

empp_status empp_get_diag(empp_ctx *ctx, empp_diag *out)
{
    if (!ctx || !out)
        return fail(EMPP_EINVAL, "NULL argument");
    if (!ctx->have_history)
        return fail(EMPP_ESTATE, "no state yet");
    empp_status st = empp_sync(ctx);
    if (st != EMPP_OK)
        return st;
    const int64_t N = ctx->cfg.n;
    const int64_t nb = (N + kBlock - 1) / kBlock;
    HIP_TRY(launch_diag(ctx->present_pos(), ctx->u(), N, ctx->present_depth(), ctx->present_head(), ctx->diag(),
                        ctx->stream));
    std::vector<double> h(nb * 7);
    double4 ref;
    HIP_TRY(hipMemcpyAsync(h.data(), ctx->diag(), nb * 7 * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipMemcpyAsync(&ref, ctx->present_pos() + ctx->present_head(), sizeof ref, hipMemcpyDeviceToHost,
                           ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    double s[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int64_t b = 0; b < nb; ++b)
        for (int k = 0; k < 7; ++k)
            s[k] += h[b * 7 + k];
    const double inv = 1.0 / (double)N;
    const double refc[3] = {ref.x, ref.y, ref.z};
    for (int k = 0; k < 3; ++k) {
        double mean = s[k] * inv;
        double var = s[3 + k] * inv - mean * mean;
        out->sigma[k] = std::sqrt(std::max(var, 0.0));
        out->centroid[k] = refc[k] + mean;
    }
    out->sigma_xy = 0.5 * (out->sigma[0] + out->sigma[1]);
    out->mean_kinetic = s[6] * inv * ctx->cfg.m * kC_LIGHT * kC_LIGHT;
    out->t = ctx->t_now;
    out->step = ctx->step;
    out->dt_last = ctx->cfg.dt;
    if (ctx->cfg.adaptive) {
        HIP_TRY(hipMemcpyAsync(&out->dt_last, ctx->ad() + 4, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    }
    return EMPP_OK;
}

empp_status empp_set_counting(empp_ctx *ctx, int32_t enable)
{
    if (!ctx)
        return fail(EMPP_EINVAL, "NULL context");
    empp_status st = set_device(ctx);
    if (st != EMPP_OK)
        return st;
    ctx->counting = enable != 0;
    HIP_TRY(hipMemsetAsync(ctx->counters(), 0, 8 * sizeof(unsigned long long), ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return EMPP_OK;
}

empp_status empp_get_counters(empp_ctx *ctx, empp_counters *out)
{
    if (!ctx || !out)
        return fail(EMPP_EINVAL, "NULL argument");
    empp_status st = set_device(ctx);
    if (st != EMPP_OK)
        return st;
    unsigned long long h[8];
    HIP_TRY(hipMemcpyAsync(h, ctx->counters(), sizeof h, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    out->pairs = h[0];
    out->before = h[1];
    out->probes = h[2];
    out->rescues = h[3];
    out->fallbacks = h[4];
    return EMPP_OK;
}

empp_status empp_set_timing(empp_ctx *ctx, int32_t enable)
{
    if (!ctx)
        return fail(EMPP_EINVAL, "NULL context");
    empp_status st = set_device(ctx);
    if (st != EMPP_OK)
        return st;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->timing = enable != 0;
    ctx->ev_used = 0;
    ctx->ev_marks.clear();
    return EMPP_OK;
}

empp_status empp_get_timing(empp_ctx *ctx, empp_timing *out)
{
    if (!ctx || !out)
        return fail(EMPP_EINVAL, "NULL argument");
    empp_status st = set_device(ctx);
    if (st != EMPP_OK)
        return st;
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    *out = empp_timing{};
    for (auto &mk : ctx->ev_marks) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ctx->ev_pool[mk.first], ctx->ev_pool[mk.first + 1]));
        if (mk.second == 0) {
            out->pair_ms += ms;
            out->pair_launches += 1;
        } else if (mk.second == 1) {
            out->push_ms += ms;
            out->push_launches += 1;
        } else {
            out->guess_ms += ms;
            out->guess_launches += 1;
        }
    }
    ctx->ev_used = 0;
    ctx->ev_marks.clear();
    return EMPP_OK;
}

static empp_status surrogate_alloc(empp_ctx *ctx)
{
    if (ctx->sg.master)
        return EMPP_OK;
    const int64_t N = ctx->cfg.n;
    const int64_t ng = (N + 63) / 64;
    struct {
        void **p;
        size_t bytes;
    } want[] = {
        {(void **)&ctx->sg.master, kParams * sizeof(float)},
        {(void **)&ctx->sg.m, kParams * sizeof(float)},
        {(void **)&ctx->sg.v, kParams * sizeof(float)},
        {(void **)&ctx->sg.grad, (kParams + 1) * sizeof(float)},
        {(void **)&ctx->sg.part, (size_t)ctx->sg.part_blocks * kPartStride * sizeof(float)},
        {(void **)&ctx->sg.net, sizeof(MlpPacked)},
        {(void **)&ctx->sg.G, (size_t)ng * N * sizeof(float)},
        {(void **)&ctx->sg.cent, (size_t)ng * sizeof(double3)},
        {(void **)&ctx->sg.cent_big, (size_t)ng * sizeof(double3)},
        {(void **)&ctx->sg.sync, (size_t)kSyncLine * (kSyncMaxBlocks + 1) * sizeof(unsigned long long)},
        {(void **)&ctx->sg.sync_fail, sizeof(unsigned int)},
        {(void **)&ctx->sg.loss_first, sizeof(float)},
    };
    for (auto &w : want) {
        hipError_t e = hipMalloc(w.p, w.bytes);
        if (e != hipSuccess)
            return fail(EMPP_ENOMEM, "hipMalloc(%zu) for the surrogate failed: %s", w.bytes, hipGetErrorString(e));
    }
    int dev = 0, nb = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(mlp_train_max_blocks(dev, &nb));
    if (nb < 1)
        return fail(EMPP_EDEVICE, "the training step does not fit on the device");
    ctx->sg.train_blocks = std::min(std::min(nb, ctx->sg.part_blocks), kSyncMaxBlocks);
    return EMPP_OK;
}

empp_status empp_surrogate_set(empp_ctx *ctx, const float *params, int64_t nparams, double sigma_ref)
{
    if (!ctx || !params)
        return fail(EMPP_EINVAL, "NULL argument");
    if (nparams != kParams)
        return fail(EMPP_EINVAL, "nparams %lld != %d", (long long)nparams, kParams);
    if (!(sigma_ref > 0.0) || !std::isfinite(sigma_ref))
        return fail(EMPP_EINVAL, "sigma_ref must be positive");
    for (int64_t i = 0; i < nparams; ++i)
        if (!std::isfinite(params[i]))
            return fail(EMPP_EINVAL, "non-finite parameter %lld", (long long)i);
    empp_status st = set_device(ctx);
    if (st != EMPP_OK || (st = surrogate_alloc(ctx)) != EMPP_OK)
        return st;
    HIP_TRY(hipMemcpyAsync(ctx->sg.master, params, kParams * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipMemsetAsync(ctx->sg.m, 0, kParams * sizeof(float), ctx->stream));
    HIP_TRY(hipMemsetAsync(ctx->sg.v, 0, kParams * sizeof(float), ctx->stream));
    HIP_TRY(launch_mlp_pack(ctx->sg.master, ctx->sg.net, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->sg.adam_step = 0;
    ctx->sg.sigma_ref = sigma_ref;
    ctx->sg.ready = true;
    return EMPP_OK;
}

empp_status empp_surrogate_get(empp_ctx *ctx, float *params, int64_t nparams)
{
    if (!ctx || !params)
        return fail(EMPP_EINVAL, "NULL argument");
    if (nparams != kParams)
        return fail(EMPP_EINVAL, "nparams %lld != %d", (long long)nparams, kParams);
    if (!ctx->sg.ready)
        return fail(EMPP_ESTATE, "no surrogate network");
    empp_status st = set_device(ctx);
    if (st != EMPP_OK)
        return st;
    HIP_TRY(hipMemcpyAsync(params, ctx->sg.master, kParams * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return EMPP_OK;
}

static SampleParams sample_params(empp_ctx *ctx, uint64_t seed)
{
    SampleParams sp{};
    sp.ring_w = ctx->ring_w();
    sp.ring_v = ctx->ring_v();
    sp.T = ctx->T();
    sp.N = ctx->cfg.n;
    sp.D = ctx->cfg.depth;
    sp.head = ctx->head;
    sp.t = ctx->t_now;
    sp.inv_sigma = 1.0 / ctx->sg.sigma_ref;
    sp.seed = seed;
    return sp;
}

static empp_status surrogate_precheck(empp_ctx *ctx, bool need_state)
{
    if (!ctx)
        return fail(EMPP_EINVAL, "NULL context");
    if (!ctx->sg.ready)
        return fail(EMPP_ESTATE, "no surrogate network (empp_surrogate_set)");
    if (need_state && (!ctx->have_history || ctx->handed_off))
        return fail(EMPP_ESTATE, "no history to sample from");
    if (need_state && ctx->cfg.depth < 5)
        return fail(EMPP_EUNSUPPORTED, "features need at least 5 history slots");
    return set_device(ctx);
}

empp_status empp_surrogate_samples_dev(empp_ctx *ctx, int64_t count, uint64_t seed, float *X_dev, float *y_dev)
{
    empp_status st = surrogate_precheck(ctx, true);
    if (st != EMPP_OK)
        return st;
    if (count < 0 || (count > 0 && (!X_dev || !y_dev)))
        return fail(EMPP_EINVAL, "bad sample buffers");
    if (count == 0)
        return EMPP_OK;
    HIP_TRY(launch_mlp_sample(sample_params(ctx, seed), nullptr, nullptr, count, X_dev, y_dev, ctx->stream));
    return EMPP_OK;
}

empp_status empp_surrogate_samples(empp_ctx *ctx, int64_t count, uint64_t seed, const int64_t *tgt, const int64_t *src,
                                   float *X, float *y)
{
    empp_status st = surrogate_precheck(ctx, true);
    if (st != EMPP_OK)
        return st;
    if (count < 0 || (count > 0 && (!X || !y)) || ((tgt == nullptr) != (src == nullptr)))
        return fail(EMPP_EINVAL, "bad sample arguments");
    if (count == 0)
        return EMPP_OK;
    const int64_t N = ctx->cfg.n;
    if (tgt)
        for (int64_t q = 0; q < count; ++q)
            if (tgt[q] < 0 || tgt[q] >= N || src[q] < 0 || src[q] >= N || tgt[q] == src[q])
                return fail(EMPP_EINVAL, "pair %lld out of range or a self pair", (long long)q);
    size_t bytes = (size_t)count * (kIn + 1) * sizeof(float) + (tgt ? 2 * count * sizeof(int64_t) : 0) + 512;
    char *tmp = nullptr;
    HIP_TRY(hipMalloc((void **)&tmp, bytes));
    float *Xd = (float *)tmp;
    float *yd = Xd + count * kIn;
    int64_t *td = tgt ? (int64_t *)(tmp + align_up((size_t)count * (kIn + 1) * sizeof(float))) : nullptr;
    int64_t *sd = tgt ? td + count : nullptr;
    auto body = [&]() -> empp_status {
        if (tgt) {
            HIP_TRY(hipMemcpyAsync(td, tgt, count * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
            HIP_TRY(hipMemcpyAsync(sd, src, count * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
        }
        HIP_TRY(launch_mlp_sample(sample_params(ctx, seed), td, sd, count, Xd, yd, ctx->stream));
        HIP_TRY(hipMemcpyAsync(X, Xd, count * kIn * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipMemcpyAsync(y, yd, count * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        return EMPP_OK;
    };
    st = body();
    (void)hipFree(tmp);
    return st;
}

empp_status empp_surrogate_forward(empp_ctx *ctx, const float *X, int64_t count, float *z)
{
    empp_status st = surrogate_precheck(ctx, false);
    if (st != EMPP_OK)
        return st;
    if (count < 0 || (count > 0 && (!X || !z)))
        return fail(EMPP_EINVAL, "bad arguments");
    if (count == 0)
        return EMPP_OK;
    float *tmp = nullptr;
    HIP_TRY(hipMalloc((void **)&tmp, (size_t)count * (kIn + 1) * sizeof(float)));
    auto body = [&]() -> empp_status {
        HIP_TRY(hipMemcpyAsync(tmp, X, count * kIn * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(launch_mlp_forward(ctx->sg.net, tmp, count, tmp + count * kIn, ctx->stream));
        HIP_TRY(hipMemcpyAsync(z, tmp + count * kIn, count * sizeof(float), hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        return EMPP_OK;
    };
    st = body();
    (void)hipFree(tmp);
    return st;
}

// Training on device rows: per optimizer step, partial gradients per
// block, their fixed-order sum into sg.grad ([kParams] gradient, then the
// sum of squared residuals) and, with apply, the Adam update of the masters
// and the packed network; kStepsPerLaunch steps per cooperative launch.
// apply = 0: one gradient evaluation of rows X[count] (batch = count).
// Synchronous; a grid-barrier wait that gave up is an error.
static empp_status surrogate_run(empp_ctx *ctx, const float *X, const float *y, int64_t count, int64_t batch,
                                 int64_t steps, double lr, double lr_final, int apply)
{
    constexpr int64_t kStepsPerLaunch = 256;
    const int nb = (int)std::min<int64_t>(ctx->sg.train_blocks, (batch + 63) / 64);
    const int64_t nl = (steps + kStepsPerLaunch - 1) / kStepsPerLaunch;
    std::vector<TrainRun> runs((size_t)nl);
    unsigned long long arrivals = 0;
    for (int64_t k = 0; k < nl; ++k) {
        TrainRun &r = runs[(size_t)k];
        r.net = ctx->sg.net;
        r.X = X;
        r.y = y;
        r.count = count;
        r.batch = (int32_t)batch;
        r.step0 = k * kStepsPerLaunch;
        r.steps = (int32_t)std::min(kStepsPerLaunch, steps - r.step0);
        r.total = steps;
        r.adam0 = ctx->sg.adam_step + r.step0;
        r.lr = lr;
        r.lr_final = lr_final;
        r.apply = apply;
        r.part = ctx->sg.part;
        r.grad = ctx->sg.grad;
        r.master = ctx->sg.master;
        r.m = ctx->sg.m;
        r.v = ctx->sg.v;
        r.loss_first = ctx->sg.loss_first;
        r.sync = ctx->sg.sync;
        r.sync_base = arrivals;
        r.fail = ctx->sg.sync_fail;
        arrivals += (unsigned long long)nb * (unsigned long long)(2 * r.steps - 1);
    }
    TrainRun *dev = nullptr;
    HIP_TRY(hipMalloc((void **)&dev, (size_t)nl * sizeof(TrainRun)));
    auto body = [&]() -> empp_status {
        HIP_TRY(hipMemcpy(dev, runs.data(), (size_t)nl * sizeof(TrainRun), hipMemcpyHostToDevice));
        HIP_TRY(launch_mlp_sync_clear(ctx->sg.sync, ctx->sg.sync_fail, ctx->stream));
        for (int64_t k = 0; k < nl; ++k)
            HIP_TRY(launch_mlp_train(dev + k, nb, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        unsigned int f = 0;
        HIP_TRY(hipMemcpy(&f, ctx->sg.sync_fail, sizeof(f), hipMemcpyDeviceToHost));
        if (f)
            return fail(EMPP_EDEVICE, "a grid barrier of the training kernel timed out");
        return EMPP_OK;
    };
    empp_status st = body();
    (void)hipFree(dev);
    if (st == EMPP_OK && apply)
        ctx->sg.adam_step += steps;
    return st;
}

empp_status empp_surrogate_loss_grad(empp_ctx *ctx, const float *X, const float *y, int64_t count, double *loss,
                                     float *grad)
{
    empp_status st = surrogate_precheck(ctx, false);
    if (st != EMPP_OK)
        return st;
    if (count <= 0 || count > (int64_t)INT32_MAX || !X || !y || !grad)
        return fail(EMPP_EINVAL, "bad arguments");
    float *tmp = nullptr;
    HIP_TRY(hipMalloc((void **)&tmp, (size_t)count * (kIn + 1) * sizeof(float)));
    std::vector<float> g(kParams + 1);
    auto body = [&]() -> empp_status {
        HIP_TRY(hipMemcpyAsync(tmp, X, count * kIn * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(hipMemcpyAsync(tmp + count * kIn, y, count * sizeof(float), hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        empp_status s2 = surrogate_run(ctx, tmp, tmp + count * kIn, count, count, 1, 0.0, 0.0, 0);
        if (s2 != EMPP_OK)
            return s2;
        HIP_TRY(hipMemcpy(g.data(), ctx->sg.grad, (kParams + 1) * sizeof(float), hipMemcpyDeviceToHost));
        return EMPP_OK;
    };
    st = body();
    (void)hipFree(tmp);
    if (st != EMPP_OK)
        return st;
    std::copy(g.begin(), g.begin() + kParams, grad);
    if (loss)
        *loss = (double)g[kParams] / (double)count;
    return EMPP_OK;
}

empp_status empp_surrogate_train(empp_ctx *ctx, const float *X_dev, const float *y_dev, int64_t count,
                                 const empp_train_cfg *cfg, empp_train_report *out)
{
    empp_status st = surrogate_precheck(ctx, false);
    if (st != EMPP_OK)
        return st;
    if (!X_dev || !y_dev || !cfg || count <= 0)
        return fail(EMPP_EINVAL, "bad arguments");
    if (cfg->batch <= 0 || cfg->batch % 64 != 0 || cfg->batch > count || cfg->steps < 0 || !(cfg->lr > 0.0f))
        return fail(EMPP_EINVAL, "bad training configuration");
    auto t0 = std::chrono::steady_clock::now();
    float first = 0.0f, last = 0.0f;
    const int64_t B = cfg->batch;
    if (cfg->steps > 0) {
        if ((st = surrogate_run(ctx, X_dev, y_dev, count, B, cfg->steps, (double)cfg->lr, (double)cfg->lr_final, 1)) !=
            EMPP_OK)
            return st;
        HIP_TRY(hipMemcpy(&first, ctx->sg.loss_first, sizeof(float), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(&last, ctx->sg.grad + kParams, sizeof(float), hipMemcpyDeviceToHost));
    }
    auto t1 = std::chrono::steady_clock::now();
    if (out) {
        out->loss_first = (double)first / (double)B;
        out->loss_last = (double)last / (double)B;
        out->steps = cfg->steps;
        out->seconds = std::chrono::duration<double>(t1 - t0).count();
    }
    return EMPP_OK;
}

empp_status empp_set_mode(empp_ctx *ctx, int32_t precision, int32_t guess)
{
    if (!ctx)
        return fail(EMPP_EINVAL, "NULL context");
    empp_config c = ctx->cfg;
    c.precision = precision;
    c.guess = guess;
    empp_status st = validate(&c);
    if (st != EMPP_OK)
        return st;
    if (guess == EMPP_GUESS_PREVIOUS && !ctx->kc())
        return fail(EMPP_EUNSUPPORTED, "warm-start brackets need a context created with that guess mode");
    ctx->cfg.precision = precision;
    ctx->cfg.guess = guess;
    return EMPP_OK;
}


// ---- two-stage strategy (Sec. 2.7) -----------------------------------------

empp_status empp_step_until_switch(empp_ctx *ctx, double eps_E, int64_t check_every, int64_t max_steps,
                                   int64_t *steps_done, double *t_sw, int32_t *switched)
{
    if (!ctx)
        return fail(EMPP_EINVAL, "NULL context");
    if (!(eps_E >= 0.0) || check_every < 1 || max_steps < 0)
        return fail(EMPP_EINVAL, "need eps_E >= 0, check_every >= 1, max_steps >= 0");
    empp_diag d0;
    empp_status st = empp_get_diag(ctx, &d0);
    if (st != EMPP_OK)
        return st;
    int64_t done = 0;
    int32_t sw = 0;
    double e_prev = d0.mean_kinetic, t_prev = d0.t;
    while (done < max_steps) {
        const int64_t k = std::min(check_every, max_steps - done);
        if ((st = empp_step(ctx, k)) != EMPP_OK)
            return st;
        done += k;
        empp_diag d;
        if ((st = empp_get_diag(ctx, &d)) != EMPP_OK)
            return st;
        const double rate = (d.mean_kinetic - e_prev) / (d.t - t_prev);
        e_prev = d.mean_kinetic;
        t_prev = d.t;
        if (std::fabs(rate) < eps_E) {
            sw = 1;
            break;
        }
    }
    if (steps_done)
        *steps_done = done;
    if (t_sw)
        *t_sw = ctx->t_now;
    if (switched)
        *switched = sw;
    return EMPP_OK;
}

empp_status empp_handoff(empp_ctx *ctx)
{
    if (!ctx)
        return fail(EMPP_EINVAL, "NULL context");
    if (!ctx->have_history)
        return fail(EMPP_ESTATE, "handoff before the history is initialised");
    if (ctx->handed_off)
        return fail(EMPP_ESTATE, "handoff already done");
    empp_status st = set_device(ctx);
    if (st != EMPP_OK)
        return st;
    // the Stage-I steps before the handoff must have succeeded
    if ((st = check_err(ctx)) != EMPP_OK)
        return st;
    const double dip_k = ctx->cfg.dipole_b0 * ctx->cfg.dipole_re * ctx->cfg.dipole_re * ctx->cfg.dipole_re;
    HIP_TRY(launch_handoff(ctx->ring_w(), ctx->cfg.depth, ctx->head, ctx->pos(), ctx->u(), ctx->cfg.n, dip_k,
                           ctx->cfg.ext_field, ctx->skey(), ctx->stime(), ctx->t_now, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->handed_off = true;
    ctx->tr_step = 0;
    return EMPP_OK;
}

empp_status empp_transport(empp_ctx *ctx, double dt_max, double gyro_fraction, int64_t nsteps)
{
    if (!ctx)
        return fail(EMPP_EINVAL, "NULL context");
    if (!ctx->handed_off)
        return fail(EMPP_ESTATE, "transport before handoff");
    if (!(dt_max > 0.0) || !std::isfinite(dt_max) || !(gyro_fraction > 0.0) || nsteps < 0)
        return fail(EMPP_EINVAL, "need dt_max > 0, gyro_fraction > 0, nsteps >= 0");
    empp_status st = set_device(ctx);
    if (st != EMPP_OK)
        return st;
    TransportParams p{};
    p.pos = ctx->pos();
    p.u = ctx->u();
    p.N = ctx->cfg.n;
    p.q_over_2m = ctx->cfg.q / (2.0 * ctx->cfg.m);
    p.dip_k = ctx->cfg.dipole_b0 * ctx->cfg.dipole_re * ctx->cfg.dipole_re * ctx->cfg.dipole_re;
    p.ext_field = ctx->cfg.ext_field;
    p.dt_max = dt_max;
    p.gyro_k = ctx->cfg.q != 0.0 ? gyro_fraction * 2.0 * M_PI * ctx->cfg.m / std::fabs(ctx->cfg.q) : INFINITY;
    p.key = ctx->skey();
    p.t = ctx->stime();
    for (int64_t k = 0; k < nsteps; ++k) {
        p.step = ctx->tr_step++;
        HIP_TRY(timed(ctx, 1, [&]() { return launch_transport(p, ctx->stream); }));
    }
    double t = 0.0;
    HIP_TRY(hipMemcpyAsync(&t, ctx->stime(), sizeof t, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->t_now = t;
    ctx->step += nsteps;
    return check_err(ctx);
}

// ---- checkpoint --------------------------------------------------------------

namespace {
struct CkptHeader {
    char magic[8];
    int64_t n;
    int32_t depth, head;
    int64_t step, tr_step;
    double t_now, t_origin;
    int32_t stage, reserved;
    double q, m, dt;
};
constexpr char kCkptMagic[8] = {'E', 'M', 'P', 'P', 'C', 'K', 'P', '1'};

// Device <-> file through a bounded host buffer.
empp_status dev_to_file(empp_ctx *ctx, FILE *f, const void *dev, uint64_t bytes)
{
    std::vector<char> buf((size_t)std::min<uint64_t>(bytes, 64ull << 20));
    for (uint64_t o = 0; o < bytes; o += buf.size()) {
        size_t k = (size_t)std::min<uint64_t>(buf.size(), bytes - o);
        HIP_TRY(hipMemcpyAsync(buf.data(), (const char *)dev + o, k, hipMemcpyDeviceToHost, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
        if (fwrite(buf.data(), 1, k, f) != k)
            return fail(EMPP_EINVAL, "checkpoint write failed: %s", strerror(errno));
    }
    return EMPP_OK;
}

empp_status file_to_dev(empp_ctx *ctx, FILE *f, void *dev, uint64_t bytes)
{
    std::vector<char> buf((size_t)std::min<uint64_t>(bytes, 64ull << 20));
    for (uint64_t o = 0; o < bytes; o += buf.size()) {
        size_t k = (size_t)std::min<uint64_t>(buf.size(), bytes - o);
        if (fread(buf.data(), 1, k, f) != k)
            return fail(EMPP_EINVAL, "checkpoint truncated");
        HIP_TRY(hipMemcpyAsync((char *)dev + o, buf.data(), k, hipMemcpyHostToDevice, ctx->stream));
        HIP_TRY(hipStreamSynchronize(ctx->stream));
    }
    return EMPP_OK;
}

// The target order indexes the history ring in the pair kernel: accept it
// only as a permutation of 0..N-1.
empp_status order_from_file(empp_ctx *ctx, FILE *f)
{
    const int64_t N = ctx->cfg.n;
    std::vector<int32_t> ord((size_t)N);
    if (fread(ord.data(), sizeof(int32_t), (size_t)N, f) != (size_t)N)
        return fail(EMPP_EINVAL, "checkpoint truncated");
    std::vector<char> seen((size_t)N, 0);
    for (int64_t i = 0; i < N; ++i) {
        const int32_t k = ord[(size_t)i];
        if (k < 0 || k >= N || seen[(size_t)k])
            return fail(EMPP_EINVAL, "corrupt checkpoint: target order is not a permutation");
        seen[(size_t)k] = 1;
    }
    HIP_TRY(hipMemcpyAsync(ctx->order(), ord.data(), N * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    return EMPP_OK;
}
}  // namespace

empp_status empp_save(empp_ctx *ctx, const char *path)
{
    if (!ctx || !path)
        return fail(EMPP_EINVAL, "NULL argument");
    if (!ctx->have_history)
        return fail(EMPP_ESTATE, "nothing to save before the history is initialised");
    empp_status st = empp_sync(ctx);
    if (st != EMPP_OK)
        return st;
    FILE *f = fopen(path, "wb");
    if (!f)
        return fail(EMPP_EINVAL, "cannot open %s: %s", path, strerror(errno));
    const int64_t N = ctx->cfg.n;
    const int D = ctx->cfg.depth;
    CkptHeader h{};
    memcpy(h.magic, kCkptMagic, 8);
    h.n = N;
    h.depth = D;
    h.head = ctx->head;
    h.step = ctx->step;
    h.tr_step = ctx->tr_step;
    h.t_now = ctx->t_now;
    h.t_origin = ctx->t_origin;
    h.stage = ctx->handed_off ? 2 : 1;
    h.q = ctx->cfg.q;
    h.m = ctx->cfg.m;
    h.dt = ctx->cfg.dt;
    if (fwrite(&h, sizeof h, 1, f) != 1)
        st = fail(EMPP_EINVAL, "checkpoint write failed: %s", strerror(errno));
    if (st == EMPP_OK)
        st = dev_to_file(ctx, f, ctx->T(), D * sizeof(double));
    if (st == EMPP_OK)
        st = dev_to_file(ctx, f, ctx->u(), 3 * N * sizeof(double));
    if (st == EMPP_OK)
        st = dev_to_file(ctx, f, ctx->order(), N * sizeof(int32_t));
    if (st == EMPP_OK && h.stage == 1) {
        st = dev_to_file(ctx, f, ctx->ring_w(), (uint64_t)N * D * sizeof(double4));
        if (st == EMPP_OK)
            st = dev_to_file(ctx, f, ctx->ring_v(), (uint64_t)N * D * sizeof(double4));
    }
    if (st == EMPP_OK && h.stage == 2) {
        st = dev_to_file(ctx, f, ctx->pos(), N * sizeof(double4));
        if (st == EMPP_OK)
            st = dev_to_file(ctx, f, ctx->skey(), 3 * sizeof(unsigned long long));
        if (st == EMPP_OK)
            st = dev_to_file(ctx, f, ctx->stime(), sizeof(double));
    }
    if (fclose(f) != 0 && st == EMPP_OK)
        st = fail(EMPP_EINVAL, "checkpoint close failed: %s", strerror(errno));
    return st;
}

empp_status empp_load(empp_ctx *ctx, const char *path)
{
    if (!ctx || !path)
        return fail(EMPP_EINVAL, "NULL argument");
    empp_status st = set_device(ctx);
    if (st != EMPP_OK)
        return st;
    FILE *f = fopen(path, "rb");
    if (!f)
        return fail(EMPP_EINVAL, "cannot open %s: %s", path, strerror(errno));
    CkptHeader h{};
    const int64_t N = ctx->cfg.n;
    const int D = ctx->cfg.depth;
    if (fread(&h, sizeof h, 1, f) != 1 || memcmp(h.magic, kCkptMagic, 8) != 0)
        st = fail(EMPP_EINVAL, "%s is not a checkpoint", path);
    else if (h.n != N || h.depth != D || h.q != ctx->cfg.q || h.m != ctx->cfg.m || h.dt != ctx->cfg.dt)
        st = fail(EMPP_EINVAL, "checkpoint (n %lld, depth %d, q, m, dt) does not match the context",
                  (long long)h.n, h.depth);
    else if ((h.stage != 1 && h.stage != 2) || h.head < 0 || h.head >= D)
        st = fail(EMPP_EINVAL, "corrupt checkpoint header");
    if (st == EMPP_OK)
        st = file_to_dev(ctx, f, ctx->T(), D * sizeof(double));
    if (st == EMPP_OK)
        st = file_to_dev(ctx, f, ctx->u(), 3 * N * sizeof(double));
    if (st == EMPP_OK)
        st = order_from_file(ctx, f);
    if (st == EMPP_OK && h.stage == 1) {
        st = file_to_dev(ctx, f, ctx->ring_w(), (uint64_t)N * D * sizeof(double4));
        if (st == EMPP_OK)
            st = file_to_dev(ctx, f, ctx->ring_v(), (uint64_t)N * D * sizeof(double4));
    }
    if (st == EMPP_OK && h.stage == 2) {
        st = file_to_dev(ctx, f, ctx->pos(), N * sizeof(double4));
        if (st == EMPP_OK)
            st = file_to_dev(ctx, f, ctx->skey(), 3 * sizeof(unsigned long long));
        if (st == EMPP_OK)
            st = file_to_dev(ctx, f, ctx->stime(), sizeof(double));
    }
    fclose(f);
    if (st != EMPP_OK) {
        // the device state is partly overwritten: nothing valid remains
        ctx->have_history = false;
        ctx->handed_off = false;
        return st;
    }
    HIP_TRY(hipMemsetAsync(ctx->E(), 0, 3 * N * sizeof(double), ctx->stream));
    HIP_TRY(hipMemsetAsync(ctx->B(), 0, 3 * N * sizeof(double), ctx->stream));
    HIP_TRY(hipStreamSynchronize(ctx->stream));
    ctx->have_bunch = false;
    ctx->have_history = true;
    ctx->handed_off = h.stage == 2;
    ctx->kc_valid = false;
    if ((st = reset_adaptive(ctx)) != EMPP_OK)
        return st;
    ctx->head = h.head;
    ctx->step = h.step;
    ctx->tr_step = h.tr_step;
    ctx->t_now = h.t_now;
    ctx->t_origin = h.t_origin;
    return EMPP_OK;
}

}  // extern "C"
