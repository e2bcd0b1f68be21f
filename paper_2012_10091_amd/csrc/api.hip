// C ABI of libmenkf: context, workspace planner, argument validation and
// dispatch to the HIP kernels.  See include/menkf.h for the contract of
// every entry point.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "common.hpp"

using namespace menkf;

struct menkf_ctx {
    Plan plan;
    void *ws = nullptr;
    size_t ws_bytes = 0;
    const int32_t *idx = nullptr;
    const int32_t *comp = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;   // menkf_cycle with an aux stream
    hipEvent_t ev_front = nullptr;                       // end of the gain's front end (deferred path)
    int n_cus = 256;                                     // compute units of the workspace's device
    char err[512] = {0};
    ~menkf_ctx() {
        if (ev_fork) hipEventDestroy(ev_fork);
        if (ev_join) hipEventDestroy(ev_join);
        if (ev_front) hipEventDestroy(ev_front);
    }
};

struct menkf_batch {
    std::vector<hipStream_t> lanes;
    std::vector<hipEvent_t> join;
    hipEvent_t fork = nullptr;
    std::vector<int32_t> lane_of;
};

struct menkf_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static thread_local char g_err[512];

static menkf_status fail(menkf_ctx *c, menkf_status st, const char *fmt, ...) {
    char *buf = c ? c->err : g_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
    return st;
}

static menkf_status hip_fail(menkf_ctx *c, hipError_t e, const char *where) {
    return fail(c, MENKF_E_HIP, "%s: %s", where, hipGetErrorString(e));
}

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }
static int roundup(int v, int m) { return (v + m - 1) / m * m; }

static menkf_status build_plan(const menkf_config *cfg, Plan *p) {
    std::memset(p, 0, sizeof(*p));
    p->cfg = *cfg;
    if (cfg->model != MENKF_BURGERS1D && cfg->model != MENKF_NS2D && cfg->model != MENKF_BURGERS1D_INLET &&
        cfg->model != MENKF_EULER1D_INLET)
        return fail(nullptr, MENKF_E_ARG,
                    "model must be MENKF_BURGERS1D, MENKF_NS2D, MENKF_BURGERS1D_INLET or MENKF_EULER1D_INLET (got %d)",
                    cfg->model);
    if (cfg->precision != MENKF_F32 && cfg->precision != MENKF_F64)
        return fail(nullptr, MENKF_E_ARG, "precision must be MENKF_F32 or MENKF_F64 (got %d)", cfg->precision);
    if (cfg->gain_mode != MENKF_GAIN_EXACT_R && cfg->gain_mode != MENKF_GAIN_SAMPLE_EE &&
        cfg->gain_mode != MENKF_GAIN_ENSEMBLE_SPACE)
        return fail(nullptr, MENKF_E_ARG, "unknown gain_mode %d", cfg->gain_mode);
    const bool euler = cfg->model == MENKF_EULER1D_INLET;
    p->dim = cfg->model == MENKF_NS2D ? 2 : 1;
    p->F = p->dim == 2 ? 4 : (euler ? 3 : 1);
    p->obs_field = euler ? 1 : 0;
    const int r = cfg->ratio;
    if (r < 1 || r > 64) return fail(nullptr, MENKF_E_ARG, "ratio must be in [1, 64] (got %d)", r);
    if (cfg->nx < 1 || cfg->nx % r) return fail(nullptr, MENKF_E_SHAPE, "nx=%d must be a positive multiple of ratio=%d", cfg->nx, r);
    if (p->dim == 1 && cfg->ny != 1) return fail(nullptr, MENKF_E_SHAPE, "1D model needs ny = 1 (got %d)", cfg->ny);
    if (p->dim == 2 && (cfg->ny < 1 || cfg->ny % r))
        return fail(nullptr, MENKF_E_SHAPE, "ny=%d must be a positive multiple of ratio=%d", cfg->ny, r);
    p->nx = cfg->nx;
    p->ny = cfg->ny;
    p->nxc = cfg->nx / r;
    p->nyc = p->dim == 2 ? cfg->ny / r : 1;
    if (p->nxc < 4 || (p->dim == 2 && p->nyc < 4))
        return fail(nullptr, MENKF_E_SHAPE, "coarse grid %dx%d too small (cubic prolongation and the stencils need >= 4 nodes per direction)", p->nxc, p->nyc);
    if (p->dim == 2 && 4LL * cfg->nx * cfg->ny * (cfg->precision == MENKF_F64 ? 8 : 4) >= (1LL << 31))
        return fail(nullptr, MENKF_E_SHAPE, "fine grid too large: one state (4 fields) must stay below 2 GiB "
                                            "(32-bit byte offsets)");
    p->nf = (long long)p->nx * p->ny;
    p->nc = (long long)p->nxc * p->nyc;
    if (cfg->n_members < 2 || cfg->n_members > 256)
        return fail(nullptr, MENKF_E_ARG, "n_members must be in [2, 256] (got %d)", cfg->n_members);
    if (cfg->n_probes < 1) return fail(nullptr, MENKF_E_ARG, "n_probes must be >= 1 (got %d)", cfg->n_probes);
    if (!(cfg->dt > 0) || !(cfg->length > 0)) return fail(nullptr, MENKF_E_ARG, "dt and length must be positive");
    if (p->dim == 1 && !(cfg->nu >= 0)) return fail(nullptr, MENKF_E_ARG, "nu must be >= 0");
    p->open = (cfg->model == MENKF_BURGERS1D_INLET || euler) ? 1 : 0;
    if (euler) {
        if (!(cfg->gamma > 1) || !(cfg->mach > 0 && cfg->mach < 1))
            return fail(nullptr, MENKF_E_ARG, "MENKF_EULER1D_INLET needs gamma > 1 and a subsonic inlet, 0 < mach < 1");
        if (!(cfg->filter_sigma >= 0 && cfg->filter_sigma <= 1))
            return fail(nullptr, MENKF_E_ARG, "filter_sigma must be in [0, 1]");
        if (cfg->nx / cfg->ratio < 8)
            return fail(nullptr, MENKF_E_SHAPE, "MENKF_EULER1D_INLET needs >= 8 coarse nodes (filter stencils)");
        const size_t ts = cfg->precision == MENKF_F64 ? 8 : 4;
        if (cfg->nx > 4096 || euler_window_lds(cfg->nx, ts) > 128 * 1024)
            return fail(nullptr, MENKF_E_UNSUPPORTED,
                        "MENKF_EULER1D_INLET keeps a state in LDS: nx = %d exceeds %d", cfg->nx,
                        cfg->precision == MENKF_F64 ? 1792 : 3612);
    }
    if (p->open) {
        if ((!euler && !std::isfinite(cfg->u0)) || !std::isfinite(cfg->omega))
            return fail(nullptr, MENKF_E_ARG, "the inlet-forced models need finite u0 (Burgers) and omega");
        if (!(cfg->theta_sigma[0] >= 0) || !(cfg->theta_sigma[1] >= 0) || !std::isfinite(cfg->theta_sigma[0]) ||
            !std::isfinite(cfg->theta_sigma[1]))
            return fail(nullptr, MENKF_E_ARG, "theta_sigma must be finite and >= 0");
        const size_t ts = cfg->precision == MENKF_F64 ? 8 : 4;
        if (!euler && (cfg->nx > 8192 || inlet_window_lds(cfg->nx, ts) > 128 * 1024))
            return fail(nullptr, MENKF_E_UNSUPPORTED,
                        "MENKF_BURGERS1D_INLET keeps a state row in LDS: nx = %d exceeds %d", cfg->nx,
                        cfg->precision == MENKF_F64 ? 5290 : 8192);
    }
    if (p->dim == 2 && !(cfg->gamma > 1 && cfg->mach > 0 && cfg->reynolds > 0 && cfg->prandtl > 0))
        return fail(nullptr, MENKF_E_ARG, "need gamma > 1, mach > 0, reynolds > 0, prandtl > 0");
    if (cfg->gain_mode != MENKF_GAIN_SAMPLE_EE && !(cfg->obs_sigma > 0))
        return fail(nullptr, MENKF_E_ARG, "obs_sigma must be > 0 with MENKF_GAIN_EXACT_R / ENSEMBLE_SPACE");
    if (cfg->gain_mode == MENKF_GAIN_SAMPLE_EE && cfg->n_probes > 2 * cfg->n_members - 2)
        return fail(nullptr, MENKF_E_ARG,
                    "MENKF_GAIN_SAMPLE_EE: Y Y^T + E E^T has rank <= 2(N-1) = %d < n_probes = %d (singular)",
                    2 * cfg->n_members - 2, cfg->n_probes);
    if (cfg->time_scheme != MENKF_TIME_SSPRK3 && cfg->time_scheme != MENKF_TIME_FIRST_ORDER)
        return fail(nullptr, MENKF_E_ARG, "time_scheme must be MENKF_TIME_SSPRK3 or MENKF_TIME_FIRST_ORDER (got %d)",
                    cfg->time_scheme);
    if (cfg->time_scheme == MENKF_TIME_FIRST_ORDER && cfg->model != MENKF_BURGERS1D_INLET)
        return fail(nullptr, MENKF_E_UNSUPPORTED, "MENKF_TIME_FIRST_ORDER is built for MENKF_BURGERS1D_INLET");
    if (cfg->anomaly_terms != 0 && cfg->anomaly_terms != 1 && cfg->anomaly_terms != 3)
        return fail(nullptr, MENKF_E_ARG, "anomaly_terms must be 0, 1 or 3 (got %d)", cfg->anomaly_terms);
    if (cfg->anomaly_terms == 0) p->cfg.anomaly_terms = 3;
    p->N = cfg->n_members;
    p->Ny = cfg->n_probes;
    p->npad = roundup(p->N, 32);
    p->kdim = roundup(cfg->gain_mode == MENKF_GAIN_SAMPLE_EE ? 2 * p->N : p->N, 64);
    p->nyp = roundup(p->Ny, CHOL_NB);
    p->mext = 2 * p->N + 1;
    p->mextp = roundup(p->mext, CHOL_NB);
    p->ld = p->nyp + p->mextp;
    const bool f64 = cfg->precision == MENKF_F64;
    p->tsize = f64 ? 8 : 4;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align256(o + bytes);
        return at;
    };
    const size_t fine = (size_t)p->nf * p->F * p->tsize;
    const size_t coarse = (size_t)p->N * p->nc * p->F * p->tsize;
    p->off_info = take(256);
    p->off_f1 = take(fine);
    p->off_f2 = take(fine);
    p->off_facc = take(fine);
    p->off_c1 = take(coarse);
    p->off_c2 = take(coarse);
    p->off_cacc = take(coarse);
    p->off_yb = take((size_t)p->nyp * p->kdim * 8);
    p->off_a = take((size_t)p->ld * p->ld * 8);
    p->off_linv = take(64 * 64 * 8);
    p->off_z = take((size_t)(p->N + 1) * p->N * 8);
    p->off_zt = take((size_t)p->npad * p->npad * (f64 ? 8 : 4));
    p->off_zstar = take((size_t)p->npad * 8);
    p->npm = roundup(p->N, CHOL_NB);
    p->lds = p->npm + p->mextp;
    p->off_p = take((size_t)p->mextp * p->mextp * 8);
    p->off_as = take((size_t)p->lds * p->lds * 8);
    size_t scratch = (size_t)(p->N + 1) * p->nyp * 8;
    if (scratch < 4096 * 8) scratch = 4096 * 8;
    p->off_scratch = take(scratch);
    if (p->open) {
        p->off_trial = take(coarse);
        p->off_thf = take((size_t)p->N * 2 * 8);
    }
    p->defer_ok = cfg->gain_mode == MENKF_GAIN_EXACT_R ? 1 : 0;
    if (p->defer_ok) {
        const int nt = p->npm / CHOL_NB;
        p->gchunks = p->nyp / 32 < 64 ? p->nyp / 32 : 64;
        p->gpc = ((p->nyp + p->gchunks - 1) / p->gchunks + 31) / 32 * 32;
        p->off_mg = take((size_t)(2 * p->npm) * (2 * p->npm) * 8);
        p->off_mlinv = take(64 * 64 * 8);
        p->off_gpart = take((size_t)p->gchunks * (nt * (nt + 1) / 2) * 4096 * 8);
    }
    p->off_judge = take((size_t)2 * JUDGE_BLOCKS * 8);
    p->ws_bytes = o;
    for (int l = 0; l < 2; ++l) {
        ns_tile_shape(cfg->precision, 0, &p->sched[l].tile_x, &p->sched[l].tile_y);
        p->sched[l].member_chunk = 0;
    }
    // the coarse ensemble's whole rows fit one workgroup: march them by
    // default, two RK stages per launch where the rows divide into 32-row
    // segments, one stage per launch where they divide into 16-row ones
    for (int rows : {PAIR_ROWS, 16})
        if (ns_march_applies(*p, MENKF_COARSE, rows)) {
            p->sched[1].tile_x = 0;
            p->sched[1].tile_y = rows;
            break;
        }
    return MENKF_OK;
}

extern "C" {

menkf_status menkf_create(const menkf_config *cfg, menkf_ctx **out) {
    if (!out) return fail(nullptr, MENKF_E_ARG, "out is NULL");
    *out = nullptr;
    if (!cfg) return fail(nullptr, MENKF_E_ARG, "cfg is NULL");
    menkf_ctx *c = new (std::nothrow) menkf_ctx();
    if (!c) return fail(nullptr, MENKF_E_ARG, "out of host memory");
    const menkf_status st = build_plan(cfg, &c->plan);
    if (st != MENKF_OK) {
        delete c;
        return st;
    }
    *out = c;
    return MENKF_OK;
}

void menkf_destroy(menkf_ctx *ctx) { delete ctx; }

const char *menkf_last_error(const menkf_ctx *ctx) { return ctx ? ctx->err : g_err; }

menkf_status menkf_workspace_size(const menkf_ctx *ctx, size_t *bytes) {
    if (!ctx || !bytes) return fail(nullptr, MENKF_E_ARG, "null argument");
    *bytes = ctx->plan.ws_bytes;
    return MENKF_OK;
}

menkf_status menkf_set_workspace(menkf_ctx *ctx, void *ws, size_t bytes) {
    if (!ctx) return fail(nullptr, MENKF_E_ARG, "ctx is NULL");
    if (!ws) return fail(ctx, MENKF_E_ARG, "workspace pointer is NULL");
    if (((uintptr_t)ws) & 255) return fail(ctx, MENKF_E_ARG, "workspace must be 256-byte aligned");
    if (bytes < ctx->plan.ws_bytes)
        return fail(ctx, MENKF_E_WORKSPACE, "workspace of %zu bytes is smaller than the %zu required", bytes,
                    ctx->plan.ws_bytes);
    ctx->ws = ws;
    ctx->ws_bytes = bytes;
    hipError_t e = hipSuccess;
    if (!ctx->ev_fork) e = hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming);
    if (e == hipSuccess && !ctx->ev_join) e = hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming);
    if (e == hipSuccess && !ctx->ev_front) e = hipEventCreateWithFlags(&ctx->ev_front, hipEventDisableTiming);
    int dev = 0, ncu = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess && ncu > 0) ctx->n_cus = ncu;
    if (e == hipSuccess) e = launch_set_word((int32_t *)((char *)ws + ctx->plan.off_info), 0, nullptr);
    if (e == hipSuccess) e = launch_set_word64((uint64_t *)((char *)ws + ctx->plan.off_info + 64), 1, nullptr);
    if (e == hipSuccess) e = launch_zero_words((int32_t *)((char *)ws + ctx->plan.off_info + JUDGE_WORDS), JW_N, nullptr);
    if (e == hipSuccess) e = launch_zero_words((int32_t *)((char *)ws + ctx->plan.off_info + PIPE_WORDS), PW_N, nullptr);
    if (e != hipSuccess) return hip_fail(ctx, e, "menkf_set_workspace");
    return MENKF_OK;
}

menkf_status menkf_set_probes(menkf_ctx *ctx, const int32_t *idx, const int32_t *comp) {
    if (!ctx) return fail(nullptr, MENKF_E_ARG, "ctx is NULL");
    if (!idx || !comp) return fail(ctx, MENKF_E_ARG, "probe tables must be non-NULL device pointers");
    // One-time host-side validation (set-up call, synchronous): every probe
    // must address a fine node and a valid component.
    const Plan &p = ctx->plan;
    std::vector<int32_t> hi(p.Ny), hc(p.Ny);
    hipError_t e = hipMemcpy(hi.data(), idx, sizeof(int32_t) * p.Ny, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(hc.data(), comp, sizeof(int32_t) * p.Ny, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "menkf_set_probes");
    for (int k = 0; k < p.Ny; ++k) {
        if (hi[k] < 0 || (long long)hi[k] >= p.nf)
            return fail(ctx, MENKF_E_ARG, "probe %d: node %d outside the fine grid of %lld nodes", k, hi[k], p.nf);
        if (hc[k] < 0 || hc[k] > (p.dim == 2 ? 1 : 0))
            return fail(ctx, MENKF_E_ARG, "probe %d: component %d invalid", k, hc[k]);
    }
    ctx->idx = idx;
    ctx->comp = comp;
    return MENKF_OK;
}

menkf_status menkf_set_observations(menkf_ctx *ctx, const int32_t *idx, const int32_t *comp) {
    return menkf_set_probes(ctx, idx, comp);
}

#define NEED_WS(ctx)                                                                         \
    do {                                                                                     \
        if (!(ctx)) return fail(nullptr, MENKF_E_ARG, "ctx is NULL");                        \
        if (!(ctx)->ws) return fail((ctx), MENKF_E_WORKSPACE, "no workspace attached");      \
    } while (0)

menkf_status menkf_forecast(menkf_ctx *ctx, int32_t level, void *state, int32_t nb, int32_t nsteps, void *prev,
                            menkf_stream stream) {
    NEED_WS(ctx);
    const Plan &p = ctx->plan;
    if (level != MENKF_FINE && level != MENKF_COARSE) return fail(ctx, MENKF_E_ARG, "bad level %d", level);
    if (!state) return fail(ctx, MENKF_E_ARG, "state is NULL");
    if (nsteps < 1) return fail(ctx, MENKF_E_ARG, "nsteps must be >= 1 (got %d)", nsteps);
    if (level == MENKF_FINE && nb != 1) return fail(ctx, MENKF_E_ARG, "the fine level takes nb = 1 (got %d)", nb);
    if (level == MENKF_COARSE && (nb < 1 || nb > p.N))
        return fail(ctx, MENKF_E_ARG, "coarse nb must be in [1, %d] (got %d)", p.N, nb);
    if (p.open) return fail(ctx, MENKF_E_ARG, "the inlet-forced models' forecasts need parameters: menkf_forecast_inlet");
    const hipError_t e = p.dim == 1 ? launch_burgers_forecast(p, level, state, nb, nsteps, prev, ctx->ws, (hipStream_t)stream)
                                    : launch_ns_forecast(p, level, state, nb, nsteps, prev, ctx->ws, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_forecast");
}

static menkf_status check_schedule(menkf_ctx *ctx, int level, const menkf_schedule *sc) {
    if (level != MENKF_FINE && level != MENKF_COARSE) return fail(ctx, MENKF_E_ARG, "bad level %d", level);
    if (!sc) return fail(ctx, MENKF_E_ARG, "schedule is NULL");
    if (sc->member_chunk < 0) return fail(ctx, MENKF_E_ARG, "member_chunk must be >= 0 (got %d)", sc->member_chunk);
    if (ns_tile_index(ctx->plan.cfg.precision, sc->tile_x, sc->tile_y) < 0)
        return fail(ctx, MENKF_E_ARG, "tile %dx%d is not in the tile list of this precision", sc->tile_x, sc->tile_y);
    return MENKF_OK;
}

menkf_status menkf_set_schedule(menkf_ctx *ctx, int32_t level, const menkf_schedule *sched) {
    if (!ctx) return fail(nullptr, MENKF_E_ARG, "ctx is NULL");
    const menkf_status st = check_schedule(ctx, level, sched);
    if (st != MENKF_OK) return st;
    menkf_schedule sc = *sched;
    if (sc.tile_x == 0 && sc.tile_y == 0) ns_tile_shape(ctx->plan.cfg.precision, 0, &sc.tile_x, &sc.tile_y);
    sc.reserved = 0;
    ctx->plan.sched[level == MENKF_FINE ? 0 : 1] = sc;
    return MENKF_OK;
}

menkf_status menkf_get_schedule(const menkf_ctx *ctx, int32_t level, menkf_schedule *sched) {
    if (!ctx || !sched) return fail(nullptr, MENKF_E_ARG, "null argument");
    if (level != MENKF_FINE && level != MENKF_COARSE) return fail(nullptr, MENKF_E_ARG, "bad level %d", level);
    *sched = ctx->plan.sched[level == MENKF_FINE ? 0 : 1];
    return MENKF_OK;
}

menkf_status menkf_autotune(menkf_ctx *ctx, int32_t level, void *scratch, int32_t nb, int32_t nsteps, int32_t reps,
                            menkf_schedule *best, float *best_ms, menkf_stream stream) {
    NEED_WS(ctx);
    if (!scratch) return fail(ctx, MENKF_E_ARG, "scratch state is NULL");
    if (reps < 1 || reps > 1000) return fail(ctx, MENKF_E_ARG, "reps must be in [1, 1000]");
    if (ctx->plan.open) return fail(ctx, MENKF_E_UNSUPPORTED, "the inlet-forced model has a single schedule");
    Plan &p = ctx->plan;
    const int li = level == MENKF_FINE ? 0 : 1;
    // candidate list
    std::vector<menkf_schedule> cand;
    const int ntiles = p.dim == 2 ? ns_tile_count(p.cfg.precision) : 1;
    std::vector<int> chunks{0};
    if (p.dim == 2 && level == MENKF_COARSE)
        for (int c = (nb + 1) / 2; c >= 1; c = (c == 1 ? 0 : (c + 1) / 2)) {
            chunks.push_back(c);
            if ((long long)c * p.nc * p.F * (long long)p.tsize < (2LL << 20)) break;   // below 2 MiB per chunk
        }
    const menkf_schedule keep = p.sched[li];
    cand.push_back(keep);
    for (int t = 0; t < ntiles; ++t)
        for (int c : chunks) {
            menkf_schedule sc{};
            ns_tile_shape(p.cfg.precision, t, &sc.tile_x, &sc.tile_y);
            if (sc.tile_x == 0 && !ns_march_applies(p, level, sc.tile_y)) continue;   // would run the default tile
            sc.member_chunk = c;
            if (sc.tile_x == keep.tile_x && sc.tile_y == keep.tile_y && sc.member_chunk == keep.member_chunk) continue;
            cand.push_back(sc);
        }
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    float tbest = 0.0f;
    int ibest = -1;
    for (size_t i = 0; i < cand.size() && e == hipSuccess; ++i) {
        p.sched[li] = cand[i];
        const menkf_status st = menkf_forecast(ctx, level, scratch, nb, nsteps, nullptr, stream);   // warm-up
        if (st != MENKF_OK) {
            p.sched[li] = keep;
            if (e0) hipEventDestroy(e0);
            if (e1) hipEventDestroy(e1);
            return st;
        }
        // best of reps individually timed forecasts (robust to interference)
        float ms = 0.0f;
        for (int r = 0; r < reps && e == hipSuccess; ++r) {
            e = hipEventRecord(e0, s);
            if (e == hipSuccess && menkf_forecast(ctx, level, scratch, nb, nsteps, nullptr, stream) != MENKF_OK)
                e = hipErrorUnknown;
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float t = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
            if (e == hipSuccess && (r == 0 || t < ms)) ms = t;
        }
        // the first candidate is the level's current schedule; another one
        // must beat the best so far by 3 % (timing noise is about 1-2 %)
        if (e == hipSuccess && (ibest < 0 || ms < tbest * (ibest == 0 ? 0.97f : 1.0f))) {
            tbest = ms;
            ibest = (int)i;
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (e != hipSuccess || ibest < 0) {
        p.sched[li] = keep;
        return hip_fail(ctx, e == hipSuccess ? hipErrorUnknown : e, "menkf_autotune");
    }
    p.sched[li] = cand[ibest];
    p.tuned_ms[li] = tbest;
    p.tuned_nsteps[li] = nsteps;
    if (best) *best = cand[ibest];
    if (best_ms) *best_ms = tbest;
    return MENKF_OK;
}

menkf_status menkf_restrict(menkf_ctx *ctx, const void *xf, void *xc, menkf_stream stream) {
    if (!ctx) return fail(nullptr, MENKF_E_ARG, "ctx is NULL");
    if (!xf || !xc) return fail(ctx, MENKF_E_ARG, "null state pointer");
    const hipError_t e = launch_restrict(ctx->plan, xf, xc, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_restrict");
}

menkf_status menkf_gain(menkf_ctx *ctx, const void *members, const void *xstar, const double *yobs, uint64_t seed,
                        uint64_t cycle, const double *eps, menkf_stream stream) {
    NEED_WS(ctx);
    if (!members || !xstar || !yobs) return fail(ctx, MENKF_E_ARG, "null input pointer");
    if (!ctx->idx) return fail(ctx, MENKF_E_ARG, "probes not set (menkf_set_probes)");
    const hipError_t e = launch_gain(ctx->plan, members, xstar, yobs, seed, cycle, eps, ctx->idx, ctx->comp, ctx->ws,
                                     (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_gain");
}

menkf_status menkf_set_cycle(menkf_ctx *ctx, uint64_t cycle, menkf_stream stream) {
    NEED_WS(ctx);
    const hipError_t e =
        launch_set_word64((uint64_t *)((char *)ctx->ws + ctx->plan.off_info + 64), cycle, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_set_cycle");
}

menkf_status menkf_get_gain(menkf_ctx *ctx, double *z, menkf_stream stream) {
    NEED_WS(ctx);
    if (!z) return fail(ctx, MENKF_E_ARG, "z is NULL");
    const hipError_t e = launch_get_gain(ctx->plan, z, ctx->ws, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_get_gain");
}

menkf_status menkf_update(menkf_ctx *ctx, void *members, void *dc, menkf_stream stream) {
    NEED_WS(ctx);
    if (!members || !dc) return fail(ctx, MENKF_E_ARG, "null pointer");
    const hipError_t e = launch_update(ctx->plan, members, dc, ctx->ws, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_update");
}

// MENKF_PROLONG_LEARNED_FALLBACK: the network's correction into the
// workspace copy W, the plain correction (Pi_F, n_sweeps sweeps) into the
// two other fine buffers when the judge needs it, then the selected one
// into xf.  Every kernel is launched on every call; the device words of
// the judge make the unneeded ones return at once.
static menkf_status learned_with_judge(menkf_ctx *ctx, const void *dc, void *xf, const void *xprev, int n_sweeps,
                                       double alpha, const menkf_net *net, const int32_t *info, hipStream_t s) {
    const Plan &p = ctx->plan;
    if (!(net->guard > 0.0f)) return fail(ctx, MENKF_E_ARG, "LEARNED_FALLBACK needs guard > 0");
    if (net->judge_every < 0) return fail(ctx, MENKF_E_ARG, "judge_every must be >= 0");
    if (net->judge_every > 0 && !(net->judge_tol >= 0.0f))
        return fail(ctx, MENKF_E_ARG, "judge_tol must be >= 0 when judging");
    int32_t *jw = (int32_t *)((char *)ctx->ws + p.off_info + JUDGE_WORDS);
    void *W = (char *)ctx->ws + p.off_f1;
    void *P[2] = {(char *)ctx->ws + p.off_f2, (char *)ctx->ws + p.off_facc};
    hipError_t e = launch_judge_pre(info, jw, net->judge_every, s);
    if (e == hipSuccess) e = launch_net_prolong(p, dc, xf, W, net, 1, jw + JW_SKIP_NET, jw + JW_TILES, s);
    if (e == hipSuccess) e = launch_judge_mid(info, jw, s);
    if (e == hipSuccess) e = launch_prolong_add(p, dc, xf, P[0], jw + JW_SKIP_PLAIN, s);
    int cur = 0;
    for (int k = 0; k < n_sweeps && e == hipSuccess; ++k) {
        e = launch_sweep(p, P[cur], xprev, P[1 - cur], alpha, jw + JW_SKIP_PLAIN, ctx->ws, s);
        cur = 1 - cur;
    }
    if (e == hipSuccess) e = launch_judge_decide(p, W, P[cur], xf, info, jw, net->judge_tol, net->judge_dev, ctx->ws, s);
    if (e == hipSuccess) e = launch_judge_select(p, W, P[cur], xf, info, jw, s);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_prolong_smooth (learned with judge)");
}

// The correction of menkf_prolong_smooth; every kernel returns at once when
// *info (the status word, or the skip word of a deferred correction) is
// non-zero.
static menkf_status prolong_impl(menkf_ctx *ctx, const void *dc, void *xf, const void *xprev, int32_t n_sweeps,
                                 double alpha, int32_t mode, const menkf_net *net, const int32_t *info,
                                 hipStream_t s) {
    const Plan &p = ctx->plan;
    if (!dc || !xf) return fail(ctx, MENKF_E_ARG, "null state pointer");
    if (n_sweeps < 0 || n_sweeps > 64) return fail(ctx, MENKF_E_ARG, "n_sweeps must be in [0, 64]");
    if (n_sweeps > 0 && !xprev) return fail(ctx, MENKF_E_ARG, "sweeps need x_{k-1} (xprev)");
    if (!(alpha > 0 && alpha <= 1)) return fail(ctx, MENKF_E_ARG, "alpha must be in (0, 1]");
    if (mode != MENKF_PROLONG_PLAIN && mode != MENKF_PROLONG_LEARNED && mode != MENKF_PROLONG_LEARNED_FALLBACK)
        return fail(ctx, MENKF_E_ARG, "bad prolongation mode %d", mode);
    void *W = (char *)ctx->ws + p.off_f1;
    hipError_t e;
    const void *src;
    if (mode == MENKF_PROLONG_PLAIN) {
        if (n_sweeps % 2 == 1) {
            e = launch_prolong_add(p, dc, xf, W, info, s);
            src = W;
        } else {
            e = launch_prolong_add(p, dc, xf, xf, info, s);
            src = xf;
        }
    } else {
        if (p.dim != 2) return fail(ctx, MENKF_E_UNSUPPORTED, "the learned prolongation is defined for the 2D model");
        if (p.cfg.precision != MENKF_F32) return fail(ctx, MENKF_E_UNSUPPORTED, "the learned prolongation runs in the F32 path");
        if (!net || !net->wpacked || !net->params)
            return fail(ctx, MENKF_E_ARG, "learned prolongation needs a menkf_net with packed weights and parameters");
        for (int i = 0; i < 4; ++i)
            if (!(net->out_scale[i] != 0.0f)) return fail(ctx, MENKF_E_ARG, "net out_scale must be non-zero");
        if (mode == MENKF_PROLONG_LEARNED_FALLBACK)
            return learned_with_judge(ctx, dc, xf, xprev, n_sweeps, alpha, net, info, s);
        // the network reads x^F_f with a halo: write the result to the workspace copy
        e = launch_net_prolong(p, dc, xf, W, net, 0, info, nullptr, s);
        src = W;
        n_sweeps = 0;
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "menkf_prolong_smooth");
    for (int k = 0; k < n_sweeps; ++k) {
        void *dst = (src == xf) ? W : xf;
        e = launch_sweep(p, src, xprev, dst, alpha, info, ctx->ws, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "menkf_prolong_smooth (sweep)");
        src = dst;
    }
    if (src != xf) {
        e = launch_copy(p, src, xf, info, s);
        if (e != hipSuccess) return hip_fail(ctx, e, "menkf_prolong_smooth (copy)");
    }
    return MENKF_OK;
}

menkf_status menkf_prolong_smooth(menkf_ctx *ctx, const void *dc, void *xf, const void *xprev, int32_t n_sweeps,
                                  double alpha, int32_t mode, const menkf_net *net, menkf_stream stream) {
    NEED_WS(ctx);
    const int32_t *info = (const int32_t *)((char *)ctx->ws + ctx->plan.off_info);
    return prolong_impl(ctx, dc, xf, xprev, n_sweeps, alpha, mode, net, info, (hipStream_t)stream);
}

// The correction left pending by the last pipelined cycle: the skip word
// (nothing pending, or a failed analysis) is set on s_skip when the call
// starts, so that a failure of this call's own analysis does not race with
// it; the correction follows on s (every kernel returns at once when the
// word is set).
static menkf_status pending_skip(menkf_ctx *ctx, hipStream_t s_skip) {
    const int32_t *info = (const int32_t *)((char *)ctx->ws + ctx->plan.off_info);
    int32_t *pw = (int32_t *)((char *)ctx->ws + ctx->plan.off_info + PIPE_WORDS);
    const hipError_t e = launch_pipe_skip(info, pw, s_skip);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_cycle (pending correction)");
}

static menkf_status pending_correction(menkf_ctx *ctx, const menkf_cycle_args *a, hipStream_t s) {
    const int32_t *pw = (const int32_t *)((char *)ctx->ws + ctx->plan.off_info + PIPE_WORDS);
    return prolong_impl(ctx, a->deltac, a->fine, a->fine_prev, a->n_sweeps, a->alpha, a->prolong_mode, a->net,
                        pw + PW_SKIP, s);
}

menkf_status menkf_recentre(menkf_ctx *ctx, void *members, const void *xf, menkf_stream stream) {
    NEED_WS(ctx);
    if (!members || !xf) return fail(ctx, MENKF_E_ARG, "null state pointer");
    const int32_t *info = (const int32_t *)((char *)ctx->ws + ctx->plan.off_info);
    const hipError_t e = launch_recentre(ctx->plan, members, xf, info, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_recentre");
}

menkf_status menkf_net_pack(const float *params, void *wpacked, menkf_stream stream) {
    if (!params || !wpacked) return fail(nullptr, MENKF_E_ARG, "null pointer");
    const hipError_t e = launch_net_pack(params, wpacked, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(nullptr, e, "menkf_net_pack");
}

menkf_status menkf_net_train_workspace_size(int32_t batch, int32_t crop, size_t *bytes) {
    if (!bytes || batch < 1 || batch > 1024 || crop < 1 || crop > 4096)
        return fail(nullptr, MENKF_E_ARG, "need 1 <= batch <= 1024, 1 <= crop <= 4096");
    *bytes = net_train_workspace(batch, crop);
    return MENKF_OK;
}

static menkf_status check_train(const menkf_net_train *t, bool adam, const char *who) {
    if (!t) return fail(nullptr, MENKF_E_ARG, "%s: null train descriptor", who);
    if (!t->params || !t->grad || !t->dproj || !t->xf || !t->target || !t->crops_dev || !t->loss_dev ||
        !t->workspace_dev)
        return fail(nullptr, MENKF_E_ARG, "%s: null pointer in the train descriptor", who);
    if (adam && (!t->adam_m || !t->adam_v || t->step < 1))
        return fail(nullptr, MENKF_E_ARG, "%s: Adam needs moment buffers and step >= 1", who);
    if (t->npairs < 1 || t->H < 8 || t->W < 8 || t->batch < 1 || t->crop < 1)
        return fail(nullptr, MENKF_E_ARG, "%s: bad sizes in the train descriptor", who);
    size_t need = 0;
    menkf_status st = menkf_net_train_workspace_size(t->batch, t->crop, &need);
    if (st != MENKF_OK) return st;
    if (t->workspace_bytes < need)
        return fail(nullptr, MENKF_E_WORKSPACE, "%s: train workspace of %zu bytes < %zu required", who,
                    t->workspace_bytes, need);
    return MENKF_OK;
}

menkf_status menkf_net_train_step(const menkf_net_train *t, menkf_stream stream) {
    menkf_status st = check_train(t, t && t->apply_adam, "menkf_net_train_step");
    if (st != MENKF_OK) return st;
    const hipError_t e = launch_net_train_step(t, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(nullptr, e, "menkf_net_train_step");
}

menkf_status menkf_net_forward(const menkf_net_train *t, menkf_stream stream) {
    menkf_status st = check_train(t, false, "menkf_net_forward");
    if (st != MENKF_OK) return st;
    const hipError_t e = launch_net_forward(t, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(nullptr, e, "menkf_net_forward");
}

menkf_status menkf_net_backward(const menkf_net_train *t, menkf_stream stream) {
    menkf_status st = check_train(t, false, "menkf_net_backward");
    if (st != MENKF_OK) return st;
    const hipError_t e = launch_net_backward(t, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(nullptr, e, "menkf_net_backward");
}

menkf_status menkf_net_adam(const menkf_net_train *t, menkf_stream stream) {
    menkf_status st = check_train(t, true, "menkf_net_adam");
    if (st != MENKF_OK) return st;
    const hipError_t e = launch_net_adam(t, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(nullptr, e, "menkf_net_adam");
}

menkf_status menkf_get_status(menkf_ctx *ctx, int32_t *info, int32_t clear, menkf_stream stream) {
    NEED_WS(ctx);
    if (!info) return fail(ctx, MENKF_E_ARG, "info is NULL");
    int32_t *dinfo = (int32_t *)((char *)ctx->ws + ctx->plan.off_info);
    hipError_t e = hipMemcpyAsync(info, dinfo, sizeof(int32_t), hipMemcpyDeviceToHost, (hipStream_t)stream);
    if (e == hipSuccess) e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "menkf_get_status");
    if (clear && *info != 0) {
        e = launch_set_word(dinfo, 0, (hipStream_t)stream);
        if (e != hipSuccess) return hip_fail(ctx, e, "menkf_get_status (clear)");
    }
    if (*info != 0)
        return fail(ctx, MENKF_E_NOT_SPD, "innovation covariance not positive definite at column %d", *info - 1);
    return MENKF_OK;
}

menkf_status menkf_observe(menkf_ctx *ctx, int32_t level, const void *state, int32_t nb, double *y,
                           menkf_stream stream) {
    if (!ctx) return fail(nullptr, MENKF_E_ARG, "ctx is NULL");
    if (level != MENKF_FINE && level != MENKF_COARSE) return fail(ctx, MENKF_E_ARG, "bad level %d", level);
    if (!state || !y) return fail(ctx, MENKF_E_ARG, "null pointer");
    if (nb < 1 || nb > 65535) return fail(ctx, MENKF_E_ARG, "nb must be in [1, 65535]");
    if (!ctx->idx) return fail(ctx, MENKF_E_ARG, "probes not set (menkf_set_probes)");
    const hipError_t e = launch_observe(ctx->plan, level, state, nb, y, ctx->idx, ctx->comp, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_observe");
}

menkf_status menkf_diagnostics(menkf_ctx *ctx, const void *xa, const void *xt, double *out, menkf_stream stream) {
    NEED_WS(ctx);
    if (!xa || !xt || !out) return fail(ctx, MENKF_E_ARG, "null pointer");
    const hipError_t e = launch_diagnostics(ctx->plan, xa, xt, out, ctx->ws, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_diagnostics");
}

menkf_status menkf_diagnostics_noalloc(menkf_ctx *ctx, const void *xa, const void *xt, double *out,
                                       menkf_stream stream) {
    if (!ctx) return fail(nullptr, MENKF_E_ARG, "ctx is NULL");
    if (!xa || !xt || !out) return fail(ctx, MENKF_E_ARG, "null pointer");
    const size_t need = diagnostics_noalloc_need(ctx->plan), cap = diagnostics_noalloc_capacity();
    if (need > cap)
        return fail(ctx, MENKF_E_WORKSPACE,
                    "menkf_diagnostics_noalloc: the reduction needs %zu doubles of scratch, the static array holds %zu",
                    need, cap);
    const hipError_t e = launch_diagnostics_noalloc(ctx->plan, xa, xt, out, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_diagnostics_noalloc");
}

menkf_status menkf_spread(menkf_ctx *ctx, const void *members, int32_t nb, double *out, menkf_stream stream) {
    NEED_WS(ctx);
    if (!members || !out) return fail(ctx, MENKF_E_ARG, "null pointer");
    if (nb < 2 || nb > ctx->plan.N) return fail(ctx, MENKF_E_ARG, "nb must be in [2, %d] (got %d)", ctx->plan.N, nb);
    const hipError_t e = launch_spread(ctx->plan, members, nb, out, ctx->ws, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_spread");
}

menkf_status menkf_residual(menkf_ctx *ctx, const void *x, const void *xprev, void *r, menkf_stream stream) {
    if (!ctx) return fail(nullptr, MENKF_E_ARG, "ctx is NULL");
    if (!x || !xprev || !r) return fail(ctx, MENKF_E_ARG, "null pointer");
    if (r == x || r == xprev) return fail(ctx, MENKF_E_ARG, "r must not alias x or xprev");
    if (ctx->plan.open) return fail(ctx, MENKF_E_UNSUPPORTED, "menkf_residual is defined for the periodic models");
    const hipError_t e = ctx->plan.dim == 2 ? launch_ns_resid(ctx->plan, x, xprev, r, (hipStream_t)stream)
                                            : launch_burgers_resid(ctx->plan, x, xprev, r, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_residual");
}

double menkf_ram_ratio(int32_t dim, int32_t ratio, int32_t n_members) {
    if (dim < 1 || ratio < 1 || n_members < 0) return -1.0;
    return 1.0 + (double)n_members / std::pow((double)ratio, (double)dim);
}

menkf_status menkf_forecast_inlet(menkf_ctx *ctx, int32_t level, void *state, int32_t nb, int32_t nsteps, void *prev,
                                  const double *theta, const double *t0, menkf_stream stream) {
    NEED_WS(ctx);
    const Plan &p = ctx->plan;
    if (!p.open) return fail(ctx, MENKF_E_ARG, "menkf_forecast_inlet needs an inlet-forced context");
    if (level != MENKF_FINE && level != MENKF_COARSE) return fail(ctx, MENKF_E_ARG, "bad level %d", level);
    if (!state || !theta || !t0) return fail(ctx, MENKF_E_ARG, "null pointer");
    if (nsteps < 1) return fail(ctx, MENKF_E_ARG, "nsteps must be >= 1 (got %d)", nsteps);
    if (level == MENKF_FINE && nb != 1) return fail(ctx, MENKF_E_ARG, "the fine level takes nb = 1 (got %d)", nb);
    if (level == MENKF_COARSE && (nb < 1 || nb > p.N))
        return fail(ctx, MENKF_E_ARG, "coarse nb must be in [1, %d] (got %d)", p.N, nb);
    const hipError_t e = launch_inlet_forecast(p, level, state, nb, nsteps, prev, theta, t0, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_forecast_inlet");
}

menkf_status menkf_param_perturb(menkf_ctx *ctx, const double *theta, double *theta_f, uint64_t seed, uint64_t cycle,
                                 menkf_stream stream) {
    NEED_WS(ctx);
    if (!ctx->plan.open) return fail(ctx, MENKF_E_ARG, "menkf_param_perturb needs an inlet-forced context");
    if (!theta || !theta_f) return fail(ctx, MENKF_E_ARG, "null pointer");
    const hipError_t e = launch_param_perturb(ctx->plan, theta, theta_f, seed, cycle, ctx->ws, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_param_perturb");
}

menkf_status menkf_param_update(menkf_ctx *ctx, const double *theta_f, double *theta_a, double *theta_mean,
                                menkf_stream stream) {
    NEED_WS(ctx);
    if (!ctx->plan.open) return fail(ctx, MENKF_E_ARG, "menkf_param_update needs an inlet-forced context");
    if (!theta_f || !theta_a || !theta_mean) return fail(ctx, MENKF_E_ARG, "null pointer");
    const hipError_t e = launch_param_update(ctx->plan, theta_f, theta_a, theta_mean, ctx->ws, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_param_update");
}

menkf_status menkf_dual_cycle(const menkf_dual_args *a, menkf_stream stream) {
    if (!a) return fail(nullptr, MENKF_E_ARG, "args is NULL");
    menkf_ctx *ctx = a->ctx;
    NEED_WS(ctx);
    const Plan &p = ctx->plan;
    if (!p.open) return fail(ctx, MENKF_E_ARG, "menkf_dual_cycle needs an inlet-forced context");
    if (!a->fine || !a->fine_prev || !a->members || !a->xstar || !a->deltac || !a->yobs || !a->theta ||
        !a->theta_mean || !a->clock)
        return fail(ctx, MENKF_E_ARG, "menkf_dual_cycle: null buffer");
    if (a->nsteps < 1) return fail(ctx, MENKF_E_ARG, "menkf_dual_cycle: nsteps must be >= 1");
    if (a->aux_stream && a->aux_stream == stream)
        return fail(ctx, MENKF_E_ARG, "menkf_dual_cycle: aux_stream must differ from stream");
    if (!ctx->idx) return fail(ctx, MENKF_E_ARG, "probes not set (menkf_set_probes)");
    hipStream_t s = (hipStream_t)stream;
    hipStream_t aux = (hipStream_t)a->aux_stream;
    char *w = (char *)ctx->ws;
    void *trial = w + p.off_trial;
    double *thf = (double *)(w + p.off_thf);
    // parameter filter: theta_f and the trial members, their forecast and
    // gain (any x* will do: only Z[:, :N] is used, so the first member
    // serves), then theta_a and its mean
    hipError_t e = launch_dual_prep(p, a->members, trial, a->theta, thf, a->seed, a->cycle, ctx->ws, s);
    if (e == hipSuccess) e = launch_inlet_forecast(p, MENKF_COARSE, trial, p.N, a->nsteps, nullptr, thf, a->clock, s);
    if (e == hipSuccess)
        e = launch_gain(p, trial, a->members, a->yobs, a->seed, a->cycle, nullptr, ctx->idx, ctx->comp, ctx->ws, s,
                        false);
    if (e == hipSuccess) e = launch_param_update(p, thf, a->theta, a->theta_mean, ctx->ws, s);
    // state filter: members with theta_a, the fine run with its mean (on
    // the second stream if given: one workgroup beside the members')
    if (e != hipSuccess) return hip_fail(ctx, e, "menkf_dual_cycle");
    if (aux) {
        e = hipEventRecord(ctx->ev_fork, s);
        if (e == hipSuccess) e = hipStreamWaitEvent(aux, ctx->ev_fork, 0);
        if (e != hipSuccess) return hip_fail(ctx, e, "menkf_dual_cycle (fork)");
    }
    hipError_t ef = launch_inlet_forecast(p, MENKF_FINE, a->fine, 1, a->nsteps, a->fine_prev, a->theta_mean, a->clock,
                                          aux ? aux : s);
    e = launch_inlet_forecast(p, MENKF_COARSE, a->members, p.N, a->nsteps, nullptr, a->theta, a->clock, s);
    if (aux) {
        // join also after a failed issue, so that a capture stays well formed
        hipError_t ej = hipEventRecord(ctx->ev_join, aux);
        if (ej == hipSuccess) ej = hipStreamWaitEvent(s, ctx->ev_join, 0);
        if (ej != hipSuccess) return hip_fail(ctx, ej, "menkf_dual_cycle (join)");
    }
    if (ef != hipSuccess) return hip_fail(ctx, ef, "menkf_dual_cycle (fine forecast)");
    if (e != hipSuccess) return hip_fail(ctx, e, "menkf_dual_cycle");
    menkf_status st = menkf_restrict(ctx, a->fine, a->xstar, stream);
    if (st == MENKF_OK) st = menkf_gain(ctx, a->members, a->xstar, a->yobs, a->seed, a->cycle, nullptr, stream);
    if (st == MENKF_OK) st = menkf_update(ctx, a->members, a->deltac, stream);
    if (st == MENKF_OK)
        st = menkf_prolong_smooth(ctx, a->deltac, a->fine, a->fine_prev, a->n_sweeps, a->alpha, MENKF_PROLONG_PLAIN,
                                  nullptr, stream);
    if (st != MENKF_OK) return st;
    e = launch_clock_advance(a->clock, (double)a->nsteps * p.cfg.dt, s);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_dual_cycle (clock)");
}

menkf_status menkf_cycle(const menkf_cycle_args *a, menkf_stream stream) {
    if (!a) return fail(nullptr, MENKF_E_ARG, "args is NULL");
    menkf_ctx *ctx = a->ctx;
    NEED_WS(ctx);
    const Plan &p = ctx->plan;
    if (!a->fine || !a->fine_prev || !a->members || !a->xstar || !a->deltac || !a->yobs)
        return fail(ctx, MENKF_E_ARG, "menkf_cycle: null buffer");
    if (a->nsteps < 1) return fail(ctx, MENKF_E_ARG, "menkf_cycle: nsteps must be >= 1");
    if (a->feedback != 0 && a->feedback != 1) return fail(ctx, MENKF_E_ARG, "menkf_cycle: feedback must be 0 or 1");
    if (a->pipelined != 0 && a->pipelined != 1) return fail(ctx, MENKF_E_ARG, "menkf_cycle: pipelined must be 0 or 1");
    if (a->pipelined && a->feedback)
        return fail(ctx, MENKF_E_ARG, "menkf_cycle: a pipelined cycle cannot recentre on the fine analysis");
    if (!ctx->idx) return fail(ctx, MENKF_E_ARG, "probes not set (menkf_set_probes)");
    menkf_status st;
    const bool aux = a->aux_stream && a->aux_stream != stream;
    if (a->pipelined) {
        st = pending_skip(ctx, (hipStream_t)stream);
        if (st == MENKF_OK && !aux) st = pending_correction(ctx, a, (hipStream_t)stream);
        if (st != MENKF_OK) return st;
    }
    if (aux && p.defer_ok) {
        // The fine forecast, x* and the small system of the x* column run on
        // the second stream while the N_y x N_y factorisation (with d* = 0)
        // runs on the first; z* follows once both are done.
        hipStream_t s0 = (hipStream_t)stream, s1 = (hipStream_t)a->aux_stream;
        st = menkf_forecast(ctx, MENKF_COARSE, a->members, p.N, a->nsteps, nullptr, stream);
        if (st != MENKF_OK) return st;
        hipError_t e = launch_gain_deferred_front(p, a->members, a->yobs, a->seed, a->cycle, ctx->idx, ctx->comp,
                                                  ctx->ws, s0);
        if (e != hipSuccess) return hip_fail(ctx, e, "menkf_cycle (gain)");
        // The small system of the x* column needs only the anomalies: it is
        // forked right after the front end and runs beside the first block
        // steps of the factorisation.
        if ((e = hipEventRecord(ctx->ev_front, s0)) == hipSuccess) e = hipStreamWaitEvent(s1, ctx->ev_front, 0);
        if (e != hipSuccess) return hip_fail(ctx, e, "menkf_cycle (fork)");
        hipError_t e1 = launch_xstar_factor(p, ctx->ws, s1);
        // a pipelined cycle applies the previous cycle's correction here,
        // beside the early block steps and off the member chain
        st = a->pipelined ? pending_correction(ctx, a, s1) : MENKF_OK;
        // The factorisation is issued next and records the second fork
        // event once its remaining trailing updates fit about three
        // workgroups per compute unit: the early block steps, bound by the
        // throughput of their updates, run without the fine forecast, which
        // then fills the GPU beside the later ones, bound by the latency of
        // the diagonal factorisations.
        hipError_t e0 = launch_gain_deferred_back(p, a->cycle, ctx->ws, s0, ctx->ev_fork, 4 * ctx->n_cus);
        if (e0 != hipSuccess) (void)hipEventRecord(ctx->ev_fork, s0);   // keep the fork well formed
        e = hipStreamWaitEvent(s1, ctx->ev_fork, 0);
        if (e != hipSuccess) return hip_fail(ctx, e, "menkf_cycle (fork)");
        if (st == MENKF_OK) st = menkf_forecast(ctx, MENKF_FINE, a->fine, 1, a->nsteps, a->fine_prev, a->aux_stream);
        if (st == MENKF_OK) st = menkf_restrict(ctx, a->fine, a->xstar, a->aux_stream);
        // join also after a failed issue, so that a capture stays well formed
        e = hipEventRecord(ctx->ev_join, s1);
        if (e == hipSuccess) e = hipStreamWaitEvent(s0, ctx->ev_join, 0);
        if (st != MENKF_OK) return st;
        if (e1 != hipSuccess) return hip_fail(ctx, e1, "menkf_cycle (x* system)");
        if (e0 != hipSuccess) return hip_fail(ctx, e0, "menkf_cycle (gain)");
        if (e != hipSuccess) return hip_fail(ctx, e, "menkf_cycle (join)");
        e = launch_xstar_gain(p, a->xstar, a->yobs, ctx->idx, ctx->comp, ctx->ws, s0);
        if (e != hipSuccess) return hip_fail(ctx, e, "menkf_cycle (x* column)");
    } else if (aux) {
        hipStream_t s0 = (hipStream_t)stream, s1 = (hipStream_t)a->aux_stream;
        hipError_t e = hipEventRecord(ctx->ev_fork, s0);
        if (e == hipSuccess) e = hipStreamWaitEvent(s1, ctx->ev_fork, 0);
        if (e != hipSuccess) return hip_fail(ctx, e, "menkf_cycle (fork)");
        st = a->pipelined ? pending_correction(ctx, a, s1) : MENKF_OK;
        if (st == MENKF_OK) st = menkf_forecast(ctx, MENKF_FINE, a->fine, 1, a->nsteps, a->fine_prev, a->aux_stream);
        if (st == MENKF_OK) st = menkf_forecast(ctx, MENKF_COARSE, a->members, p.N, a->nsteps, nullptr, stream);
        // join also after a failed issue, so that a capture stays well formed
        e = hipEventRecord(ctx->ev_join, s1);
        if (e == hipSuccess) e = hipStreamWaitEvent(s0, ctx->ev_join, 0);
        if (st != MENKF_OK) return st;
        if (e != hipSuccess) return hip_fail(ctx, e, "menkf_cycle (join)");
        st = menkf_restrict(ctx, a->fine, a->xstar, stream);
        if (st == MENKF_OK) st = menkf_gain(ctx, a->members, a->xstar, a->yobs, a->seed, a->cycle, nullptr, stream);
    } else {
        st = menkf_forecast(ctx, MENKF_FINE, a->fine, 1, a->nsteps, a->fine_prev, stream);
        if (st == MENKF_OK) st = menkf_forecast(ctx, MENKF_COARSE, a->members, p.N, a->nsteps, nullptr, stream);
        if (st == MENKF_OK) st = menkf_restrict(ctx, a->fine, a->xstar, stream);
        if (st == MENKF_OK) st = menkf_gain(ctx, a->members, a->xstar, a->yobs, a->seed, a->cycle, nullptr, stream);
    }
    if (st == MENKF_OK) st = menkf_update(ctx, a->members, a->deltac, stream);
    if (st == MENKF_OK && a->pipelined) {
        // the correction is left pending for the next call (or the flush)
        const hipError_t e = launch_set_word((int32_t *)((char *)ctx->ws + p.off_info + PIPE_WORDS) + PW_PEND, 1,
                                             (hipStream_t)stream);
        return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_cycle (pending word)");
    }
    if (st == MENKF_OK)
        st = menkf_prolong_smooth(ctx, a->deltac, a->fine, a->fine_prev, a->n_sweeps, a->alpha, a->prolong_mode,
                                  a->net, stream);
    if (st == MENKF_OK && a->feedback) st = menkf_recentre(ctx, a->members, a->fine, stream);
    return st;
}

menkf_status menkf_cycle_flush(const menkf_cycle_args *a, menkf_stream stream) {
    if (!a) return fail(nullptr, MENKF_E_ARG, "args is NULL");
    menkf_ctx *ctx = a->ctx;
    NEED_WS(ctx);
    if (!a->fine || !a->fine_prev || !a->deltac) return fail(ctx, MENKF_E_ARG, "menkf_cycle_flush: null buffer");
    menkf_status st = pending_skip(ctx, (hipStream_t)stream);
    if (st == MENKF_OK) st = pending_correction(ctx, a, (hipStream_t)stream);
    if (st != MENKF_OK) return st;
    const hipError_t e = launch_set_word((int32_t *)((char *)ctx->ws + ctx->plan.off_info + PIPE_WORDS) + PW_PEND, 0,
                                         (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(ctx, e, "menkf_cycle_flush");
}

// Estimated device time (us) of one cycle of an instance, for the lane
// assignment: autotuned forecast times when known, otherwise a per-point
// stencil cost; plus the latency-bound chain of Cholesky block steps.
static double cycle_cost(const menkf_cycle_args &a) {
    const Plan &p = a.ctx->plan;
    const double per_point_stage = 1.6e-5;   // us per grid point and RK stage (FP32, 2D)
    const int stages = p.dim == 2 ? 4 : 3;
    double t = 0.0;
    const double pts[2] = {(double)p.nf, (double)p.N * (double)p.nc};
    for (int l = 0; l < 2; ++l)
        t += p.tuned_ms[l] > 0 ? 1e3 * p.tuned_ms[l] * a.nsteps / p.tuned_nsteps[l]
                               : per_point_stage * stages * a.nsteps * pts[l];
    t += 60.0 * (p.nyp / CHOL_NB);
    t += 5e-5 * (double)p.nf * (1 + a.n_sweeps);
    return t;
}

menkf_status menkf_batch_create(int32_t n_lanes, menkf_batch **out) {
    if (!out) return fail(nullptr, MENKF_E_ARG, "out is NULL");
    *out = nullptr;
    if (n_lanes < 1 || n_lanes > 16) return fail(nullptr, MENKF_E_ARG, "n_lanes must be in [1, 16] (got %d)", n_lanes);
    menkf_batch *b = new (std::nothrow) menkf_batch();
    if (!b) return fail(nullptr, MENKF_E_ARG, "out of host memory");
    hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int i = 0; i < n_lanes && e == hipSuccess; ++i) {
        hipStream_t s = nullptr;
        hipEvent_t ev = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) b->lanes.push_back(s);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) b->join.push_back(ev);
    }
    if (e != hipSuccess) {
        menkf_batch_destroy(b);
        return hip_fail(nullptr, e, "menkf_batch_create");
    }
    *out = b;
    return MENKF_OK;
}

void menkf_batch_destroy(menkf_batch *b) {
    if (!b) return;
    for (hipEvent_t ev : b->join) hipEventDestroy(ev);
    for (hipStream_t s : b->lanes) hipStreamDestroy(s);
    if (b->fork) hipEventDestroy(b->fork);
    delete b;
}

menkf_status menkf_batch_cycle(menkf_batch *b, const menkf_cycle_args *inst, int32_t n, menkf_stream stream) {
    if (!b || !inst) return fail(nullptr, MENKF_E_ARG, "null argument");
    if (n < 1) return fail(nullptr, MENKF_E_ARG, "n must be >= 1 (got %d)", n);
    for (int i = 0; i < n; ++i) {
        if (!inst[i].ctx || !inst[i].ctx->ws) return fail(nullptr, MENKF_E_ARG, "instance %d: no context or workspace", i);
        for (int j = 0; j < i; ++j)
            if (inst[j].ctx == inst[i].ctx) return fail(nullptr, MENKF_E_ARG, "instances %d and %d share a context", j, i);
    }
    // longest-processing-time-first assignment to the least loaded lane
    const int L = (int)b->lanes.size();
    std::vector<double> cost(n), load(L, 0.0);
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) {
        cost[i] = cycle_cost(inst[i]);
        order[i] = i;
    }
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    b->lane_of.assign(n, 0);
    std::vector<std::vector<int>> per_lane(L);
    for (int i : order) {
        int l = 0;
        for (int k = 1; k < L; ++k)
            if (load[k] < load[l]) l = k;
        load[l] += cost[i];
        b->lane_of[i] = l;
        per_lane[l].push_back(i);
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipEventRecord(b->fork, s);
    for (int l = 0; l < L && e == hipSuccess; ++l) e = hipStreamWaitEvent(b->lanes[l], b->fork, 0);
    if (e != hipSuccess) return hip_fail(nullptr, e, "menkf_batch_cycle (fork)");
    menkf_status st = MENKF_OK;
    for (int l = 0; l < L && st == MENKF_OK; ++l)
        for (int i : per_lane[l]) {
            st = menkf_cycle(&inst[i], b->lanes[l]);
            if (st != MENKF_OK) {
                fail(nullptr, st, "instance %d: %s", i, inst[i].ctx->err);
                break;
            }
        }
    // join every lane, also after a failed issue, so a capture stays well formed
    for (int l = 0; l < L && e == hipSuccess; ++l) {
        e = hipEventRecord(b->join[l], b->lanes[l]);
        if (e == hipSuccess) e = hipStreamWaitEvent(s, b->join[l], 0);
    }
    if (st != MENKF_OK) return st;
    return e == hipSuccess ? MENKF_OK : hip_fail(nullptr, e, "menkf_batch_cycle (join)");
}

menkf_status menkf_batch_lanes(const menkf_batch *b, int32_t *lane_of, int32_t n) {
    if (!b || !lane_of) return fail(nullptr, MENKF_E_ARG, "null argument");
    if (n != (int)b->lane_of.size()) return fail(nullptr, MENKF_E_ARG, "n = %d, last batch had %zu instances", n, b->lane_of.size());
    for (int i = 0; i < n; ++i) lane_of[i] = b->lane_of[i];
    return MENKF_OK;
}

menkf_status menkf_graph_begin(menkf_stream stream) {
    if (!stream) return fail(nullptr, MENKF_E_ARG, "graph capture needs a non-default stream");
    const hipError_t e = hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeRelaxed);
    return e == hipSuccess ? MENKF_OK : hip_fail(nullptr, e, "menkf_graph_begin");
}

menkf_status menkf_graph_end(menkf_stream stream, menkf_graph **out) {
    if (!out) return fail(nullptr, MENKF_E_ARG, "out is NULL");
    *out = nullptr;
    menkf_graph *g = new (std::nothrow) menkf_graph();
    if (!g) return fail(nullptr, MENKF_E_ARG, "out of host memory");
    hipError_t e = hipStreamEndCapture((hipStream_t)stream, &g->graph);
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (g->graph) hipGraphDestroy(g->graph);
        delete g;
        return hip_fail(nullptr, e, "menkf_graph_end");
    }
    *out = g;
    return MENKF_OK;
}

menkf_status menkf_graph_launch(menkf_graph *g, menkf_stream stream) {
    if (!g) return fail(nullptr, MENKF_E_ARG, "graph is NULL");
    const hipError_t e = hipGraphLaunch(g->exec, (hipStream_t)stream);
    return e == hipSuccess ? MENKF_OK : hip_fail(nullptr, e, "menkf_graph_launch");
}

void menkf_graph_destroy(menkf_graph *g) {
    if (!g) return;
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
