// Time integration of the Landau-Lifshitz equation (paper Sec. 2.1) with an
// explicit Runge-Kutta (4,5) pair, adaptive per state (Sec. 3.1), or with
// the classical fourth-order scheme at a fixed step.
//
// Every stage is one launch of the fused field kernel: it evaluates the
// right-hand side at the stage input and writes the next stage input (or the
// RK4 update, or the float64 Dormand-Prince error estimate).  A small
// control kernel then decides acceptance and the next step per state, and
// (DP45) a commit pass applies the accepted step, restores |m| = 1 and forms
// the next attempt's first stage input.  Nothing returns to the host between
// attempts; runs of 1, 2, 4, 8 and kGraphSteps attempts are captured in
// hipGraphs and a run of c attempts replays them by the binary digits of c.  States of a batch never couple: each has its own field,
// time, step size and flags, and finished or failed states are frozen.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "common.h"

namespace tmag {
namespace {

// Dormand-Prince 5(4) stage weights a_sj (first-same-as-last: the last row
// is the fifth-order solution).
constexpr double kDpA[7][6] = {
    {0, 0, 0, 0, 0, 0},
    {1.0 / 5, 0, 0, 0, 0, 0},
    {3.0 / 40, 9.0 / 40, 0, 0, 0, 0},
    {44.0 / 45, -56.0 / 15, 32.0 / 9, 0, 0, 0},
    {19372.0 / 6561, -25360.0 / 2187, 64448.0 / 6561, -212.0 / 729, 0, 0},
    {9017.0 / 3168, -355.0 / 33, 46732.0 / 5247, 49.0 / 176, -5103.0 / 18656, 0},
    {35.0 / 384, 0, 500.0 / 1113, 125.0 / 192, -2187.0 / 6784, 11.0 / 84}};

// Run parameters passed by value to the prologue (RunParam order).
struct RunParams {
    double v[RP_COUNT];
};

// Prologue of tm_run, one launch: thread i packs element i of the caller's
// states into the padded state y (zeros in the padding); threads i < B also
// reset the control of state i, i < 3B copy the applied fields (zero when
// none), i < RP_COUNT store the run parameters the step kernels read.
__global__ void k_begin_run(const float* __restrict__ m, int64_t n, int64_t np, int64_t B,
                            float* __restrict__ y, const float* __restrict__ Ha_in, float* __restrict__ Ha,
                            RunParams rp, double* __restrict__ prm, const double* __restrict__ t_in,
                            const double* __restrict__ dt_in, double* __restrict__ t,
                            double* __restrict__ h, double* __restrict__ dt, int64_t* __restrict__ steps,
                            int64_t* __restrict__ rejected, int32_t* __restrict__ flags,
                            int32_t* __restrict__ acc) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < B * np * 3) {
        const int64_t s = i / (3 * np), r = i % (3 * np);
        y[i] = r < 3 * n ? m[s * 3 * n + r] : 0.0f;
    }
    if (i < RP_COUNT) prm[i] = rp.v[i];
    if (i < 3 * B) Ha[i] = Ha_in ? Ha_in[i] : 0.0f;
    if (i < B) {
        const double t0 = t_in[i], d0 = dt_in[i], t_end = rp.v[RP_TEND];
        t[i] = t0;
        dt[i] = d0;
        double hh = d0;
        int32_t f = 0;
        if (t_end > 0.0 && t0 + hh > t_end) hh = t_end - t0;
        if (rp.v[RP_MAX_STEPS] <= 0.0 || (t_end > 0.0 && t0 >= t_end)) f = FLAG_DONE;
        h[i] = f ? 0.0 : hh;
        flags[i] = f;
        steps[i] = 0;
        rejected[i] = 0;
        acc[i] = 0;
    }
}

// Epilogue of tm_run, one launch: thread i unpacks element i of the final
// states into the caller's array; threads i < B also hand back t, dt and the
// accepted steps of state i and gather its counts and flags into stat
// ([3][B]: accepted, rejected, flags) for one copy to the host.
__global__ void k_end_run(const float* __restrict__ y, int64_t n, int64_t np, int64_t B, float* __restrict__ m,
                          const double* __restrict__ t, const double* __restrict__ dt,
                          const int64_t* __restrict__ steps, const int64_t* __restrict__ rejected,
                          const int32_t* __restrict__ flags, double* __restrict__ t_out,
                          double* __restrict__ dt_out, int64_t* __restrict__ steps_out,
                          int64_t* __restrict__ stat) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < B * n * 3) {
        const int64_t s = i / (3 * n), r = i % (3 * n);
        m[i] = y[s * 3 * np + r];
    }
    if (i < B) {
        t_out[i] = t[i];
        dt_out[i] = dt[i];
        if (steps_out) steps_out[i] = steps[i];
        stat[i] = steps[i];
        stat[B + i] = rejected[i];
        stat[2 * B + i] = flags[i];
    }
}

EpiArgs stage_args(Workspace* w, float* kout, const float* const* kprev, int nprev,
                   const double* coef, float* ynext) {
    EpiArgs e{};
    e.out = kout;
    e.out_stride = 0;
    e.Ha = w->Ha;
    e.y = w->y;
    for (int j = 0; j < nprev; ++j) e.kprev[j] = kprev[j];
    for (int j = 0; j <= nprev; ++j) e.coef[j] = static_cast<float>(coef[j]);
    e.nprev = nprev;
    e.ynext = ynext;
    e.h = w->h;
    e.params = w->params;
    e.errp = w->errp;
    e.dmxp = w->dmxp;
    e.pstride = w->pstride;
    e.t = w->t;
    e.dt = w->dt;
    e.steps = w->steps;
    e.rejected = w->rejected;
    e.flags = w->flags;
    e.snap = w->snap;
    return e;
}

// DP45 first stage: k1 = f(y), stage-2 input y + h a21 k1.
tm_status dp_first(const Problem* p, Workspace* w, int64_t B, hipStream_t s) {
    const double c[1] = {kDpA[1][0]};
    EpiArgs e = stage_args(w, w->k[0], nullptr, 0, c, w->ya);
    return launch_field(p, Epi::STAGE, B, w->y, e, s);
}

// One attempted DP45 step: stages 2..7, control, commit.
tm_status dp_attempt(const Problem* p, Workspace* w, int64_t B, hipStream_t s) {
    float* in[7] = {nullptr, w->ya, w->yb, w->ya, w->yb, w->ya, w->y5};
    float* nxt[7] = {nullptr, w->yb, w->ya, w->yb, w->ya, w->y5, nullptr};
    const float* kp[6] = {w->k[0], w->k[1], w->k[2], w->k[3], w->k[4], w->k[5]};
    for (int st = 1; st < 6; ++st) {  // stages 2..6 (0-based st)
        double c[7];
        for (int j = 0; j <= st; ++j) c[j] = kDpA[st + 1][j];
        EpiArgs e = stage_args(w, w->k[st], kp, st, c, nxt[st]);
        w->frag_chain = st >= 2;  // stage 2 reads the committed attempt's input
        tm_status r = launch_field(p, Epi::STAGE, B, in[st], e, s);
        if (r != TM_OK) return r;
    }
    const double none[7] = {0, 0, 0, 0, 0, 0, 0};
    EpiArgs e = stage_args(w, w->k[6], kp, 6, none, nullptr);
    w->frag_chain = true;
    tm_status r = launch_field(p, Epi::DP_LAST, B, w->y5, e, s);
    if (r != TM_OK) return r;
    return launch_commit(p, w, B, s);  // step control fused into the commit pass
}

// RK4 control values: the workspace's own (t, h, steps, flags) or its
// second set.
struct RkCtl {
    double* t;
    double* h;
    int64_t* steps;
    int32_t* flags;
};
RkCtl rk_set(Workspace* w, int which) {
    return which == 0 ? RkCtl{w->t, w->h, w->steps, w->flags} : RkCtl{w->t1, w->h1, w->steps1, w->flags1};
}

// One classical RK4 step whose stages read the control values `in`.  With
// `out` the last stage also advances the control into `out` (no launch of
// its own); else the control pass advances `in` in place.
tm_status rk4_attempt(const Problem* p, Workspace* w, int64_t B, int renorm, const RkCtl& in, const RkCtl* out,
                      hipStream_t s) {
    const float* kp[3] = {w->k[0], w->k[1], w->k[2]};
    const double half[1] = {0.5}, one[1] = {1.0};
    auto with_ctl = [&](EpiArgs e) {
        e.h = in.h;
        e.t = in.t;
        e.steps = in.steps;
        e.flags = in.flags;
        return e;
    };
    tm_status r;
    EpiArgs e1 = with_ctl(stage_args(w, w->k[0], nullptr, 0, half, w->ya));
    w->frag_chain = false;
    if ((r = launch_field(p, Epi::STAGE, B, w->y, e1, s)) != TM_OK) return r;
    EpiArgs e2 = with_ctl(stage_args(w, w->k[1], nullptr, 0, half, w->yb));
    w->frag_chain = true;  // stages 2, 3 and 4 read the previous stage's output
    if ((r = launch_field(p, Epi::STAGE, B, w->ya, e2, s)) != TM_OK) return r;
    EpiArgs e3 = with_ctl(stage_args(w, w->k[2], nullptr, 0, one, w->ya));
    w->frag_chain = true;
    if ((r = launch_field(p, Epi::STAGE, B, w->yb, e3, s)) != TM_OK) return r;
    const double fin[4] = {1.0 / 6, 2.0 / 6, 2.0 / 6, 1.0 / 6};
    EpiArgs e4 = with_ctl(stage_args(w, nullptr, kp, 3, fin, nullptr));
    e4.y_mut = w->y;
    e4.renorm = renorm;
    if (out) {
        e4.rk_t_out = out->t;
        e4.rk_h_out = out->h;
        e4.rk_steps_out = out->steps;
        e4.rk_flags_out = out->flags;
    }
    w->frag_chain = true;
    if ((r = launch_field(p, Epi::RK4_FINAL, B, w->ya, e4, s)) != TM_OK) return r;
    return out ? TM_OK : launch_control(w, B, TM_RK4, s);
}

}  // namespace

tm_status enqueue_attempts(const Problem* p, Workspace* w, int integ, int64_t B, int renorm,
                           int count, hipStream_t s) {
    if (integ == TM_RK4) {
        // pairs of steps advance the control in their last stages, from the
        // workspace's set into the second and back; an odd last step uses
        // the control pass
        const RkCtl c0 = rk_set(w, 0), c1 = rk_set(w, 1);
        int i = 0;
        for (; i + 1 < count; i += 2) {
            tm_status r = rk4_attempt(p, w, B, renorm, c0, &c1, s);
            if (r == TM_OK) r = rk4_attempt(p, w, B, renorm, c1, &c0, s);
            if (r != TM_OK) return r;
        }
        return i < count ? rk4_attempt(p, w, B, renorm, c0, nullptr, s) : TM_OK;
    }
    for (int i = 0; i < count; ++i) {
        tm_status r = dp_attempt(p, w, B, s);
        if (r != TM_OK) return r;
    }
    return TM_OK;
}

tm_status capture(const Problem* p, Workspace* w, int integ, int64_t B, int renorm, int count,
                  hipGraphExec_t* out) {
    if (!w->cap_stream) TM_TRY_HIP(hipStreamCreateWithFlags(&w->cap_stream, hipStreamNonBlocking));
    TM_TRY_HIP(hipStreamBeginCapture(w->cap_stream, hipStreamCaptureModeThreadLocal));
    tm_status r = enqueue_attempts(p, w, integ, B, renorm, count, w->cap_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(w->cap_stream, &g);
    if (r != TM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return r;
    }
    TM_TRY_HIP(e);
    e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    TM_TRY_HIP(e);
    return TM_OK;
}

namespace {
__global__ void k_init_slot(int64_t i, double dt0, double* __restrict__ t, double* __restrict__ h,
                            double* __restrict__ dt, int64_t* __restrict__ steps,
                            int64_t* __restrict__ rejected, int32_t* __restrict__ flags,
                            int32_t* __restrict__ acc) {
    if (threadIdx.x != 0) return;
    t[i] = 0.0;
    dt[i] = dt0;
    h[i] = dt0;
    steps[i] = 0;
    rejected[i] = 0;
    flags[i] = 0;
    acc[i] = 0;
}

__global__ void k_free_slot(int64_t i, double* __restrict__ h, int32_t* __restrict__ flags) {
    if (threadIdx.x != 0) return;
    h[i] = 0.0;
    flags[i] = FLAG_DONE;
}
}  // namespace

// Starts state `i` of a batch: control reset, k1 = f(y_i) and the first
// stage input, touching no other state.
tm_status start_slot(const Problem* p, Workspace* w, int64_t i, double dt0, hipStream_t s) {
    k_init_slot<<<1, 64, 0, s>>>(i, dt0, w->t, w->h, w->dt, w->steps, w->rejected, w->flags, w->acc);
    TM_TRY_HIP(hipGetLastError());
    const int64_t o = i * 3 * p->np;
    const double c[1] = {kDpA[1][0]};
    EpiArgs e = stage_args(w, w->k[0] + o, nullptr, 0, c, w->ya + o);
    e.Ha = w->Ha + 3 * i;
    e.y = w->y + o;
    e.h = w->h + i;
    e.params = w->params;
    return launch_field(p, Epi::STAGE, 1, w->y + o, e, s);
}

tm_status free_slot(Workspace* w, int64_t i, hipStream_t s) {
    k_free_slot<<<1, 64, 0, s>>>(i, w->h, w->flags);
    TM_TRY_HIP(hipGetLastError());
    return TM_OK;
}

}  // namespace tmag

using namespace tmag;

extern "C" tm_status tm_run(tm_problem* pp, tm_integrator integ, int64_t B, float* m, const float* Ha,
                            double* t, double* dt, int64_t* steps_out, const tm_run_cfg* cfg,
                            tm_run_stats* stats, hipStream_t s) {
    Problem* p = reinterpret_cast<Problem*>(pp);
    auto t0 = std::chrono::steady_clock::now();
    TM_REQUIRE(p && m && t && dt && cfg && B >= 1, TM_EINVAL, "tm_run: null argument or B < 1");
    TM_REQUIRE(integ == TM_RK4 || integ == TM_DP45, TM_EINVAL, "tm_run: unknown integrator");
    TM_REQUIRE(cfg->max_steps >= 0 && cfg->max_attempts >= 0, TM_EINVAL, "tm_run: negative limits");
    TM_REQUIRE(integ == TM_RK4 || (cfg->atol > 0.0 || cfg->rtol > 0.0), TM_EINVAL,
               "tm_run: DP45 needs atol > 0 or rtol > 0");
    TM_REQUIRE((reinterpret_cast<uintptr_t>(m) & 15) == 0, TM_EINVAL, "tm_run: m must be 16-byte aligned");
    TM_REQUIRE(B <= (int64_t(1) << 16), TM_EINVAL, "tm_run: batch too large");
    TM_REQUIRE(!cfg->persistent || persistent_eligible(p, integ, B), TM_EINVAL,
               "tm_run: persistent mode needs RK4, one state and an FP32 SYM6 operator of at most %lld "
               "padded tiles", static_cast<long long>(kPersistMaxTiles));
    TM_TRY_HIP(hipSetDevice(p->ctx->device));
    tm_status st = ensure_workspace(p, B);
    if (st != TM_OK) return st;
    Workspace* w = p->ws.get();
    // a graph holds B in its launch shapes: re-capture when B or the scheme changes
    const int renorm = cfg->renorm ? 1 : 0;
    if (w->graph1 && (w->graph_integ != static_cast<int>(integ) || w->graph_B != B ||
                      w->graph_renorm != renorm))
        w->drop_graphs();
    RunParams rp{};
    rp.v[RP_ATOL] = cfg->atol;
    rp.v[RP_RTOL] = cfg->rtol;
    rp.v[RP_TEND] = cfg->t_end;
    rp.v[RP_DTMIN] = cfg->dt_min;
    rp.v[RP_DMDT_STOP] = cfg->dmdt_stop;
    rp.v[RP_MAX_STEPS] = static_cast<double>(cfg->max_steps);
    rp.v[RP_RENORM] = cfg->renorm ? 1.0 : 0.0;
    {
        const int64_t cnt = B * p->np * 3;  // >= 3 B and >= RP_COUNT (np >= 128)
        k_begin_run<<<static_cast<unsigned>((cnt + 255) / 256), 256, 0, s>>>(
            m, p->n, p->np, B, w->y, Ha, w->Ha, rp, w->params, t, dt, w->t, w->h, w->dt, w->steps,
            w->rejected, w->flags, w->acc);
        TM_TRY_HIP(hipGetLastError());
    }
    int64_t attempts = 0;
    const bool persistent = cfg->persistent != 0;
    if (persistent) {
        st = launch_persistent_rk4(p, w, cfg, s);
        if (st != TM_OK) return st;
        attempts = cfg->max_steps;
        TM_TRY_HIP(hipMemcpyAsync(w->host_flags, w->bar_fail, 4, hipMemcpyDeviceToHost, s));
    }
    if (integ == TM_DP45) {
        st = dp_first(p, w, B, s);
        if (st != TM_OK) return st;
    }
    if (!persistent && cfg->use_graph && !w->graph1) {
        hipGraphExec_t* gs[5] = {&w->graph1, &w->graphP[0], &w->graphP[1], &w->graphP[2], &w->graphK};
        const int counts[5] = {1, 2, 4, 8, kGraphSteps};
        for (int i = 0; i < 5; ++i) {
            st = capture(p, w, integ, B, renorm, counts[i], gs[i]);
            if (st != TM_OK) {
                w->drop_graphs();
                return st;
            }
        }
        w->graph_integ = static_cast<int>(integ);
        w->graph_B = B;
        w->graph_renorm = renorm;
    }
    auto run_chunk = [&](int64_t cnt) -> tm_status {
        if (!cfg->use_graph) return enqueue_attempts(p, w, integ, B, renorm, static_cast<int>(cnt), s);
        const int64_t q = cnt / kGraphSteps, r = cnt % kGraphSteps;
        for (int64_t i = 0; i < q; ++i) TM_TRY_HIP(hipGraphLaunch(w->graphK, s));
        for (int b = 3; b >= 1; --b)
            if (r & (1 << b)) TM_TRY_HIP(hipGraphLaunch(w->graphP[b - 1], s));
        if (r & 1) TM_TRY_HIP(hipGraphLaunch(w->graph1, s));
        return TM_OK;
    };
    if (persistent) {
        // the whole run was one launch
    } else if (cfg->max_attempts > 0) {
        st = run_chunk(cfg->max_attempts);
        if (st != TM_OK) return st;
        attempts = cfg->max_attempts;
    } else {
        const int64_t poll = cfg->poll_every > 0 ? cfg->poll_every : 64;
        const int64_t cap = integ == TM_RK4 ? cfg->max_steps : 64 * cfg->max_steps + 4096;
        while (attempts < cap) {
            int64_t cnt = integ == TM_RK4 ? std::min(cap - attempts, cap) : std::min(poll, cap - attempts);
            st = run_chunk(cnt);
            if (st != TM_OK) return st;
            attempts += cnt;
            if (integ == TM_RK4) break;
            TM_TRY_HIP(hipMemcpyAsync(w->host_flags, w->flags, B * 4, hipMemcpyDeviceToHost, s));
            TM_TRY_HIP(hipStreamSynchronize(s));
            bool all = true;
            for (int64_t i = 0; i < B && all; ++i) all = w->host_flags[i] != 0;
            if (all) break;
        }
    }
    // results back to the caller's buffers, counts and flags to the host
    k_end_run<<<static_cast<unsigned>((B * p->n * 3 + 255) / 256), 256, 0, s>>>(
        w->y, p->n, p->np, B, m, w->t, w->dt, w->steps, w->rejected, w->flags, t, dt, steps_out, w->stat);
    TM_TRY_HIP(hipGetLastError());
    TM_TRY_HIP(hipMemcpyAsync(w->host_stat, w->stat, B * 24, hipMemcpyDeviceToHost, s));
    TM_TRY_HIP(hipStreamSynchronize(s));
    if (persistent && w->host_flags[0] != 0) {
        set_error("tm_run: a grid barrier of the persistent RK4 kernel timed out");
        return TM_EDEVICE;
    }
    int64_t amin = INT64_MAX, amax = 0, rej = 0;
    int32_t done = 0, failed = 0, nonfinite = 0;
    for (int64_t i = 0; i < B; ++i) {
        amin = std::min(amin, w->host_stat[i]);
        amax = std::max(amax, w->host_stat[i]);
        rej += w->host_stat[B + i];
        const int32_t f = static_cast<int32_t>(w->host_stat[2 * B + i]);
        if (f & FLAG_DONE) ++done;
        if (f & (FLAG_NONFINITE | FLAG_STEP)) ++failed;
        if (f & FLAG_NONFINITE) ++nonfinite;
    }
    if (stats) {
        stats->attempts = attempts;
        stats->accepted_min = amin;
        stats->accepted_max = amax;
        stats->rejected = rej;
        stats->states_done = done;
        stats->states_failed = failed;
        stats->elapsed_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
    if (nonfinite) {
        set_error("tm_run: %d state(s) produced non-finite values", nonfinite);
        return TM_ENONFINITE;
    }
    if (failed) {
        set_error("tm_run: %d state(s) stopped by step-size underflow", failed);
        return TM_ESTEP;
    }
    if (cfg->max_attempts == 0 && done < B) {
        set_error("tm_run: %lld state(s) not finished after %lld attempts",
                  static_cast<long long>(B - done), static_cast<long long>(attempts));
        return TM_ESTEP;
    }
    return TM_OK;
}

namespace tmag {

OpTimer*& op_timer() {
    static thread_local OpTimer* t = nullptr;
    return t;
}

namespace {

// Holds the stream for `ticks` of the constant-rate wall clock (one wave,
// bounded by construction), so that the host can enqueue a whole timed run
// behind it and the kernels then follow each other without host gaps, as
// in a graph replay.
__global__ void k_hold(int64_t ticks) {
    const long long t0 = wall_clock64();
    while (wall_clock64() - t0 < ticks) __builtin_amdgcn_s_sleep(8);
}

}  // namespace
}  // namespace tmag

extern "C" tm_status tm_profile_run(tm_problem* pp, tm_integrator integ, int64_t B, float* m, const float* Ha,
                                    double* t, double* dt, const tm_run_cfg* cfg, double* op_ms,
                                    int64_t* op_launches, hipStream_t s) {
    Problem* p = reinterpret_cast<Problem*>(pp);
    TM_REQUIRE(p && cfg && op_ms && op_launches, TM_EINVAL, "tm_profile_run: null argument");
    TM_REQUIRE(cfg->max_attempts >= 1 && cfg->max_attempts <= 100000, TM_EINVAL,
               "tm_profile_run: max_attempts must be in [1, 100000]");
    TM_REQUIRE(op_timer() == nullptr, TM_EBUSY, "tm_profile_run: already timing on this thread");
    TM_TRY_HIP(hipSetDevice(p->ctx->device));
    // operator passes: the first evaluation and six per attempt (DP45), four per step (RK4)
    const int64_t launches = integ == TM_DP45 ? 1 + 6 * cfg->max_attempts : 4 * cfg->max_attempts;
    OpTimer timer;
    timer.ev.assign(2 * launches, nullptr);
    hipError_t e = hipSuccess;
    for (auto& ev : timer.ev)
        if (e == hipSuccess) e = hipEventCreate(&ev);
    tm_status st = TM_OK;
    if (e != hipSuccess) {
        set_error("tm_profile_run: event creation failed: %s", hipGetErrorString(e));
        st = TM_EDEVICE;
    }
    if (st == TM_OK) {
        // a head start for the host: 1 ms per attempt of enqueueing (about
        // 13 launches with events; generous, so that a profiler's slower API
        // calls still finish first)
        int rate_khz = 0;
        if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, p->ctx->device) != hipSuccess ||
            rate_khz <= 0)
            rate_khz = 100000;
        const double hold_us = std::min(200000.0, 2000.0 + 1000.0 * static_cast<double>(cfg->max_attempts));
        k_hold<<<1, 64, 0, s>>>(static_cast<int64_t>(hold_us * rate_khz / 1000.0));
        if (hipGetLastError() != hipSuccess) {
            set_error("tm_profile_run: hold kernel launch failed");
            st = TM_EDEVICE;
        }
    }
    if (st == TM_OK) {
        tm_run_cfg c = *cfg;
        c.use_graph = 0;  // direct launches: every operator pass gets its own event pair
        tm_run_stats rs{};
        op_timer() = &timer;
        st = tm_run(pp, integ, B, m, Ha, t, dt, nullptr, &c, &rs, s);  // returns after a stream sync
        op_timer() = nullptr;
    }
    double sum = 0.0;
    if (st == TM_OK) {
        for (int64_t i = 0; i < timer.used && st == TM_OK; ++i) {
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, timer.ev[2 * i], timer.ev[2 * i + 1]) != hipSuccess) {
                set_error("tm_profile_run: no kernel timestamps for launch %lld", static_cast<long long>(i));
                st = TM_EDEVICE;
            }
            sum += ms;
        }
    }
    for (auto& ev : timer.ev)
        if (ev) (void)hipEventDestroy(ev);
    if (st != TM_OK) return st;
    *op_ms = sum;
    *op_launches = timer.used;
    return TM_OK;
}

namespace tmag {
namespace {

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Times `iters` launches of one epilogue variant of the field kernel on the
// problem's workspace (inputs and outputs never alias).
tm_status time_field(Problem* p, int64_t B, int mode, int32_t iters, hipStream_t s, double* avg_ms) {
    Workspace* w = p->ws.get();
    const float* kp[6] = {w->k[0], w->k[1], w->k[2], w->k[3], w->k[4], w->k[5]};
    double c[7] = {kDpA[2][0], kDpA[2][1], 0, 0, 0, 0, 0};
    EpiArgs e;
    Epi ep;
    const float* X;
    if (mode == 1) {
        e = EpiArgs{};
        e.out = w->hd;
        e.out_stride = 3 * p->np;
        ep = Epi::HD;
        X = w->ya;
    } else if (mode == 2) {
        const double none[7] = {0, 0, 0, 0, 0, 0, 0};
        e = stage_args(w, w->k[6], kp, 6, none, nullptr);
        ep = Epi::DP_LAST;
        X = w->y5;
    } else {
        // the stage-2 launch of a Dormand-Prince attempt: reads ya, k1, y; writes k2, yb
        e = stage_args(w, w->k[1], kp, 1, c, w->yb);
        ep = Epi::STAGE;
        X = w->ya;
    }
    // mode 4: stage launches as inside an attempt, each reading the previous
    // one's output (ya -> yb -> ya ...), so that the batched product takes
    // the right operand its previous stage wrote
    const EpiArgs e_back = mode == 4 ? stage_args(w, w->k[2], kp, 1, c, w->ya) : e;
    int parity = 0;
    // stages of a state with h = 0 are skipped: give every state a step
    k_fill<<<static_cast<unsigned>((B + 255) / 256), 256, 0, s>>>(w->h, B, 1e-15);
    TM_TRY_HIP(hipGetLastError());
    hipEvent_t e0, e1;
    TM_TRY_HIP(hipEventCreate(&e0));
    TM_TRY_HIP(hipEventCreate(&e1));
    // mode 3: the operator pass alone where the evaluation has more than one
    // launch (the pair-symmetric tile pass); otherwise the whole evaluation
    const bool tiles_only = mode == 3 && is_psym(p->T->layout);
    auto one = [&]() {
        if (tiles_only) return launch_psym_tiles(p, B, X, w->h, w->Ha, s);
        if (mode != 4) return launch_field(p, ep, B, X, e, s);
        // the first launch converts its input; every later one reads the copy
        w->frag_chain = parity > 0;
        const bool fwd = parity++ % 2 == 0;
        return launch_field(p, ep, B, fwd ? w->ya : w->yb, fwd ? e : e_back, s);
    };
    tm_status st = one();  // untimed first launch
    if (st == TM_OK && hipEventRecord(e0, s) != hipSuccess) st = TM_EDEVICE;
    for (int32_t i = 0; i < iters && st == TM_OK; ++i) st = one();
    float ms = 0.0f;
    if (st == TM_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&ms, e0, e1) != hipSuccess)) {
        set_error("field kernel timing: event failure");
        st = TM_EDEVICE;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == TM_OK) *avg_ms = static_cast<double>(ms) / iters;
    return st;
}

}  // namespace
}  // namespace tmag

extern "C" tm_status tm_profile_field_mode(tm_problem* pp, int64_t B, int32_t mode, int32_t iters,
                                           hipStream_t s, double* avg_ms, int64_t* bytes_out) {
    Problem* p = reinterpret_cast<Problem*>(pp);
    TM_REQUIRE(p && avg_ms && B >= 1 && iters >= 1 && mode >= 0 && mode <= 4, TM_EINVAL,
               "tm_profile_field: bad arguments");
    TM_TRY_HIP(hipSetDevice(p->ctx->device));
    tm_status st = ensure_workspace(p, B);
    if (st != TM_OK) return st;
    st = time_field(p, B, mode, iters, s, avg_ms);
    if (st != TM_OK) return st;
    if (bytes_out) {
        // operator bytes as stored (SYM6: 24 n^2; DENSE9: 36 n^2 algorithmic;
        // BSR6: row pointers, columns and six planes; PSYM6 / PSYM4: the
        // stored tile pairs) + states in and out
        const Tensor* T = p->T;
        const int64_t op = (T->layout == TM_LAYOUT_BSR6 || is_psym(T->layout)) ? T->bytes - (T->pairs ? T->npairs * 8 : 0)
                           : T->layout == TM_LAYOUT_DENSE9 ? (T->cblk ? 20 : 36) * p->n * p->n
                                                           : 24 * p->n * p->n;
        *bytes_out = op + 24 * p->n * B;
    }
    return TM_OK;
}

extern "C" tm_status tm_profile_field(tm_problem* pp, int64_t B, int32_t iters, hipStream_t s,
                                      double* avg_ms, int64_t* bytes_out) {
    return tm_profile_field_mode(pp, B, 0, iters, s, avg_ms, bytes_out);
}

extern "C" int32_t tm_num_shapes(void) { return kNumShapes; }

extern "C" tm_status tm_shape_info(int32_t shape, int32_t* threads, int32_t* tiles,
                                   int32_t* nontemporal, int32_t* waves_cap) {
    TM_REQUIRE(shape >= 0 && shape < kNumShapes, TM_EINVAL, "tm_shape_info: bad shape %d", shape);
    static const int32_t tab[kNumShapes][4] = {
#define TM_SHAPE(i, BL, TT, NT, WPE) {BL, TT, NT, WPE},
        TM_FIELD_SHAPES(TM_SHAPE)
#undef TM_SHAPE
    };
    if (threads) *threads = tab[shape][0];
    if (tiles) *tiles = tab[shape][1];
    if (nontemporal) *nontemporal = tab[shape][2];
    if (waves_cap) *waves_cap = tab[shape][3];
    return TM_OK;
}

extern "C" tm_status tm_problem_shape(const tm_problem* pp, int32_t* shape) {
    const Problem* p = reinterpret_cast<const Problem*>(pp);
    TM_REQUIRE(p && shape, TM_EINVAL, "tm_problem_shape: null argument");
    *shape = p->shape >= 0 ? p->shape : default_shape(p->n);
    return TM_OK;
}

extern "C" tm_status tm_problem_set_shape(tm_problem* pp, int32_t shape) {
    Problem* p = reinterpret_cast<Problem*>(pp);
    TM_REQUIRE(p && shape >= -1 && shape < kNumShapes, TM_EINVAL, "tm_problem_set_shape: bad shape");
    if (p->shape != shape && p->ws) {
        p->ws->drop_graphs();  // captured graphs hold the old launch shape
    }
    p->shape = shape;
    return TM_OK;
}

namespace tmag {
namespace {

// The candidates tm_problem_tune times for p: the K-split counts of the
// batched product, cached / nontemporal tile-pass loads of the pair-symmetric
// layouts, or the launch shapes of the six-plane stage kernel; none for the
// other operators (one kernel shape each).
enum class TuneKind { SPLITS, LOADS, SHAPES, NONE };

TuneKind tune_kind(const Problem* p) {
    if (p->T->layout == TM_LAYOUT_DENSE9 && p->T->prec != TM_PREC_FP64) return TuneKind::SPLITS;
    if (is_psym(p->T->layout)) return TuneKind::LOADS;
    if (p->T->layout == TM_LAYOUT_SYM6) return TuneKind::SHAPES;
    return TuneKind::NONE;
}

void drop_graphs(Problem* p) {
    if (p->ws) p->ws->drop_graphs();
}

// Applies choice c of kind k to p (captured graphs hold the old kernels and
// are dropped when it changes); false if c is not a candidate.
bool apply_choice(Problem* p, TuneKind k, int c) {
    static const int kCand[] = {2, 3, 4, 5, 6, 8};
    switch (k) {
        case TuneKind::SPLITS: {
            bool ok = gemm_aligned_nq(p, c) > 0;
            for (int q : kCand) ok = ok || (q == c && c <= p->T->ld / kGemmKC);
            if (!ok) return false;
            if (p->gemm_splits != c) drop_graphs(p);
            p->gemm_splits = c;
            return true;
        }
        case TuneKind::LOADS:
            if (c != 0 && c != 1) return false;
            if (p->psym_nt != c) drop_graphs(p);
            p->psym_nt = c;
            return true;
        case TuneKind::SHAPES:
            if (c < 0 || c >= kNumShapes) return false;
            if (p->shape != c) drop_graphs(p);
            p->shape = c;
            return true;
        case TuneKind::NONE:
            return c == -1;
    }
    return false;
}

}  // namespace
}  // namespace tmag

extern "C" tm_status tm_problem_apply(tm_problem* pp, int32_t choice) {
    Problem* p = reinterpret_cast<Problem*>(pp);
    TM_REQUIRE(p, TM_EINVAL, "tm_problem_apply: null problem");
    const TuneKind kind = tune_kind(p);
    TM_REQUIRE(kind != TuneKind::NONE, TM_EINVAL, "tm_problem_apply: this operator has no choices");
    TM_REQUIRE(apply_choice(p, kind, choice), TM_EINVAL, "tm_problem_apply: %d is not a candidate for this problem",
               static_cast<int>(choice));
    return TM_OK;
}

extern "C" tm_status tm_problem_tune(tm_problem* pp, int64_t B, int32_t iters, hipStream_t s,
                                     int32_t* chosen, double* best_ms) {
    Problem* p = reinterpret_cast<Problem*>(pp);
    TM_REQUIRE(p && B >= 1 && iters != 0, TM_EINVAL, "tm_problem_tune: bad arguments");
    TM_TRY_HIP(hipSetDevice(p->ctx->device));
    const TuneKind kind = tune_kind(p);
    if (iters > 0) {
        // a result for the same device, operator layout / precision, tile
        // count and batch is reused without timing
        TuneResult hit;
        if (tune_lookup(p, B, &hit) && apply_choice(p, kind, hit.choice)) {
            tm_status st = ensure_workspace(p, B);
            if (st != TM_OK) return st;
            if (chosen) *chosen = hit.choice;
            if (best_ms) *best_ms = hit.ms;
            return TM_OK;
        }
    }
    const int32_t reps = iters > 0 ? iters : -iters;
    tm_status st = ensure_workspace(p, B);
    if (st != TM_OK) return st;
    std::vector<int> cand;
    if (kind == TuneKind::SPLITS) {
        for (int c : {2, 3, 4, 5, 6, 8})
            if (c <= p->T->ld / kGemmKC) cand.push_back(c);
        for (int q = 2; q <= 8; ++q)
            if (gemm_aligned_nq(p, kGemmAligned + q)) cand.push_back(kGemmAligned + q);
    } else if (kind == TuneKind::LOADS) {
        cand = {0, 1};
    } else if (kind == TuneKind::SHAPES) {
        for (int c = 0; c < kNumShapes; ++c) cand.push_back(c);
    } else {
        cand = {-1};
    }
    const int keep_splits = p->gemm_splits, keep_nt = p->psym_nt, keep_shape = p->shape;
    int best = cand.front();
    double best_t = 1e30;
    for (int c : cand) {
        if (kind == TuneKind::SPLITS) p->gemm_splits = c;
        if (kind == TuneKind::LOADS) p->psym_nt = c;
        if (kind == TuneKind::SHAPES) p->shape = c;
        double ms = 0.0;
        st = ensure_workspace(p, B);  // the split count sizes the partial sums
        if (st == TM_OK) st = time_field(p, B, 0, reps, s, &ms);
        if (st != TM_OK) {
            p->gemm_splits = keep_splits;
            p->psym_nt = keep_nt;
            p->shape = keep_shape;
            return st;
        }
        if (ms < best_t) {
            best_t = ms;
            best = c;
        }
    }
    // back to the previous settings, then the winner (graphs dropped if it differs)
    p->gemm_splits = keep_splits;
    p->psym_nt = keep_nt;
    p->shape = keep_shape;
    (void)apply_choice(p, kind, best);
    if (kind == TuneKind::SPLITS) {
        st = ensure_workspace(p, B);
        if (st != TM_OK) return st;
    }
    TuneResult r;
    r.choice = best;
    r.ms = best_t;
    tune_store(p, B, r);
    if (chosen) *chosen = best;
    if (best_ms) *best_ms = best_t;
    return TM_OK;
}
