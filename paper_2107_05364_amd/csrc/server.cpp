// Serving: continuous batching of LLG relaxation requests.
//
// Requests that share a geometry (same canonical bytes, found through the
// context's tensor cache by geometry hash) and the same material and run
// settings form a group.  A group owns one problem whose integration
// workspace holds `max_slots` states; each request occupies one slot.  A
// scheduler thread admits queued requests into free slots (or new groups,
// when the tensor and workspace bytes fit the memory budget) and advances
// every active group in rounds of `steps_per_round` attempted DP45 steps
// from a captured hipGraph on the group's own stream.  Groups overlap on the
// device and progress independently: when a group's round ends (its event
// completes) the scheduler collects the slots whose state reached equilibrium
// (max_a |dm/dt|_a < threshold: Brown's first equation, paper Sec. 2.1) or
// their step cap, and frees them for the next request.  A state's arithmetic
// never depends on its slot or on the other states of the batch, so a result
// is the same alone and in the mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <thread>

#include "common.h"

using namespace tmag;

extern "C" tm_status tm_geometry_create(tm_ctx*, int64_t, const double*, const double*, tm_geom**);
extern "C" tm_status tm_geometry_destroy(tm_geom*);
extern "C" tm_status tm_tensor_assemble(tm_ctx*, const tm_geom*, tm_prec, tm_layout, hipStream_t,
                                        tm_tensor**);
extern "C" tm_status tm_tensor_release(tm_tensor*);
extern "C" tm_status tm_problem_create(tm_ctx*, const tm_geom*, tm_tensor*, const tm_material*,
                                       tm_problem**);
extern "C" tm_status tm_problem_destroy(tm_problem*);

namespace {

using clock_t_ = std::chrono::steady_clock;

struct Req {
    uint64_t ticket = 0;
    int64_t n = 0;
    std::vector<double> centers, sizes, Ms, Ku, easy;
    double A = 0, alpha = 0, gamma0 = 0;
    int32_t ll_form = 0;
    float Ha[3] = {0, 0, 0};
    std::vector<float> m;  // initial, then final state
    double dt0 = 0, atol = 0, rtol = 0, dmdt_stop = 0;
    int64_t max_steps = 0;
    uint64_t ghash = 0;
    clock_t_::time_point t_submit;
    // result
    bool done = false;
    int32_t status = TM_EBUSY;
    int64_t steps = 0;
    double t = 0, latency_ms = 0;
    int32_t cache_hit = 0;
};

struct Group {
    std::string key;
    tm_geom* geom = nullptr;
    tm_tensor* tensor = nullptr;
    tm_problem* prob = nullptr;
    Problem* P = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    std::vector<Req*> slot;  // nullptr: free
    int64_t bytes = 0;       // bytes charged to the server budget
    bool launched = false;
};

std::string group_key(const Req& r) {
    // the geometry's canonical bytes, material and run settings, all compared
    // exactly (the hash leads, so unlike keys usually differ in the first bytes)
    std::string k(reinterpret_cast<const char*>(&r.ghash), 8);
    auto add = [&k](const void* p, size_t len) { k.append(static_cast<const char*>(p), len); };
    add(&r.n, 8);
    add(r.centers.data(), r.centers.size() * 8);
    add(r.sizes.data(), r.sizes.size() * 8);
    add(r.Ms.data(), r.Ms.size() * 8);
    add(&r.A, 8);
    add(&r.alpha, 8);
    add(&r.gamma0, 8);
    add(&r.ll_form, 4);
    add(r.Ku.data(), r.Ku.size() * 8);
    add(r.easy.data(), r.easy.size() * 8);
    add(&r.atol, 8);
    add(&r.rtol, 8);
    add(&r.dmdt_stop, 8);
    add(&r.max_steps, 8);
    return k;
}

}  // namespace

struct tm_server {
    Ctx* ctx = nullptr;
    tm_server_cfg cfg{};
    int64_t budget = 0, used = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req*> queue;
    std::map<uint64_t, Req*> tickets;
    std::vector<Group*> groups;
    uint64_t next_ticket = 1;
    bool stopping = false;
    std::thread th;

    void run();
    bool try_place(Req* r);
    void finish(Group* g, size_t i, int32_t status);
    void drop_group(Group* g);
};

namespace {

// Meshes of identical tiles above kPsymMinTiles are served with the pair-
// symmetric operator (about half the bytes streamed per step; a third of them
// for a single layer, PSYM4), others with the
// six planes: below that size the step is launch-bound and the single fused
// six-plane launch per evaluation beats the pair-symmetric two (measured on
// the film sizes: 900 tiles 25 k vs 19 k steps/s, 1600 tiles 11.7 k vs 14.5 k).
constexpr int64_t kPsymMinTiles = 1200;

bool identical_tiles(const std::vector<double>& sizes) {
    for (size_t i = 3; i < sizes.size(); i += 3)
        if (sizes[i] != sizes[0] || sizes[i + 1] != sizes[1] || sizes[i + 2] != sizes[2]) return false;
    return true;
}

// One layer: every centre at the same z (the xz and yz components vanish).
bool single_layer(const std::vector<double>& centers) {
    for (size_t i = 5; i < centers.size(); i += 3)
        if (centers[i] != centers[2]) return false;
    return true;
}

int64_t operator_bytes(int64_t n, tm_layout layout) {
    if (is_psym(layout)) {
        const int64_t nt = (n + kPsTile - 1) / kPsTile;
        return nt * (nt + 1) / 2 * (psym_planes(layout) * kPsTile * kPsTile * 4 + 8);
    }
    return 6 * n * round_up(n, 4) * 4;
}

int64_t workspace_bytes(int64_t n, int64_t B, tm_layout layout) {
    const int64_t np = padded_tiles(n);
    int64_t b = 12 * B * 3 * np * 4 + B * 128 + 16 * B * n + 4096 + ((n + 255) / 256) * B * 32;
    if (is_psym(layout)) {
        const int64_t nt = (n + kPsTile - 1) / kPsTile;
        b += B * nt * nt * 3 * kPsTile * 4;
    }
    return b;
}

}  // namespace

void tm_server::finish(Group* g, size_t i, int32_t status) {
    Req* r = g->slot[i];
    Workspace* w = g->P->ws.get();
    const int64_t np = g->P->np;
    int64_t steps = 0;
    double t = 0;
    hipError_t e = hipMemcpyAsync(r->m.data(), w->y + i * 3 * np, r->n * 12, hipMemcpyDeviceToHost,
                                  g->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&steps, w->steps + i, 8, hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(&t, w->t + i, 8, hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    (void)free_slot(w, static_cast<int64_t>(i), g->stream);
    g->slot[i] = nullptr;
    std::lock_guard<std::mutex> lk(mu);
    r->steps = steps;
    r->t = t;
    r->status = e == hipSuccess ? status : TM_EDEVICE;
    r->latency_ms = std::chrono::duration<double, std::milli>(clock_t_::now() - r->t_submit).count();
    r->done = true;
    cv_done.notify_all();
}

void tm_server::drop_group(Group* g) {
    (void)hipStreamSynchronize(g->stream);
    if (g->prob) tm_problem_destroy(g->prob);
    if (g->tensor) tm_tensor_release(g->tensor);  // stays cached for later hits
    if (g->geom) tm_geometry_destroy(g->geom);
    (void)hipEventDestroy(g->ev);
    (void)hipStreamDestroy(g->stream);
    used -= g->bytes;
    delete g;
}

// Places r into a free slot of its group, or opens a new group when the
// budget allows.  Returns false if it must wait.
bool tm_server::try_place(Req* r) {
    const std::string key = group_key(*r);
    Group* g = nullptr;
    for (Group* q : groups)
        if (q->key == key) {
            auto it = std::find(q->slot.begin(), q->slot.end(), nullptr);
            if (it != q->slot.end()) {
                if (q->launched) return false;  // mid-round: placed when the round ends
                g = q;
                break;
            }
        }
    const int64_t B = cfg.max_slots;
    if (!g) {
        if (static_cast<int>(groups.size()) >= cfg.max_groups) return false;
        // bytes a new group needs: the operator unless cached, plus the slots
        bool cached = false;
        const tm_layout layout = r->n > kPsymMinTiles && identical_tiles(r->sizes)
                                     ? (single_layer(r->centers) ? TM_LAYOUT_PSYM4 : TM_LAYOUT_PSYM6)
                                     : TM_LAYOUT_SYM6;
        const int64_t tbytes = operator_bytes(r->n, layout);
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            for (Tensor* T : ctx->cache)
                if (T->hash == r->ghash && T->n == r->n && T->prec == TM_PREC_FP32 && T->layout == layout &&
                    T->centers == r->centers && T->sizes == r->sizes)
                    cached = true;
        }
        const int64_t need = (cached ? 0 : tbytes) + workspace_bytes(r->n, B, layout);
        if (used + need > budget) {
            if (groups.empty()) {  // nothing will ever free up: refuse
                std::lock_guard<std::mutex> lk(mu);
                r->status = TM_ENOMEM;
                r->done = true;
                cv_done.notify_all();
                return true;
            }
            return false;
        }
        g = new Group();
        g->key = key;
        g->slot.assign(B, nullptr);
        tm_status st = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) == hipSuccess &&
                               hipEventCreateWithFlags(&g->ev, hipEventDisableTiming) == hipSuccess
                           ? TM_OK
                           : TM_EDEVICE;
        if (st == TM_OK)
            st = tm_geometry_create(reinterpret_cast<tm_ctx*>(ctx), r->n, r->centers.data(),
                                    r->sizes.data(), &g->geom);
        int64_t hits0 = ctx->cache_hits;
        if (st == TM_OK)
            st = tm_tensor_assemble(reinterpret_cast<tm_ctx*>(ctx), g->geom, TM_PREC_FP32, layout, g->stream,
                                    &g->tensor);
        r->cache_hit = ctx->cache_hits > hits0 ? 1 : 0;
        tm_material mat{r->Ms.data(), r->A, r->Ku.empty() ? nullptr : r->Ku.data(),
                        r->easy.empty() ? nullptr : r->easy.data(), r->alpha, r->gamma0, r->ll_form};
        if (st == TM_OK)
            st = tm_problem_create(reinterpret_cast<tm_ctx*>(ctx), g->geom, g->tensor, &mat, &g->prob);
        if (st == TM_OK) {
            g->P = reinterpret_cast<Problem*>(g->prob);
            st = ensure_workspace(g->P, B);
        }
        if (st == TM_OK) {
            Workspace* w = g->P->ws.get();
            double* hp = w->host_params;
            hp[RP_ATOL] = r->atol;
            hp[RP_RTOL] = r->rtol;
            hp[RP_TEND] = 0.0;
            hp[RP_DTMIN] = 0.0;
            hp[RP_DMDT_STOP] = r->dmdt_stop;
            hp[RP_MAX_STEPS] = static_cast<double>(r->max_steps);
            hp[RP_RENORM] = 1.0;
            if (hipMemcpyAsync(w->params, hp, RP_COUNT * 8, hipMemcpyHostToDevice, g->stream) != hipSuccess)
                st = TM_EDEVICE;
            for (int64_t i = 0; i < B && st == TM_OK; ++i) st = free_slot(w, i, g->stream);
            if (st == TM_OK) st = capture(g->P, w, TM_DP45, B, 1, kGraphSteps, &w->graphK);
            if (st == TM_OK) {
                w->graph_integ = TM_DP45;
                w->graph_B = B;
                w->graph_renorm = 1;
            }
        }
        if (st != TM_OK) {
            std::string msg = tm_last_error();
            if (g->prob) tm_problem_destroy(g->prob);
            if (g->tensor) tm_tensor_release(g->tensor);
            if (g->geom) tm_geometry_destroy(g->geom);
            if (g->ev) (void)hipEventDestroy(g->ev);
            if (g->stream) (void)hipStreamDestroy(g->stream);
            delete g;
            if (st == TM_ENOMEM && !groups.empty()) return false;  // wait for memory
            std::lock_guard<std::mutex> lk(mu);
            r->status = st;
            r->done = true;
            cv_done.notify_all();
            return true;
        }
        g->bytes = need;
        used += need;
        groups.push_back(g);
    } else {
        r->cache_hit = 1;
    }
    // load the state into a free slot and start it
    size_t i = std::find(g->slot.begin(), g->slot.end(), nullptr) - g->slot.begin();
    Workspace* w = g->P->ws.get();
    const int64_t o = static_cast<int64_t>(i) * 3 * g->P->np;
    tm_status st = TM_OK;
    if (hipMemcpyAsync(w->y + o, r->m.data(), r->n * 12, hipMemcpyHostToDevice, g->stream) != hipSuccess ||
        hipMemcpyAsync(w->Ha + 3 * i, r->Ha, 12, hipMemcpyHostToDevice, g->stream) != hipSuccess)
        st = TM_EDEVICE;
    if (st == TM_OK) st = start_slot(g->P, w, static_cast<int64_t>(i), r->dt0, g->stream);
    // pageable sources: make the copies complete before the host buffers move on
    if (st == TM_OK && hipStreamSynchronize(g->stream) != hipSuccess) st = TM_EDEVICE;
    if (st != TM_OK) {
        std::lock_guard<std::mutex> lk(mu);
        r->status = st;
        r->done = true;
        cv_done.notify_all();
        return true;
    }
    g->slot[i] = r;
    return true;
}

void tm_server::run() {
    (void)hipSetDevice(ctx->device);
    std::vector<Req*> waiting;
    auto has_work = [](const Group* g) {
        for (Req* r : g->slot)
            if (r) return true;
        return false;
    };
    for (;;) {
        bool inflight = false;
        for (Group* g : groups) inflight = inflight || g->launched;
        {
            std::unique_lock<std::mutex> lk(mu);
            bool busy = !waiting.empty() || inflight;
            for (Group* g : groups) busy = busy || has_work(g);
            if (!busy) cv_work.wait(lk, [&] { return stopping || !queue.empty(); });
            while (!queue.empty()) {
                waiting.push_back(queue.front());
                queue.pop_front();
            }
            bool active = !waiting.empty() || inflight;
            for (Group* g : groups) active = active || has_work(g);
            if (stopping && !active) break;
        }
        bool progressed = false;
        // collect every group whose round has completed; the others keep running
        for (Group* g : groups) {
            if (!g->launched) continue;
            const hipError_t q = hipEventQuery(g->ev);
            if (q == hipErrorNotReady) continue;
            g->launched = false;
            progressed = true;
            if (q != hipSuccess) {
                for (size_t i = 0; i < g->slot.size(); ++i)
                    if (g->slot[i]) finish(g, i, TM_EDEVICE);
                continue;
            }
            Workspace* w = g->P->ws.get();
            for (size_t i = 0; i < g->slot.size(); ++i) {
                if (!g->slot[i]) continue;
                const int32_t f = w->host_flags[i];
                if (f & FLAG_NONFINITE)
                    finish(g, i, TM_ENONFINITE);
                else if (f & FLAG_STEP)
                    finish(g, i, TM_ESTEP);
                else if (f & FLAG_CAPPED)
                    finish(g, i, TM_ESTEP);  // step cap reached before equilibrium
                else if (f & FLAG_DONE)
                    finish(g, i, TM_OK);
            }
        }
        // admission in arrival order into idle groups or new ones; a request
        // whose group is mid-round, or that does not fit, waits
        std::vector<Req*> still;
        for (Req* r : waiting) {
            if (try_place(r))
                progressed = true;
            else
                still.push_back(r);
        }
        waiting.swap(still);
        // the next round of the idle groups with work; with max_active > 0 only
        // the max_active groups holding the oldest requests advance, so that
        // the device is not split over every resident group (the oldest
        // requests finish first, as in arrival order)
        std::vector<Group*> order;
        for (Group* g : groups)
            if (has_work(g)) order.push_back(g);
        auto oldest = [](const Group* g) {
            clock_t_::time_point t = clock_t_::time_point::max();
            for (const Req* r : g->slot)
                if (r && r->t_submit < t) t = r->t_submit;
            return t;
        };
        std::stable_sort(order.begin(), order.end(),
                         [&](const Group* a, const Group* b) { return oldest(a) < oldest(b); });
        if (cfg.max_active > 0 && static_cast<int>(order.size()) > cfg.max_active) order.resize(cfg.max_active);
        for (Group* g : order) {
            if (g->launched) continue;
            Workspace* w = g->P->ws.get();
            const int rounds = std::max(1, cfg.steps_per_round / kGraphSteps);
            bool ok = true;
            for (int k = 0; k < rounds && ok; ++k) ok = hipGraphLaunch(w->graphK, g->stream) == hipSuccess;
            ok = ok && hipMemcpyAsync(w->host_flags, w->flags, g->slot.size() * 4, hipMemcpyDeviceToHost,
                                      g->stream) == hipSuccess;
            ok = ok && hipEventRecord(g->ev, g->stream) == hipSuccess;
            g->launched = ok;
            progressed = true;
            if (!ok)
                for (size_t i = 0; i < g->slot.size(); ++i)
                    if (g->slot[i]) finish(g, i, TM_EDEVICE);
        }
        // idle groups without work are closed when others wait for memory or
        // group room; their tensors stay cached
        std::vector<Group*> keep;
        for (Group* g : groups) {
            if (!g->launched && !has_work(g) && !waiting.empty())
                drop_group(g);
            else
                keep.push_back(g);
        }
        groups.swap(keep);
        if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    for (Group* g : groups) drop_group(g);
    groups.clear();
}

extern "C" {

tm_status tm_server_create(tm_ctx* c, const tm_server_cfg* cfg, tm_server** out) {
    TM_REQUIRE(c && cfg && out, TM_EINVAL, "tm_server_create: null argument");
    TM_REQUIRE(cfg->max_slots >= 1 && cfg->max_slots <= 4096 && cfg->max_groups >= 1 &&
                   cfg->steps_per_round >= 1 && cfg->max_active >= 0,
               TM_EINVAL, "tm_server_create: bad slot / group / round settings");
    TM_REQUIRE(cfg->prec == TM_PREC_FP32, TM_EINVAL, "tm_server_create: only FP32 operators are served");
    Ctx* ctx = reinterpret_cast<Ctx*>(c);
    tm_server* s = new tm_server();
    s->ctx = ctx;
    s->cfg = *cfg;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        s->budget = cfg->memory_budget > 0 ? std::min(cfg->memory_budget, ctx->budget) : ctx->budget;
        ctx->live_servers += 1;
    }
    s->th = std::thread([s] { s->run(); });
    *out = s;
    return TM_OK;
}

tm_status tm_server_submit(tm_server* s, const tm_request* q, uint64_t* ticket) {
    TM_REQUIRE(s && q && ticket && q->centers && q->sizes && q->m0 && q->mat.Ms, TM_EINVAL,
               "tm_server_submit: null argument");
    TM_REQUIRE(q->n >= 1 && q->dt0 > 0.0 && q->max_steps >= 1 && (q->atol > 0.0 || q->rtol > 0.0),
               TM_EINVAL, "tm_server_submit: n, dt0, max_steps and a tolerance must be positive");
    for (int64_t i = 0; i < 3 * q->n; ++i)
        TM_REQUIRE(std::isfinite(q->centers[i]) && std::isfinite(q->sizes[i]) && q->sizes[i] > 0.0,
                   TM_EINVAL, "tm_server_submit: bad geometry at tile %lld", static_cast<long long>(i / 3));
    Req* r = new Req();
    r->n = q->n;
    r->centers.assign(q->centers, q->centers + 3 * q->n);
    r->sizes.assign(q->sizes, q->sizes + 3 * q->n);
    r->Ms.assign(q->mat.Ms, q->mat.Ms + q->n);
    if (q->mat.Ku) {
        TM_REQUIRE(q->mat.easy, TM_EINVAL, "tm_server_submit: Ku without easy axes");
        r->Ku.assign(q->mat.Ku, q->mat.Ku + q->n);
        r->easy.assign(q->mat.easy, q->mat.easy + 3 * q->n);
    }
    r->A = q->mat.A_exch;
    r->alpha = q->mat.alpha;
    r->gamma0 = q->mat.gamma0;
    r->ll_form = q->mat.ll_form;
    for (int i = 0; i < 3; ++i) r->Ha[i] = static_cast<float>(q->Ha[i]);
    r->m.assign(q->m0, q->m0 + 3 * q->n);
    r->dt0 = q->dt0;
    r->atol = q->atol;
    r->rtol = q->rtol;
    r->dmdt_stop = q->dmdt_stop;
    r->max_steps = q->max_steps;
    r->ghash = geometry_hash(q->n, q->centers, q->sizes);
    r->t_submit = clock_t_::now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        TM_REQUIRE(!s->stopping, TM_EBUSY, "tm_server_submit: server is stopping");
        r->ticket = s->next_ticket++;
        s->tickets[r->ticket] = r;
        s->queue.push_back(r);
    }
    s->cv_work.notify_one();
    *ticket = r->ticket;
    return TM_OK;
}

tm_status tm_server_poll(tm_server* s, uint64_t ticket, int32_t wait, tm_result* res, float* m_out) {
    TM_REQUIRE(s && res, TM_EINVAL, "tm_server_poll: null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    TM_REQUIRE(it != s->tickets.end(), TM_ENOTFOUND, "tm_server_poll: unknown ticket %llu",
               static_cast<unsigned long long>(ticket));
    Req* r = it->second;
    if (wait) s->cv_done.wait(lk, [r] { return r->done; });
    res->status = r->done ? r->status : TM_EBUSY;
    res->steps = r->steps;
    res->t = r->t;
    res->latency_ms = r->latency_ms;
    res->cache_hit = r->cache_hit;
    if (r->done && m_out) std::memcpy(m_out, r->m.data(), r->m.size() * 4);
    return TM_OK;
}

tm_status tm_server_destroy(tm_server* s) {
    TM_REQUIRE(s, TM_EINVAL, "tm_server_destroy: null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
    }
    s->cv_work.notify_all();
    if (s->th.joinable()) s->th.join();
    for (auto& kv : s->tickets) delete kv.second;
    {
        std::lock_guard<std::mutex> lk(s->ctx->mu);
        s->ctx->live_servers -= 1;
    }
    delete s;
    return TM_OK;
}

}  // extern "C"
