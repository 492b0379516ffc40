// server.cpp -- continuous-batching serving of SR solves (misr_server_*).
//
// The paper super-resolves each rotation angle's frames as soon as they are
// captured, reusing the system matrices built once per acquisition (Sec. 2.2).
// Here every request is one such solve.  A scheduler thread admits queued
// requests while device memory (a byte budget) and slots allow, keeps each
// admitted solve's SCG state resident on the device, and advances all admitted
// solves together: every SCG pass of every solve runs in the same kernel
// launches over one work list of (view, tile) items, so requests that arrive
// while others run join at the next pass boundary.  Each solve keeps its own
// state and reductions (fixed order per solve), so its result does not depend
// on which other solves share the launches.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <functional>
#include <tuple>
#include <map>
#include <thread>

#include "runtime.h"

using namespace misr;

namespace {

double now_us() {
    using namespace std::chrono;
    return duration<double, std::micro>(steady_clock::now().time_since_epoch()).count();
}

struct OpKey {
    int H, W, s, K, P;
    std::vector<double> shifts, psf;
    bool operator<(const OpKey &o) const {
        return std::tie(H, W, s, K, P, shifts, psf) <
               std::tie(o.H, o.W, o.s, o.K, o.P, o.shifts, o.psf);
    }
};

struct SReq {
    uint64_t id = 0;
    misr_request req{};
    std::vector<double> shifts, psf;
    misr_req_state state = MISR_REQ_QUEUED;
    misr_req_stats stats{};
    bool cancel = false;
    misr_op *op = nullptr;
    size_t bytes = 0;
    long long n = 0;      // HR pixels
    size_t es = 4;
    int passes = 0;       // passes enqueued
    bool fresh = true;    // init not yet enqueued
    // device memory owned by the server for this request
    DevMem xwork, ydev, dstate;
    SolveBufs bufs;
    void *x0dev = nullptr;
    const void *ydev_ptr = nullptr;
    ScgState *st_dev = nullptr;
    IterRec *trace_dev = nullptr;
};

}  // namespace

struct misr_server {
    misr_ctx *ctx = nullptr;
    misr_server_config cfg{};
    hipStream_t stream = nullptr;
    std::thread th;
    std::mutex mu;
    std::condition_variable cv, cv_done;
    bool closing = false;
    uint64_t next_id = 1;
    std::deque<SReq *> queue;
    std::map<uint64_t, std::unique_ptr<SReq>> reqs;
    std::vector<SReq *> active;   // scheduler thread only
    size_t used = 0;
    int alloc_count = 0;
    std::map<OpKey, misr_op *> ops;
    // work list of all active solves; per class, the running solves' items
    // come first and the newly admitted ones' after, so that the init passes
    // of the new solves run over a sub-range and leave their partial sums where
    // the next pass of the whole list reads them
    struct List {
        Plan pl;
        std::vector<int> new_begin;          // per class: first item of the new solves
        std::vector<SolveRef> refs_new;      // the new solves only
        DevMem projs, items, counts, refs, drefs_new, partials;
    } all;
    std::string last_error;

    void run();
    bool setup(SReq *r);
    void release(SReq *r);
    void build_list(List &L, const std::vector<SReq *> &rs);
    hipError_t enqueue_init(List &L);
    hipError_t enqueue_image(List &L, int kind);
    void finish(SReq *r, misr_req_state st, misr_status code);
};

static size_t request_bytes(const misr_request &q, long long n, size_t es, int K, long long m) {
    size_t b = (size_t)n * es * 2 + (size_t)n * 16;           // x pair, p pair, g pair
    if (!q.on_device) b += (size_t)K * m * es + (size_t)n * es;  // y and x staged on device
    b += sizeof(ScgState) + (size_t)std::max(1, q.params.n_iter) * sizeof(IterRec);
    return b;
}

bool misr_server::setup(SReq *r) {
    const misr_request &q = r->req;
    if (cfg.fail_alloc_n > 0 && ++alloc_count == cfg.fail_alloc_n) return false;
    misr_geometry g = q.geom;
    g.shifts_lr = r->shifts.data();
    g.psf_1d = r->psf.data();
    OpKey key{g.hr_h, g.hr_w, g.scale, g.n_frames, g.psf_size, r->shifts, r->psf};
    auto it = ops.find(key);
    if (it == ops.end()) {
        misr_op *op = nullptr;
        if (misr_op_create(ctx, &g, &op) != MISR_OK) return false;
        it = ops.emplace(key, op).first;
    }
    r->op = it->second;
    const long long m = (long long)(g.hr_h / g.scale) * (g.hr_w / g.scale) * g.n_frames;
    if (r->bufs.ensure(r->n, r->es) != hipSuccess) return false;
    const size_t per = (size_t)std::max(1, q.params.n_iter);
    if (r->dstate.ensure(sizeof(ScgState) + per * sizeof(IterRec)) != hipSuccess) return false;
    r->st_dev = r->dstate.as<ScgState>();
    r->trace_dev = (IterRec *)(r->dstate.as<char>() + sizeof(ScgState));
    if (q.on_device) {
        r->x0dev = q.x_out;
        r->ydev_ptr = q.y;
        if (q.x0 != q.x_out &&
            hipMemcpyAsync(q.x_out, q.x0, r->n * r->es, hipMemcpyDeviceToDevice, stream) !=
                hipSuccess)
            return false;
    } else {
        if (r->xwork.ensure(r->n * r->es) != hipSuccess) return false;
        if (r->ydev.ensure(m * r->es) != hipSuccess) return false;
        r->x0dev = r->xwork.p;
        r->ydev_ptr = r->ydev.p;
        if (hipMemcpyAsync(r->xwork.p, q.x0, r->n * r->es, hipMemcpyHostToDevice, stream) !=
                hipSuccess ||
            hipMemcpyAsync(r->ydev.p, q.y, m * r->es, hipMemcpyHostToDevice, stream) !=
                hipSuccess)
            return false;
    }
    ScgState st;
    std::memset(&st, 0, sizeof st);
    st.lam = q.params.scg_lambda1;
    st.sigma = q.params.scg_sigma;
    st.N = r->n;
    st.n_iter = q.params.n_iter;
    st.success = 1;
    st.active = 1;
    for (int dy = 0; dy < 3; ++dy)
        for (int dx = 0; dx < 3; ++dx)
            st.wt.gam[dy * 3 + dx] =
                (dx == 0 && dy == 0) || dx >= q.params.btv_w || dy >= q.params.btv_w
                    ? 0.f
                    : (float)(q.params.lambda_reg * std::pow(q.params.alpha_btv, dx + dy));
    st.wt.eps = (float)q.params.eps;
    st.wt.eps_data = (float)q.params.eps_data;
    st.wt.data_p = q.params.data_p;
    st.wt.x_rounding = q.params.x_rounding;
    return hipMemcpyAsync(r->st_dev, &st, sizeof st, hipMemcpyHostToDevice, stream) ==
               hipSuccess &&
           hipStreamSynchronize(stream) == hipSuccess;   // st lives on this stack frame
}

void misr_server::release(SReq *r) {
    r->xwork.release();
    r->ydev.release();
    r->dstate.release();
    r->bufs.x1.release();
    r->bufs.p0.release();
    r->bufs.p1.release();
    r->bufs.g0.release();
    r->bufs.g1.release();
    std::lock_guard<std::mutex> lk(mu);
    used -= std::min(used, r->bytes);
}

void misr_server::build_list(List &L, const std::vector<SReq *> &rs) {
    Plan &pl = L.pl;
    pl.projs.clear();
    pl.items.clear();
    pl.classes.clear();
    pl.counts.clear();
    pl.refs.clear();
    L.new_begin.clear();
    L.refs_new.clear();
    std::map<std::pair<int, int>, std::vector<SReq *>> groups;
    std::vector<std::pair<int, int>> order;
    for (int pass = 0; pass < 2; ++pass)       // running solves first, then new ones
        for (SReq *r : rs) {
            if (r->fresh != (pass == 1)) continue;
            auto key = std::make_pair(r->op->s, r->op->Lp);
            if (!groups.count(key)) order.push_back(key);
            groups[key].push_back(r);
        }
    for (auto &key : order) {
        Plan::Cls c{key.first, key.second, (int)pl.items.size(), 0};
        int nb = -1;
        for (SReq *r : groups[key]) {
            if (r->fresh && nb < 0) nb = (int)pl.items.size();
            const misr_op *op = r->op;
            Proj P;
            std::memset(&P, 0, sizeof P);
            P.x[0] = r->x0dev;
            P.x[1] = r->bufs.x1.p;
            P.p[0] = r->bufs.p0.as<float>();
            P.p[1] = r->bufs.p1.as<float>();
            P.g[0] = r->bufs.g0.as<float>();
            P.g[1] = r->bufs.g1.as<float>();
            P.y = r->ydev_ptr;
            P.ld = op->W;
            P.Hb = op->H;
            P.Wb = op->W;
            P.oy1 = P.uy1 = op->H;
            P.ox1 = P.ux1 = op->W;
            P.ntx = (op->W + op->TW - 1) / op->TW;
            P.st = r->st_dev;
            P.op = op->opdev.as<OpDev>();
            const int nty = (op->H + op->TH - 1) / op->TH;
            const int pj = (int)pl.projs.size();
            pl.projs.push_back(P);
            const int i0 = (int)pl.items.size();
            for (int ty = 0; ty < nty; ++ty)
                for (int tx = 0; tx < P.ntx; ++tx) pl.items.push_back(Item{pj, ty, tx, 0});
            // untiled views: the update pass walks the same items as the trial pass
            const int ni = (int)pl.items.size() - i0;
            pl.refs.push_back(SolveRef{r->st_dev, r->trace_dev, i0, ni, i0, ni});
            if (r->fresh) L.refs_new.push_back(pl.refs.back());
        }
        c.count = (int)pl.items.size() - c.start;
        pl.classes.push_back(c);
        L.new_begin.push_back(nb < 0 ? (int)pl.items.size() : nb);
    }
    // counts: per class items, n solves, per class new items, n new solves
    for (auto &c : pl.classes) pl.counts.push_back(c.count);
    pl.counts.push_back((int)pl.refs.size());
    for (size_t c = 0; c < pl.classes.size(); ++c)
        pl.counts.push_back(pl.classes[c].start + pl.classes[c].count - L.new_begin[c]);
    pl.counts.push_back((int)L.refs_new.size());
    const size_t np = pl.projs.size(), ni = pl.items.size(), ns = pl.refs.size();
    bool ok = L.projs.ensure(np * sizeof(Proj)) == hipSuccess &&
              L.items.ensure(ni * sizeof(Item)) == hipSuccess &&
              L.counts.ensure(pl.counts.size() * sizeof(int)) == hipSuccess &&
              L.refs.ensure(ns * sizeof(SolveRef)) == hipSuccess &&
              L.drefs_new.ensure((L.refs_new.size() + 1) * sizeof(SolveRef)) == hipSuccess &&
              L.partials.ensure(ni * kNV * sizeof(double)) == hipSuccess;
    if (ok) {
        (void)hipMemcpyAsync(L.projs.p, pl.projs.data(), np * sizeof(Proj),
                             hipMemcpyHostToDevice, stream);
        (void)hipMemcpyAsync(L.items.p, pl.items.data(), ni * sizeof(Item),
                             hipMemcpyHostToDevice, stream);
        (void)hipMemcpyAsync(L.counts.p, pl.counts.data(), pl.counts.size() * sizeof(int),
                             hipMemcpyHostToDevice, stream);
        (void)hipMemcpyAsync(L.refs.p, pl.refs.data(), ns * sizeof(SolveRef),
                             hipMemcpyHostToDevice, stream);
        if (!L.refs_new.empty())
            (void)hipMemcpyAsync(L.drefs_new.p, L.refs_new.data(),
                                 L.refs_new.size() * sizeof(SolveRef), hipMemcpyHostToDevice,
                                 stream);
    }
}

// Init of the newly admitted solves over their sub-range of the list: cost
// and gradient at x0, Moller's init, update pass (p = -g0) with curvature.
hipError_t misr_server::enqueue_init(List &L) {
    const int nc = (int)L.pl.classes.size();
    const int *cnt = L.counts.as<int>();
    const misr_dtype dt = active.empty() ? MISR_F32 : active[0]->req.params.img_dtype;
    auto image = [&](int kind) {
        for (int c = 0; c < nc; ++c) {
            const Plan::Cls &cl = L.pl.classes[c];
            const int nb = L.new_begin[c], n = cl.start + cl.count - nb;
            if (n <= 0) continue;
            hipError_t e = launch_image(cl.S, cl.Lp, n, stream, L.projs.as<Proj>(),
                                        L.items.as<Item>() + nb, cnt + nc + 1 + c,
                                        L.partials.as<double>() + (size_t)nb * kNV, kind,
                                        (int)dt);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    hipError_t e = image(KIND_COSTGRAD);
    if (e == hipSuccess)
        e = launch_scalar((int)L.refs_new.size(), stream, L.drefs_new.as<SolveRef>(),
                          cnt + 2 * nc + 1, L.partials.as<double>(), L.partials.as<double>(),
                          PHASE_INIT);
    if (e == hipSuccess) e = image(KIND_UPCURV);
    return e;
}

hipError_t misr_server::enqueue_image(List &L, int kind) {
    const int nc = (int)L.pl.classes.size();
    for (int c = 0; c < nc; ++c) {
        const Plan::Cls &cl = L.pl.classes[c];
        const misr_dtype dt = active.empty() ? MISR_F32 : active[0]->req.params.img_dtype;
        hipError_t e = launch_image(cl.S, cl.Lp, cl.count, stream, L.projs.as<Proj>(),
                                    L.items.as<Item>() + cl.start, L.counts.as<int>() + c,
                                    L.partials.as<double>() + (size_t)cl.start * kNV, kind,
                                    (int)dt);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

void misr_server::finish(SReq *r, misr_req_state st, misr_status code) {
    std::function<void()> cb;
    {
        std::lock_guard<std::mutex> lk(mu);
        r->state = st;
        r->stats.status = code;
        r->stats.t_done_us = now_us();
    }
    cv_done.notify_all();
    if (r->req.done_cb) r->req.done_cb(r->id, code, r->req.user);
}

void misr_server::run() {
    (void)hipSetDevice(ctx->dev);
    for (;;) {
        std::vector<SReq *> admitted, cancelled;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] { return closing || !queue.empty() || !active.empty(); });
            if (closing && queue.empty() && active.empty()) break;
            // admission by free device memory and slots, first come first served
            while (!queue.empty() &&
                   (int)(active.size() + admitted.size()) < std::max(1, cfg.max_slots)) {
                SReq *r = queue.front();
                if (used + r->bytes > cfg.hbm_budget_bytes) {
                    if (active.empty() && admitted.empty()) {
                        queue.pop_front();
                        r->state = MISR_REQ_FAILED;
                        r->stats.status = MISR_E_NOMEM;
                        r->stats.t_done_us = now_us();
                        cv_done.notify_all();
                        continue;
                    }
                    break;
                }
                queue.pop_front();
                used += r->bytes;
                r->state = MISR_REQ_RUNNING;
                r->stats.t_admit_us = now_us();
                admitted.push_back(r);
            }
            for (SReq *r : active)
                if (r->cancel) cancelled.push_back(r);
        }
        for (SReq *r : cancelled) {
            active.erase(std::find(active.begin(), active.end(), r));
            release(r);
            finish(r, MISR_REQ_CANCELLED, MISR_E_CANCELLED);
        }
        std::vector<SReq *> fresh;
        for (SReq *r : admitted) {
            if (!setup(r)) {
                (void)hipStreamSynchronize(stream);
                release(r);
                finish(r, MISR_REQ_FAILED, MISR_E_NOMEM);
                continue;
            }
            active.push_back(r);
            fresh.push_back(r);
        }
        if (active.empty()) continue;
        // passes this cycle: up to the earliest completion (at most 8)
        int n_ep = 8;
        for (SReq *r : active) n_ep = std::min(n_ep, r->req.params.n_iter - r->passes);
        n_ep = std::max(n_ep, 0);
        hipError_t e = hipSuccess;
        build_list(all, active);
        if (!fresh.empty()) {
            e = enqueue_init(all);
            for (SReq *r : fresh) r->fresh = false;
        }
        const int ns = (int)all.pl.refs.size();
        const int *d_ns = all.counts.as<int>() + all.pl.classes.size();
        for (int ep = 0; ep < n_ep && e == hipSuccess; ++ep) {
            e = launch_scalar(ns, stream, all.refs.as<SolveRef>(), d_ns, all.partials.as<double>(),
                              all.partials.as<double>(), PHASE_A);
            if (e == hipSuccess) e = enqueue_image(all, KIND_TRIAL);
            if (e == hipSuccess)
                e = launch_scalar(ns, stream, all.refs.as<SolveRef>(), d_ns,
                                  all.partials.as<double>(), all.partials.as<double>(), PHASE_B);
            if (e == hipSuccess) e = enqueue_image(all, KIND_UPCURV);
        }
        std::vector<SReq *> done;
        for (SReq *r : active) {
            r->passes += n_ep;
            if (r->passes >= r->req.params.n_iter) done.push_back(r);
        }
        // results of finished solves: current iterate into the caller's buffer
        for (SReq *r : done) {
            if (e != hipSuccess) break;
            const int idx = (int)(std::find(active.begin(), active.end(), r) - active.begin());
            (void)idx;
            for (size_t j = 0; j < all.pl.projs.size(); ++j)
                if (all.pl.projs[j].st == r->st_dev)
                    e = launch_finalize(stream, all.projs.as<Proj>() + j, 1,
                                        (int)r->req.params.img_dtype);
            if (e == hipSuccess && !r->req.on_device)
                e = hipMemcpyAsync(r->req.x_out, r->xwork.p, r->n * r->es, hipMemcpyDeviceToHost,
                                   stream);
        }
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        for (SReq *r : done) {
            ScgState st;
            misr_status code = MISR_E_HIP;
            if (e == hipSuccess &&
                hipMemcpy(&st, r->st_dev, sizeof st, hipMemcpyDeviceToHost) == hipSuccess) {
                code = st.stop == 2 ? MISR_E_NUMERIC : MISR_OK;
                r->stats.n_passes = st.it;
                r->stats.n_success = st.n_success;
                r->stats.E_final = st.E;
            }
            active.erase(std::find(active.begin(), active.end(), r));
            release(r);
            finish(r, code == MISR_OK ? MISR_REQ_DONE : MISR_REQ_FAILED, code);
        }
        if (e != hipSuccess) {
            // a device error fails every running request
            std::vector<SReq *> rs = active;
            active.clear();
            for (SReq *r : rs) {
                release(r);
                finish(r, MISR_REQ_FAILED, MISR_E_HIP);
            }
        }
    }
}

// ---------------------------------------------------------------- C ABI
extern "C" misr_status misr_server_create(misr_ctx *ctx, const misr_server_config *cfg,
                                          misr_server **out) {
    if (!ctx || !cfg || !out) return set_error(MISR_E_INVAL, "NULL argument");
    if (cfg->max_slots < 1 || cfg->hbm_budget_bytes == 0)
        return set_error(MISR_E_INVAL, "max_slots >= 1 and hbm_budget_bytes > 0 required");
    *out = nullptr;
    if (hipSetDevice(ctx->dev) != hipSuccess) return set_error(MISR_E_HIP, "hipSetDevice");
    auto s = std::make_unique<misr_server>();
    s->ctx = ctx;
    s->cfg = *cfg;
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
        return set_error(MISR_E_HIP, "stream creation failed");
    misr_server *raw = s.release();
    ctx->users++;
    raw->th = std::thread([raw] { raw->run(); });
    *out = raw;
    return MISR_OK;
}

extern "C" misr_status misr_server_submit(misr_server *s, const misr_request *req,
                                          uint64_t *id) {
    if (!s || !req || !id) return set_error(MISR_E_INVAL, "NULL argument");
    misr_status st = misr_geometry_check(&req->geom);
    if (st != MISR_OK) return st;
    if ((st = misr_params_check(&req->params)) != MISR_OK) return st;
    if (req->params.data_p != 2 || req->params.tile_lr > 0)
        return set_error(MISR_E_INVAL, "served solves: L2 data term, untiled");
    if (!req->y || !req->x0 || !req->x_out) return set_error(MISR_E_INVAL, "NULL buffer");
    auto r = std::make_unique<SReq>();
    r->req = *req;
    r->shifts.assign(req->geom.shifts_lr, req->geom.shifts_lr + 2 * req->geom.n_frames);
    r->psf.assign(req->geom.psf_1d, req->geom.psf_1d + req->geom.psf_size);
    r->n = (long long)req->geom.hr_h * req->geom.hr_w;
    r->es = dtype_size(req->params.img_dtype);
    const long long m = (long long)(req->geom.hr_h / req->geom.scale) *
                        (req->geom.hr_w / req->geom.scale);
    r->bytes = request_bytes(*req, r->n, r->es, req->geom.n_frames, m);
    r->stats.t_submit_us = now_us();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->closing) return set_error(MISR_E_INVAL, "server is shutting down");
    if (s->cfg.max_queue > 0 && (int)s->queue.size() >= s->cfg.max_queue)
        return set_error(MISR_E_BUSY, "queue full (%d)", s->cfg.max_queue);
    // every admitted request shares one storage type (one launch per class)
    for (auto &kv : s->reqs)
        if ((kv.second->state == MISR_REQ_QUEUED || kv.second->state == MISR_REQ_RUNNING) &&
            kv.second->req.params.img_dtype != req->params.img_dtype)
            return set_error(MISR_E_INVAL, "requests in flight use another img_dtype");
    r->id = s->next_id++;
    *id = r->id;
    s->queue.push_back(r.get());
    s->reqs.emplace(r->id, std::move(r));
    s->cv.notify_all();
    return MISR_OK;
}

extern "C" misr_status misr_server_poll(misr_server *s, uint64_t id, misr_req_state *state,
                                        misr_req_stats *stats) {
    if (!s) return set_error(MISR_E_INVAL, "NULL server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return set_error(MISR_E_NOTFOUND, "unknown request %llu",
                                              (unsigned long long)id);
    if (state) *state = it->second->state;
    if (stats) *stats = it->second->stats;
    return MISR_OK;
}

extern "C" misr_status misr_server_wait(misr_server *s, uint64_t id, int64_t timeout_us) {
    if (!s) return set_error(MISR_E_INVAL, "NULL server");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return set_error(MISR_E_NOTFOUND, "unknown request %llu",
                                              (unsigned long long)id);
    SReq *r = it->second.get();
    auto pending = [&] {
        return r->state == MISR_REQ_QUEUED || r->state == MISR_REQ_RUNNING;
    };
    if (timeout_us < 0)
        s->cv_done.wait(lk, [&] { return !pending(); });
    else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us),
                                  [&] { return !pending(); }))
        return set_error(MISR_E_TIMEOUT, "request %llu still pending", (unsigned long long)id);
    return MISR_OK;
}

extern "C" misr_status misr_server_cancel(misr_server *s, uint64_t id) {
    if (!s) return set_error(MISR_E_INVAL, "NULL server");
    SReq *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = s->reqs.find(id);
        if (it == s->reqs.end())
            return set_error(MISR_E_NOTFOUND, "unknown request %llu", (unsigned long long)id);
        r = it->second.get();
        if (r->state == MISR_REQ_QUEUED) {
            s->queue.erase(std::find(s->queue.begin(), s->queue.end(), r));
            r->state = MISR_REQ_CANCELLED;
            r->stats.status = MISR_E_CANCELLED;
            r->stats.t_done_us = now_us();
        } else if (r->state == MISR_REQ_RUNNING) {
            r->cancel = true;
            r = nullptr;
        } else {
            r = nullptr;
        }
    }
    s->cv_done.notify_all();
    if (r && r->req.done_cb) r->req.done_cb(r->id, MISR_E_CANCELLED, r->req.user);
    return MISR_OK;
}

extern "C" misr_status misr_server_destroy(misr_server *s) {
    if (!s) return set_error(MISR_E_INVAL, "NULL server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->closing = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    for (auto &kv : s->ops) misr_op_destroy(kv.second);
    (void)hipStreamDestroy(s->stream);
    misr_ctx *ctx = s->ctx;
    delete s;
    ctx->users--;
    return MISR_OK;
}
