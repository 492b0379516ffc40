// server.cpp -- continuous-batching serving of SR solves (misr_server_*).
//
// The paper super-resolves each rotation angle's frames as soon as they are
// captured, reusing the system matrices built once per acquisition (Sec. 3.2).
// Here every request is one such solve.  A scheduler thread admits queued
// requests while device memory (a byte budget) and slots allow, keeps each
// admitted solve's SCG state resident on the device, and advances all admitted
// solves together: every SCG pass of every solve runs in the same kernel
// launches over one work list of (view, tile) items, so requests that arrive
// while others run join at the next pass boundary.  Each solve keeps its own
// state and reductions (fixed order per solve), so its result does not depend
// on which other solves share the launches, nor on the cycles it sits out
// when the server orders the admitted solves (shortest or earliest finish
// first).
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
    int H, W, s, K, P, ell;
    std::vector<double> shifts, psf, psf_frames, warps, psf_2d;
    bool operator<(const OpKey &o) const {
        return std::tie(H, W, s, K, P, ell, shifts, psf, psf_frames, warps, psf_2d) <
               std::tie(o.H, o.W, o.s, o.K, o.P, o.ell, o.shifts, o.psf, o.psf_frames, o.warps,
                        o.psf_2d);
    }
};

// A cached operator: the requests admitted on it hold references; with none
// it is idle and may be evicted (least recently used first).  Every request
// that used it has retired, so none of the work still in flight reads its
// tables; its destruction waits for the device all the same.
struct OpEnt {
    misr_op *op = nullptr;
    int refs = 0;
    size_t bytes = 0;        // device bytes of its tables, charged to admission
    uint64_t last_use = 0;
};

struct SReq {
    uint64_t id = 0;
    misr_request req{};
    std::vector<double> shifts, psf, psf_frames, warps, psf_2d;   // geometry copies
    OpKey key;            // its operator's cache key
    OpEnt *ope = nullptr; // the cache entry it holds a reference on (admitted only)
    size_t op_bytes = 0;  // estimate of its operator's tables, if not cached
    misr_req_state state = MISR_REQ_QUEUED;
    misr_req_stats stats{};
    bool cancel = false;
    misr_op *op = nullptr;
    size_t bytes = 0;
    long long n = 0;      // HR pixels
    size_t es = 4;
    int passes = 0;       // passes enqueued
    bool fresh = true;    // init not yet enqueued
    bool sel = false;     // advanced by the cycle being built
    // device memory owned by the server for this request
    DevMem xwork, ydev, dstate;
    SolveBufs bufs;
    TileSet tiles;        // tiled requests (params.tile_lr > 0): per-tile buffers
    bool tiled = false;
    bool staged = false;  // iterate in library views: tiled, or FP32 over a 16-bit x
    int view0 = 0, nviews = 0;   // its views in the current work list
    void *x0dev = nullptr;
    const void *ydev_ptr = nullptr;
    ScgState *st_dev = nullptr;
    IterRec *trace_dev = nullptr;
    ScgState *h_st = nullptr;     // pinned host slot: initial state up, final state down
    // outcome for a request retired without a result (cancelled, failed set-up)
    misr_req_state drop_state = MISR_REQ_FAILED;
    misr_status drop_code = MISR_E_HIP;
    void set_pool(MemPool *pl) {
        xwork.pool = ydev.pool = dstate.pool = pl;
        bufs.set_pool(pl);
        tiles.pool = pl;
    }
};

// Pinned host staging buffer (grown on demand).
struct Pinned {
    void *h = nullptr;
    size_t cap = 0;
    ~Pinned() {
        if (h) (void)hipHostFree(h);
    }
    bool ensure(size_t n) {
        if (n <= cap && h) return true;
        if (h) (void)hipHostFree(h);
        h = nullptr;
        cap = 0;
        if (hipHostMalloc(&h, n, hipHostMallocDefault) != hipSuccess) return false;
        cap = n;
        return true;
    }
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
    int list_count = 0;           // work-list builds (fault hook fail_list_n)
    std::map<OpKey, OpEnt> ops;   // guarded by mu
    uint64_t use_clock = 0;
    int n_idle = 0;
    // work list of all active solves; per class, the running solves' items
    // come first and the newly admitted ones' after, so that the init passes
    // of the new solves run over a sub-range of each class.
    // Device counts: [0,nc) trial items per class, [nc,2nc) update items per
    // class, 2nc solves, 2nc+1 halo copies, then the same four for the new
    // solves only at offset 2nc+2.
    struct List {
        Plan pl;
        std::vector<int> nb, nbu;            // per class: first trial / update item of the new solves
        std::vector<SolveRef> refs_new;      // the new solves only
        std::vector<HaloCopy> halos_new;     // halo copies of the new solves only
        std::vector<int> counts;
        // device copies of the arrays above, all in one block (one upload)
        struct View {
            void *p = nullptr;
            template <typename T>
            T *as() const { return (T *)p; }
        } projs, items, items_u, counts_d, refs, drefs_new, halos, halos_new_d;
        DevMem blob, partials, partials_u;
        Pinned stage;                        // the packed arrays, pinned for the upload
        int nc() const { return (int)pl.classes.size(); }
        const int *cnt(int off) const { return counts_d.as<int>() + off; }
    };
    // A cycle: the passes enqueued for the admitted solves in one scheduler
    // step.  Two cycles alternate: while one runs on the device the scheduler
    // builds and enqueues the next, then retires the first; so the device
    // does not idle at cycle boundaries and a cycle's buffers are rewritten
    // only after it has completed.
    struct Cycle {
        List list;
        hipEvent_t ev0 = nullptr, ev1 = nullptr;   // start and end of its work
        bool pending = false;
        hipError_t err = hipSuccess;
        int n_ep = 0;
        double mpx = 0;                            // HR Mpx advanced per pass
        std::vector<SReq *> done, dropped;
    } cyc[2];
    MemPool pool;                 // request buffers, reused across requests
    Pinned slots_mem;             // pinned ScgState slots, one per admitted request
    std::vector<ScgState *> free_slots;
    double us_per_mpx_pass = 40.0;   // running estimate of the device time per pass
    std::string last_error;

    void run();
    void retire(Cycle &C);
    bool setup(SReq *r);
    void release(SReq *r);
    hipError_t build_list(List &L, const std::vector<SReq *> &rs);
    // idle operators evicted (caller holds mu) until at most keep remain idle
    // and, if need > 0, until used + need fits the budget; the operators of
    // the requests being admitted (spare) are kept
    void evict_idle(int keep, size_t need, const std::vector<SReq *> *spare = nullptr);
    int max_idle() const { return cfg.max_idle_ops > 0 ? cfg.max_idle_ops : 8; }
    hipError_t enqueue_init(List &L, const std::vector<SReq *> &rs);
    hipError_t enqueue_image(List &L, int kind, bool fresh);
    hipError_t enqueue_scalar(List &L, int phase, bool fresh);
    hipError_t enqueue_halo(List &L, bool fresh);
    // storage code of the image launches (every admitted request shares
    // img_dtype and x_work)
    int launch_code() const {
        if (active.empty()) return st_code(ST_F32, ST_F32);
        const misr_params &p = active[0]->req.params;
        return st_code(view_stype(p), frame_stype(p));
    }
    void finish(SReq *r, misr_req_state st, misr_status code);
};

// Device bytes a request holds while admitted.  A tiled request keeps every
// tile (halo included) with its own x pair, p pair and g pair; an FP32
// iterate over a 16-bit image adds an FP32 copy of x0.
static size_t request_bytes(const misr_request &q, long long n, size_t es, int K, long long m) {
    const size_t ev = view_esize(q.params);
    size_t b = 0;
    if (q.params.tile_lr > 0) {
        const int s = q.geom.scale, H = q.geom.hr_h, W = q.geom.hr_w;
        const int T = q.params.tile_lr * s, Hh = q.params.halo_lr * s;
        for (int a = 0; a * T < H; ++a)
            for (int c = 0; c * T < W; ++c) {
                const long long rows = std::min(H, (a + 1) * T + Hh) - std::max(0, a * T - Hh);
                const long long cols = std::min(W, (c + 1) * T + Hh) - std::max(0, c * T - Hh);
                b += (size_t)(rows * cols) * (ev * 2 + 16);
            }
    } else {
        b = (size_t)n * ev * 2 + (size_t)n * 16;           // x pair, p pair, g pair
    }
    if (!q.on_device)   // y and x staged on device
        b += (size_t)K * m * (q.params.y_u16 ? 2 : es) + (size_t)n * es;
    b += sizeof(ScgState) + (size_t)std::max(1, q.params.n_iter) * sizeof(IterRec);
    return b;
}

// Device bytes of a request's share of the work lists: its trial and update
// items (an Item and kNV FP64 partial sums each), views and halo copies, in
// each of the two alternating cycles' lists.  Server operators keep tile
// variant 0.
static size_t list_bytes(const misr_request &q, bool general) {
    const int H = q.geom.hr_h, W = q.geom.hr_w, s = q.geom.scale, K = q.geom.n_frames;
    long long ni = 0, nu = 0, nviews = 1, nhalo = 0;
    auto cd = [](long long a, long long b) { return (a + b - 1) / b; };
    if (general) {
        ni = nu = general_mf_plan(&q.geom, nullptr, nullptr)
                      ? mf_lr_tiles(H, W, s, K) + mf_hr_tiles(H, W)
                      : cd((long long)K * (H / s) * (W / s), kGenRows) +
                            cd((long long)H * W, kGenRows);
    } else {
        const int Lp = padded_band(s, band_length(&q.geom));
        const int TH = tile_hr(s, Lp), TW = tile_wr(s, Lp), TWt = tile_wt(s, Lp);
        if (TH <= 0 || TW <= 0 || TWt <= 0) return 0;   // rejected at op creation
        if (q.params.tile_lr <= 0) {
            ni = cd(H, TH) * cd(W, TWt);
            nu = cd(H, TH) * cd(W, TW);
        } else {
            const int T = q.params.tile_lr * s, Hh = q.params.halo_lr * s;
            nviews = 0;
            for (int a = 0; a * T < H; ++a)
                for (int c = 0; c * T < W; ++c) {
                    const int R0 = a * T, R1 = std::min(H, R0 + T), C0 = c * T,
                              C1 = std::min(W, C0 + T);
                    const int hb = std::min(H, R1 + Hh) - std::max(0, R0 - Hh);
                    const int wb = std::min(W, C1 + Hh) - std::max(0, C0 - Hh);
                    ni += cd(R1 - R0, TH) * cd(C1 - C0, TWt);
                    nu += cd(hb, TH) * cd(wb, TW);
                    ++nviews;
                }
            nhalo = 8 * nviews;
        }
    }
    const size_t per = (size_t)(ni + nu) * (sizeof(Item) + kNV * sizeof(double)) +
                       (size_t)nviews * sizeof(Proj) + (size_t)nhalo * 2 * sizeof(HaloCopy) +
                       2 * sizeof(SolveRef);
    return 2 * per;
}

// Device bytes of an operator's tables before it is built: the banded
// factors' weight rows, a matrix-free general operator's blur-and-bin
// kernels, or the sparse A and A^T of a stored general geometry (at most
// (P + s + 2)^2 entries of 8 B per LR pixel and frame, each way).
static size_t op_bytes_estimate(const misr_geometry &g, bool general) {
    const long long h = g.hr_h / g.scale, w = g.hr_w / g.scale;
    if (general && general_mf_plan(&g, nullptr, nullptr)) {
        const long long Q = g.scale + g.psf_size - 1;
        return (size_t)(4 * Q * Q * g.n_frames) + sizeof(OpDev);
    }
    if (general) {
        const long long e = (long long)(g.psf_size + g.scale + 2) * (g.psf_size + g.scale + 2);
        return (size_t)(2 * 8 * e * g.n_frames * h * w) + sizeof(OpDev);
    }
    const int Lp = padded_band(g.scale, band_length(&g));
    int pad_y = 0, pad_x = 0;
    band_pad_after(g.scale, Lp, pad_y, pad_x);
    return (size_t)g.n_frames * (size_t)(h + w + 2 * kPadRows + pad_y + pad_x) *
               (size_t)std::max(Lp, 1) * 4 + sizeof(OpDev);
}

// Device bytes an operator holds.
static size_t op_bytes(const misr_op *op) {
    return op->wy.n + op->wx.n + op->opdev.n + op->a_col.n + op->a_val.n + op->t_col.n +
           op->t_val.n + op->gker.n;
}

void misr_server::evict_idle(int keep, size_t need, const std::vector<SReq *> *spare) {
    auto kept = [&](const OpKey &k) {
        if (spare)
            for (const SReq *r : *spare)
                if (!(r->key < k) && !(k < r->key)) return true;
        return false;
    };
    while (n_idle > 0) {
        const bool over = n_idle > keep;
        const bool short_mem = need > 0 && used + need > cfg.hbm_budget_bytes;
        if (!over && !short_mem) return;
        auto lru = ops.end();
        for (auto it = ops.begin(); it != ops.end(); ++it) {
            if (it->second.refs != 0 || kept(it->first)) continue;
            if (lru == ops.end() || it->second.last_use < lru->second.last_use) lru = it;
        }
        if (lru == ops.end()) return;
        used -= std::min(used, lru->second.bytes);
        // a device error seen here also fails the next cycle's launches
        (void)misr_op_destroy(lru->second.op);
        ops.erase(lru);
        --n_idle;
    }
}

bool misr_server::setup(SReq *r) {
    const misr_request &q = r->req;
    if (cfg.fail_alloc_n > 0 && ++alloc_count == cfg.fail_alloc_n) return false;
    misr_geometry g = q.geom;
    g.shifts_lr = r->shifts.empty() ? nullptr : r->shifts.data();
    g.psf_1d = r->psf.empty() ? nullptr : r->psf.data();
    g.psf_frames = r->psf_frames.empty() ? nullptr : r->psf_frames.data();
    g.warps = r->warps.empty() ? nullptr : r->warps.data();
    g.psf_2d = r->psf_2d.empty() ? nullptr : r->psf_2d.data();
    {
        std::unique_lock<std::mutex> lk(mu);
        auto it = ops.find(r->key);
        if (it == ops.end()) {
            lk.unlock();   // building a general operator takes a while
            misr_op *op = nullptr;
            if (misr_op_create(ctx, &g, &op) != MISR_OK) return false;
            lk.lock();
            OpEnt ent;
            ent.op = op;
            ent.bytes = op_bytes(op);
            used += ent.bytes;
            it = ops.emplace(r->key, ent).first;
        } else if (it->second.refs == 0) {
            --n_idle;
        }
        it->second.refs++;
        it->second.last_use = ++use_clock;
        r->ope = &it->second;
        r->op = it->second.op;
    }
    if (r->tiled && (check_tiling(r->op, q.params) != MISR_OK ||
                     ensure_tiles(r->op, q.params, r->tiles) != hipSuccess))
        return false;
    const long long m = (long long)(g.hr_h / g.scale) * (g.hr_w / g.scale) * g.n_frames;
    if (!r->tiled && r->bufs.ensure_view(r->n, q.params) != hipSuccess) return false;
    if (r->op->general && r->bufs.res.ensure((size_t)kGenVecs * m * 4) != hipSuccess)
        return false;
    const size_t per = (size_t)std::max(1, q.params.n_iter);
    if (r->dstate.ensure(sizeof(ScgState) + per * sizeof(IterRec)) != hipSuccess) return false;
    r->st_dev = r->dstate.as<ScgState>();
    r->trace_dev = (IterRec *)(r->dstate.as<char>() + sizeof(ScgState));
    if (q.on_device) {
        r->x0dev = q.x_out;
        r->ydev_ptr = q.y;
        if (q.x0 && q.x0 != q.x_out &&
            hipMemcpyAsync(q.x_out, q.x0, r->n * r->es, hipMemcpyDeviceToDevice, stream) !=
                hipSuccess)
            return false;
    } else {
        if (r->xwork.ensure(r->n * r->es) != hipSuccess) return false;
        const size_t ye = q.params.y_u16 ? 2 : r->es;   // frame element size
        if (r->ydev.ensure(m * ye) != hipSuccess) return false;
        r->x0dev = r->xwork.p;
        r->ydev_ptr = r->ydev.p;
        if ((q.x0 && hipMemcpyAsync(r->xwork.p, q.x0, r->n * r->es, hipMemcpyHostToDevice,
                                    stream) != hipSuccess) ||
            hipMemcpyAsync(r->ydev.p, q.y, m * ye, hipMemcpyHostToDevice, stream) !=
                hipSuccess)
            return false;
    }
    if (free_slots.empty()) return false;
    r->h_st = free_slots.back();
    free_slots.pop_back();
    ScgState &st = *r->h_st;
    init_state(st, q.params, r->n);
    if (r->staged) {
        st.xglob = r->x0dev;     // scattered into the views at init, gathered at the end
        st.ldg = g.hr_w;
    }
    // the slot stays untouched until the final state comes back into it
    return hipMemcpyAsync(r->st_dev, r->h_st, sizeof st, hipMemcpyHostToDevice, stream) ==
           hipSuccess;
}

void misr_server::release(SReq *r) {
    if (r->h_st) free_slots.push_back(r->h_st);
    r->h_st = nullptr;
    r->xwork.release();
    r->ydev.release();
    r->dstate.release();
    r->bufs.x1.release();
    r->bufs.p0.release();
    r->bufs.p1.release();
    r->bufs.g0.release();
    r->bufs.g1.release();
    r->bufs.x0w.release();
    r->bufs.res.release();
    r->tiles.bufs.clear();
    r->tiles.x0.clear();
    std::lock_guard<std::mutex> lk(mu);
    used -= std::min(used, r->bytes);
    if (r->ope) {
        if (--r->ope->refs == 0) {
            r->ope->last_use = ++use_clock;
            ++n_idle;
        }
        r->ope = nullptr;
        evict_idle(max_idle(), 0);
    }
}

hipError_t misr_server::build_list(List &L, const std::vector<SReq *> &rs) {
    Plan &pl = L.pl;
    pl.projs.clear();
    pl.items.clear();
    pl.items_u.clear();
    pl.classes.clear();
    pl.classes_u.clear();
    pl.refs.clear();
    pl.halos.clear();
    L.nb.clear();
    L.nbu.clear();
    L.refs_new.clear();
    L.halos_new.clear();
    std::map<std::pair<int, int>, std::vector<SReq *>> groups;
    std::vector<std::pair<int, int>> order;
    for (int pass = 0; pass < 2; ++pass)       // running solves first, then new ones
        for (SReq *r : rs) {
            if (r->fresh != (pass == 1)) continue;
            auto key = std::make_pair(r->op->s, r->op->kernel_key());
            if (!groups.count(key)) order.push_back(key);
            groups[key].push_back(r);
        }
    for (auto &key : order) {
        Plan::Cls c{key.first, key.second, (int)pl.items.size(), 0};
        Plan::Cls cu{key.first, key.second, (int)pl.items_u.size(), 0};
        int nb = -1, nbu = -1;
        for (SReq *r : groups[key]) {
            if (r->fresh && nb < 0) {
                nb = (int)pl.items.size();
                nbu = (int)pl.items_u.size();
            }
            const int i0 = (int)pl.items.size(), iu0 = (int)pl.items_u.size();
            const size_t h0 = pl.halos.size();
            r->view0 = (int)pl.projs.size();
            add_views(r->op, r->req.params, r->ydev_ptr, r->x0dev, &r->bufs, &r->tiles, pl.projs,
                      pl.items, pl.items_u, pl.halos);
            r->nviews = (int)pl.projs.size() - r->view0;
            for (int j = r->view0; j < (int)pl.projs.size(); ++j) pl.projs[j].st = r->st_dev;
            pl.refs.push_back(SolveRef{r->st_dev, r->trace_dev, i0, (int)pl.items.size() - i0,
                                       iu0, (int)pl.items_u.size() - iu0});
            if (r->fresh) {
                L.refs_new.push_back(pl.refs.back());
                L.halos_new.insert(L.halos_new.end(), pl.halos.begin() + h0, pl.halos.end());
            }
        }
        c.count = (int)pl.items.size() - c.start;
        cu.count = (int)pl.items_u.size() - cu.start;
        pl.classes.push_back(c);
        pl.classes_u.push_back(cu);
        L.nb.push_back(nb < 0 ? (int)pl.items.size() : nb);
        L.nbu.push_back(nbu < 0 ? (int)pl.items_u.size() : nbu);
    }
    const int nc = L.nc();
    L.counts.clear();
    for (auto &c : pl.classes) L.counts.push_back(c.count);
    for (auto &c : pl.classes_u) L.counts.push_back(c.count);
    L.counts.push_back((int)pl.refs.size());
    L.counts.push_back((int)pl.halos.size());
    for (int c = 0; c < nc; ++c)
        L.counts.push_back(pl.classes[c].start + pl.classes[c].count - L.nb[c]);
    for (int c = 0; c < nc; ++c)
        L.counts.push_back(pl.classes_u[c].start + pl.classes_u[c].count - L.nbu[c]);
    L.counts.push_back((int)L.refs_new.size());
    L.counts.push_back((int)L.halos_new.size());
    const size_t np = pl.projs.size(), ni = pl.items.size(), nu = pl.items_u.size(),
                 ns = pl.refs.size(), nh = pl.halos.size(), nhn = L.halos_new.size();
    struct Up {
        List::View *d;
        const void *h;
        size_t n;
    } ups[] = {{&L.projs, pl.projs.data(), np * sizeof(Proj)},
               {&L.items, pl.items.data(), ni * sizeof(Item)},
               {&L.items_u, pl.items_u.data(), nu * sizeof(Item)},
               {&L.counts_d, L.counts.data(), L.counts.size() * sizeof(int)},
               {&L.refs, pl.refs.data(), ns * sizeof(SolveRef)},
               {&L.drefs_new, L.refs_new.data(), L.refs_new.size() * sizeof(SolveRef)},
               {&L.halos, pl.halos.data(), nh * sizeof(HaloCopy)},
               {&L.halos_new_d, L.halos_new.data(), nhn * sizeof(HaloCopy)}};
    size_t total = 0;
    for (auto &u : ups) total += (u.n + 255) & ~(size_t)255;
    total = std::max<size_t>(total, 256);
    if (cfg.fail_list_n > 0 && ++list_count == cfg.fail_list_n) return hipErrorOutOfMemory;
    if (!L.stage.ensure(total)) return hipErrorOutOfMemory;
    hipError_t e = L.blob.ensure(total);
    if (e == hipSuccess) e = L.partials.ensure(std::max<size_t>(ni, 1) * kNV * sizeof(double));
    if (e == hipSuccess) e = L.partials_u.ensure(std::max<size_t>(nu, 1) * kNV * sizeof(double));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return e;
    }
    char *hp = (char *)L.stage.h, *dp = L.blob.as<char>();
    for (auto &u : ups) {
        if (u.n) std::memcpy(hp, u.h, u.n);
        u.d->p = dp;
        const size_t step = (u.n + 255) & ~(size_t)255;
        hp += step;
        dp += step;
    }
    return hipMemcpyAsync(L.blob.p, L.stage.h, (size_t)(hp - (char *)L.stage.h),
                          hipMemcpyHostToDevice, stream);
}

// Image pass over the whole list (fresh = false) or over the new solves' tail
// of each class (fresh = true).
hipError_t misr_server::enqueue_image(List &L, int kind, bool fresh) {
    const int nc = L.nc();
    const bool upd = kind == KIND_UPCURV;
    const auto &cls = upd ? L.pl.classes_u : L.pl.classes;
    const Item *items = upd ? L.items_u.as<Item>() : L.items.as<Item>();
    double *part = upd ? L.partials_u.as<double>() : L.partials.as<double>();
    const int code = launch_code();
    for (int c = 0; c < nc; ++c) {
        const int first = fresh ? (upd ? L.nbu[c] : L.nb[c]) : cls[c].start;
        const int n = cls[c].start + cls[c].count - first;
        if (n <= 0) continue;
        const int cidx = (fresh ? 2 * nc + 2 : 0) + (upd ? nc : 0) + c;
        // band length 0: the class of general operators
        hipError_t e =
            cls[c].Lp == 0
                ? launch_general(n, stream, L.projs.as<Proj>(), items + first, L.cnt(cidx),
                                 part + (size_t)first * kNV, kind, cls[c].S)
                : launch_image(cls[c].S, cls[c].Lp, n, stream, L.projs.as<Proj>(), items + first,
                               L.cnt(cidx), part + (size_t)first * kNV, kind, code);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t misr_server::enqueue_scalar(List &L, int phase, bool fresh) {
    const int nc = L.nc();
    const int n = fresh ? (int)L.refs_new.size() : (int)L.pl.refs.size();
    if (n == 0) return hipSuccess;
    return launch_scalar(n, stream, fresh ? L.drefs_new.as<SolveRef>() : L.refs.as<SolveRef>(),
                         L.cnt((fresh ? 2 * nc + 2 : 0) + 2 * nc), L.partials.as<double>(),
                         L.partials_u.as<double>(), phase);
}

hipError_t misr_server::enqueue_halo(List &L, bool fresh) {
    const int nc = L.nc();
    const size_t n = fresh ? L.halos_new.size() : L.pl.halos.size();
    if (n == 0) return hipSuccess;
    return launch_halo(stream, L.projs.as<Proj>(),
                       fresh ? L.halos_new_d.as<HaloCopy>() : L.halos.as<HaloCopy>(),
                       L.cnt((fresh ? 2 * nc + 2 : 0) + 2 * nc + 1), (int)n);
}

// Init of the newly admitted solves over their sub-range of the list: start
// points computed on the device where asked for; tiled ones scatter x0 into
// their tiles; cost and gradient at x0 (and its halo
// exchange), Moller's init, update pass (p = -g0) with curvature, then steps
// 1-5 of their first pass.
hipError_t misr_server::enqueue_init(List &L, const std::vector<SReq *> &rs) {
    hipError_t e = hipSuccess;
    for (SReq *r : rs)   // start points computed on the device
        if (e == hipSuccess && r->fresh && r->req.params.x_init > 0)
            e = launch_init(stream, r->req.params.x_init, init_args(r->op), r->ydev_ptr,
                            r->x0dev, (int)r->req.params.img_dtype);
    for (SReq *r : rs)
        if (e == hipSuccess && r->fresh && r->staged)
            e = launch_scatter(stream, L.projs.as<Proj>() + r->view0, r->nviews,
                               view_stype(r->req.params), (int)r->req.params.img_dtype);
    if (e == hipSuccess) e = enqueue_image(L, KIND_COSTGRAD, true);
    if (e == hipSuccess) e = enqueue_halo(L, true);
    if (e == hipSuccess) e = enqueue_scalar(L, PHASE_INIT, true);
    if (e == hipSuccess) e = enqueue_image(L, KIND_UPCURV, true);
    if (e == hipSuccess) e = enqueue_scalar(L, PHASE_A, true);
    return e;
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

// Completion of a cycle: finished requests report their final state (copied
// into their pinned slot by the cycle), dropped ones their outcome; all give
// their buffers back.  The cycle's device time updates the pass estimate.
void misr_server::retire(Cycle &C) {
    const hipError_t e = C.err != hipSuccess ? C.err : hipEventSynchronize(C.ev1);
    if (e == hipSuccess && C.n_ep > 0 && C.mpx > 0) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, C.ev0, C.ev1) == hipSuccess && ms > 0.f) {
            const double est = ms * 1e3 / (C.n_ep * C.mpx);
            us_per_mpx_pass = 0.7 * us_per_mpx_pass + 0.3 * est;
        }
    }
    for (SReq *r : C.done) {
        misr_status code = MISR_E_HIP;
        if (e == hipSuccess) {
            const ScgState &st = *r->h_st;
            code = st.stop == 2 ? MISR_E_NUMERIC : MISR_OK;
            r->stats.n_passes = st.it;
            r->stats.n_success = st.n_success;
            r->stats.E_final = st.E;
        }
        release(r);
        finish(r, code == MISR_OK ? MISR_REQ_DONE : MISR_REQ_FAILED, code);
    }
    for (SReq *r : C.dropped) {
        release(r);
        finish(r, r->drop_state, r->drop_code);
    }
    C.done.clear();
    C.dropped.clear();
    C.pending = false;
    C.err = hipSuccess;
    C.n_ep = 0;
    C.mpx = 0;
}

void misr_server::run() {
    (void)hipSetDevice(ctx->dev);
    int cur = 0;
    for (;;) {
        std::vector<SReq *> admitted;
        Cycle &C = cyc[cur];          // retired: free to rebuild
        Cycle &P = cyc[cur ^ 1];      // possibly still on the device
        {
            std::unique_lock<std::mutex> lk(mu);
            cv.wait(lk, [&] {
                return closing || !queue.empty() || !active.empty() || P.pending;
            });
            if (closing && queue.empty() && active.empty() && !P.pending) break;
            // admission by free device memory, slots and host state slots,
            // first come first served (orders 1 and 2: fill_mpx then picks the
            // solves of each cycle instead of holding requests back)
            const int cap = std::min<int>(std::max(1, cfg.max_slots), (int)free_slots.size() +
                                                                           (int)active.size());
            double held_mpx = 0;   // HR pixels of the solves that will run next cycle
            for (SReq *r : active) held_mpx += r->n * 1e-6;
            while (!queue.empty() && (int)(active.size() + admitted.size()) < cap) {
                SReq *r = queue.front();
                if (cfg.order == 0 && cfg.fill_mpx > 0 && !(active.empty() && admitted.empty()) &&
                    held_mpx + r->n * 1e-6 > cfg.fill_mpx)
                    break;
                // its buffers, and its operator's tables unless cached
                const size_t need = r->bytes + (ops.count(r->key) ? 0 : r->op_bytes);
                if (used + need > cfg.hbm_budget_bytes) {
                    admitted.push_back(r);   // its operator, and those admitted before it, stay
                    evict_idle(0, need, &admitted);
                    admitted.pop_back();
                }
                if (used + need > cfg.hbm_budget_bytes) {
                    if (active.empty() && admitted.empty() && !P.pending) {
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
                held_mpx += r->n * 1e-6;
                r->state = MISR_REQ_RUNNING;
                r->stats.t_admit_us = now_us();
                admitted.push_back(r);
            }
            for (SReq *r : active)
                if (r->cancel) {
                    r->drop_state = MISR_REQ_CANCELLED;
                    r->drop_code = MISR_E_CANCELLED;
                    C.dropped.push_back(r);
                }
        }
        for (SReq *r : C.dropped) active.erase(std::find(active.begin(), active.end(), r));
        for (SReq *r : admitted) {
            r->set_pool(&pool);
            if (!setup(r)) {
                r->drop_state = MISR_REQ_FAILED;
                r->drop_code = MISR_E_NOMEM;
                C.dropped.push_back(r);
                continue;
            }
            active.push_back(r);
        }
        hipError_t e = hipSuccess;
        if (!active.empty()) {
            // the solves this cycle advances: all admitted ones, or those first
            // by the order's key, as many as fill_mpx holds: the work left
            // (shortest first), or the arrival time plus the device time the
            // work left takes at the current estimate (earliest finish first)
            std::vector<SReq *> run = active;
            if (cfg.order > 0 && cfg.fill_mpx > 0) {
                const double us_px = us_per_mpx_pass * 1e-6;
                auto key = [&](const SReq *r) {
                    const double left = (double)r->n * (r->req.params.n_iter - r->passes);
                    return cfg.order == 1 ? left : r->stats.t_submit_us + us_px * left;
                };
                std::stable_sort(run.begin(), run.end(),
                                 [&](const SReq *a, const SReq *b) { return key(a) < key(b); });
                std::vector<SReq *> pick;
                double m = 0;
                for (SReq *r : run)
                    if (pick.empty() || m + r->n * 1e-6 <= cfg.fill_mpx) {
                        pick.push_back(r);
                        m += r->n * 1e-6;
                    }
                run.swap(pick);
            }
            // passes this cycle: about 3 ms of device time, at most 64, and no
            // further than the earliest completion
            double mpx = 0;
            for (SReq *r : run) mpx += r->n * 1e-6;
            int n_ep = (int)(3000.0 / std::max(1e-3, us_per_mpx_pass * mpx));
            n_ep = std::max(1, std::min(64, n_ep));
            for (SReq *r : run) n_ep = std::min(n_ep, r->req.params.n_iter - r->passes);
            n_ep = std::max(n_ep, 0);
            if (build_list(C.list, run) != hipSuccess) {
                // no work list for this cycle: its requests fail before any launch
                for (SReq *r : active) {
                    r->drop_state = MISR_REQ_FAILED;
                    r->drop_code = MISR_E_NOMEM;
                    C.dropped.push_back(r);
                }
                active.clear();
                run.clear();
                n_ep = 0;
            }
            if (!run.empty()) e = hipEventRecord(C.ev0, stream);
            bool any_fresh = false;
            for (SReq *r : run) any_fresh |= r->fresh;
            if (e == hipSuccess && any_fresh) e = enqueue_init(C.list, run);
            for (SReq *r : run) r->fresh = false;
            // Each pass ends with steps 1-5 of the next one (phase A), so that
            // no partial sums outlive a cycle: the next cycle's list may place
            // a running solve's items elsewhere.  After a solve's last pass
            // phase A finds it inactive and changes nothing.
            List &L = C.list;
            for (int ep = 0; ep < n_ep && e == hipSuccess; ++ep) {
                e = enqueue_image(L, KIND_TRIAL, false);
                if (e == hipSuccess) e = enqueue_halo(L, false);
                if (e == hipSuccess) e = enqueue_scalar(L, PHASE_B, false);
                if (e == hipSuccess) e = enqueue_image(L, KIND_UPCURV, false);
                if (e == hipSuccess) e = enqueue_scalar(L, PHASE_A, false);
            }
            // finished solves: current iterate into the caller's buffer and the
            // final state into the request's pinned slot
            for (SReq *r : run) {
                r->passes += n_ep;
                r->sel = true;
            }
            std::vector<SReq *> still;
            for (SReq *r : active) {
                const bool sel = r->sel;
                r->sel = false;
                if (!sel || r->passes < r->req.params.n_iter) {
                    still.push_back(r);
                    continue;
                }
                const Proj *pv = L.projs.as<Proj>() + r->view0;
                const int vt = view_stype(r->req.params), gt = (int)r->req.params.img_dtype;
                if (e == hipSuccess)
                    e = r->staged ? launch_gather(stream, pv, r->nviews, vt, gt, 0)
                                  : launch_finalize(stream, pv, r->nviews, vt);
                if (e == hipSuccess && !r->req.on_device)
                    e = hipMemcpyAsync(r->req.x_out, r->xwork.p, r->n * r->es,
                                       hipMemcpyDeviceToHost, stream);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(r->h_st, r->st_dev, sizeof(ScgState),
                                       hipMemcpyDeviceToHost, stream);
                C.done.push_back(r);
            }
            active.swap(still);
            C.n_ep = n_ep;
            C.mpx = mpx;
        }
        if (e == hipSuccess && (!C.done.empty() || !C.dropped.empty() || C.n_ep > 0))
            e = hipEventRecord(C.ev1, stream);
        if (e != hipSuccess) {
            // a device error fails every request of this cycle and every running one
            C.err = e;
            for (SReq *r : active) {
                r->drop_state = MISR_REQ_FAILED;
                r->drop_code = MISR_E_HIP;
                C.dropped.push_back(r);
            }
            active.clear();
        }
        C.pending = !C.done.empty() || !C.dropped.empty() || C.n_ep > 0 || C.err != hipSuccess;
        if (P.pending) retire(P);
        if (C.pending && active.empty()) retire(C);   // nothing follows: finish now
        cur ^= 1;
    }
    if (cyc[0].pending) retire(cyc[0]);
    if (cyc[1].pending) retire(cyc[1]);
}

// ---------------------------------------------------------------- C ABI
extern "C" misr_status misr_server_create(misr_ctx *ctx, const misr_server_config *cfg,
                                          misr_server **out) {
    if (!ctx || !cfg || !out) return set_error(MISR_E_INVAL, "NULL argument");
    if (cfg->max_slots < 1 || cfg->hbm_budget_bytes == 0 || cfg->fill_mpx < 0)
        return set_error(MISR_E_INVAL,
                         "max_slots >= 1, hbm_budget_bytes > 0 and fill_mpx >= 0 required");
    if (cfg->max_idle_ops < 0) return set_error(MISR_E_INVAL, "max_idle_ops >= 0 required");
    if (cfg->order < 0 || cfg->order > 2) return set_error(MISR_E_INVAL, "order 0, 1 or 2 required");
    *out = nullptr;
    if (hipSetDevice(ctx->dev) != hipSuccess) return set_error(MISR_E_HIP, "hipSetDevice");
    auto s = std::make_unique<misr_server>();
    s->ctx = ctx;
    s->cfg = *cfg;
    auto undo = [&] {
        for (auto &c : s->cyc) {
            if (c.ev0) (void)hipEventDestroy(c.ev0);
            if (c.ev1) (void)hipEventDestroy(c.ev1);
        }
        if (s->stream) (void)hipStreamDestroy(s->stream);
    };
    if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess)
        return set_error(MISR_E_HIP, "stream creation failed");
    for (auto &c : s->cyc)
        if (hipEventCreate(&c.ev0) != hipSuccess || hipEventCreate(&c.ev1) != hipSuccess) {
            undo();
            return set_error(MISR_E_HIP, "event creation failed");
        }
    const int nslots = std::max(1, cfg->max_slots);
    if (!s->slots_mem.ensure((size_t)nslots * sizeof(ScgState))) {
        undo();
        return set_error(MISR_E_NOMEM, "pinned host memory for %d solve states", nslots);
    }
    for (int i = nslots - 1; i >= 0; --i)
        s->free_slots.push_back((ScgState *)s->slots_mem.h + i);
    s->pool.limit = cfg->hbm_budget_bytes;
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
    const bool general = req->geom.warps || req->geom.psf_2d;
    if (general && (req->params.img_dtype != MISR_F32 || req->params.y_u16 ||
                    req->params.tile_lr > 0 || req->params.x_init == 2))
        return set_error(MISR_E_INVAL, "general geometries (warps, psf_2d) are served with FP32 "
                         "images, untiled, x_init 0 or 1");
    if (!req->y || !req->x_out || (!req->x0 && req->params.x_init == 0))
        return set_error(MISR_E_INVAL, "NULL buffer (x0 may be NULL only with x_init > 0)");
    auto r = std::make_unique<SReq>();
    r->req = *req;
    const int K = req->geom.n_frames, P = req->geom.psf_size;
    if (req->geom.shifts_lr) r->shifts.assign(req->geom.shifts_lr, req->geom.shifts_lr + 2 * K);
    if (req->geom.psf_1d) r->psf.assign(req->geom.psf_1d, req->geom.psf_1d + P);
    if (req->geom.warps) r->warps.assign(req->geom.warps, req->geom.warps + 6 * K);
    if (req->geom.psf_2d) r->psf_2d.assign(req->geom.psf_2d, req->geom.psf_2d + (size_t)K * P * P);
    if (req->geom.psf_frames)
        r->psf_frames.assign(req->geom.psf_frames,
                             req->geom.psf_frames + 2 * (size_t)req->geom.n_frames *
                                                        req->geom.psf_size);
    r->n = (long long)req->geom.hr_h * req->geom.hr_w;
    r->tiled = req->params.tile_lr > 0;
    r->staged = r->tiled || iterate_fp32(req->params);
    r->es = dtype_size(req->params.img_dtype);
    const long long m = (long long)(req->geom.hr_h / req->geom.scale) *
                        (req->geom.hr_w / req->geom.scale);
    r->bytes = request_bytes(*req, r->n, r->es, req->geom.n_frames, m);
    if (general) r->bytes += (size_t)kGenVecs * m * K * 4;   // its LR vectors
    r->bytes += list_bytes(*req, general);
    r->op_bytes = op_bytes_estimate(req->geom, general);
    r->key = OpKey{req->geom.hr_h, req->geom.hr_w, req->geom.scale, K, P,
                   general ? req->geom.general_ell : 0, r->shifts, r->psf, r->psf_frames,
                   r->warps, r->psf_2d};
    r->stats.t_submit_us = now_us();
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->closing) return set_error(MISR_E_INVAL, "server is shutting down");
    if (s->cfg.max_queue > 0 && (int)s->queue.size() >= s->cfg.max_queue)
        return set_error(MISR_E_BUSY, "queue full (%d)", s->cfg.max_queue);
    // every admitted request shares one storage type (one launch per class)
    for (auto &kv : s->reqs)
        if ((kv.second->state == MISR_REQ_QUEUED || kv.second->state == MISR_REQ_RUNNING) &&
            (kv.second->req.params.img_dtype != req->params.img_dtype ||
             view_stype(kv.second->req.params) != view_stype(req->params) ||
             frame_stype(kv.second->req.params) != frame_stype(req->params)))
            return set_error(MISR_E_INVAL,
                             "requests in flight use another img_dtype, x_work or y_u16");
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
    if (stats) {
        *stats = it->second->stats;
        stats->bytes = it->second->bytes;
        stats->op_bytes = it->second->op_bytes;
    }
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

extern "C" misr_status misr_server_query(misr_server *s, misr_server_info *out) {
    if (!s || !out) return set_error(MISR_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(s->mu);
    out->queued = (int32_t)s->queue.size();
    int running = 0;
    for (auto &kv : s->reqs) running += kv.second->state == MISR_REQ_RUNNING;
    out->running = running;
    out->n_ops = (int32_t)s->ops.size();
    out->n_idle_ops = s->n_idle;
    out->used_bytes = s->used;
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
    // a device error raised by the server's work (or earlier work) is
    // reported by this call, after everything is freed
    const hipError_t sync_err = hipDeviceSynchronize();
    s->reqs.clear();   // their buffers went back to the pool when they retired
    for (auto &kv : s->ops) misr_op_destroy(kv.second.op);
    for (auto &c : s->cyc) {
        if (c.ev0) (void)hipEventDestroy(c.ev0);
        if (c.ev1) (void)hipEventDestroy(c.ev1);
    }
    (void)hipStreamDestroy(s->stream);
    misr_ctx *ctx = s->ctx;
    delete s;
    ctx->users--;
    if (sync_err != hipSuccess)
        return hip_fail(sync_err, "device error seen while destroying a server");
    return MISR_OK;
}
