// abi.cpp -- the C ABI of libmisr.so: validation, operator construction,
// workspace management and the device-resident SCG solve driver.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>

#include "runtime.h"

using namespace misr;

namespace misr {

static thread_local std::string g_err;

misr_status set_error(misr_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

misr_status hip_fail(hipError_t e, const char *what) {
    return set_error(e == hipErrorOutOfMemory ? MISR_E_NOMEM : MISR_E_HIP, "%s: %s", what,
                     hipGetErrorString(e));
}

size_t dtype_size(misr_dtype dt) { return dt == MISR_F32 ? 4 : 2; }

hipError_t PlanDev::upload(Plan &pl, int n_iter, hipStream_t stream) {
    hipError_t e;
    const size_t np = pl.projs.size(), ni = pl.items.size(), ns = pl.states.size();
    if ((e = projs.ensure(np * sizeof(Proj))) != hipSuccess) return e;
    if ((e = items.ensure(ni * sizeof(Item))) != hipSuccess) return e;
    if ((e = counts.ensure(pl.counts.size() * sizeof(int))) != hipSuccess) return e;
    if ((e = states.ensure(ns * sizeof(ScgState))) != hipSuccess) return e;
    if ((e = partials.ensure(ni * kNV * sizeof(double))) != hipSuccess) return e;
    if ((e = refs.ensure(ns * sizeof(SolveRef))) != hipSuccess) return e;
    // per-pass records of each solve (only solves write them)
    const size_t per = (size_t)(n_iter > 0 ? n_iter : 0);
    if (per > 0 && (e = traces.ensure(ns * per * sizeof(IterRec))) != hipSuccess) return e;
    n_iter_max = (int)per;
    ScgState *sd = states.as<ScgState>();
    for (size_t j = 0; j < np; ++j) pl.projs[j].st = sd + pl.proj_solve[j];
    pl.refs.resize(ns);
    for (size_t i = 0; i < ns; ++i)
        pl.refs[i] = SolveRef{sd + i, per ? traces.as<IterRec>() + i * per : nullptr,
                              pl.item0[i], pl.nitems[i]};
    if ((e = hipMemcpyAsync(projs.p, pl.projs.data(), np * sizeof(Proj), hipMemcpyHostToDevice,
                            stream)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(items.p, pl.items.data(), ni * sizeof(Item), hipMemcpyHostToDevice,
                            stream)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(counts.p, pl.counts.data(), pl.counts.size() * sizeof(int),
                            hipMemcpyHostToDevice, stream)) != hipSuccess)
        return e;
    if ((e = hipMemcpyAsync(refs.p, pl.refs.data(), ns * sizeof(SolveRef),
                            hipMemcpyHostToDevice, stream)) != hipSuccess)
        return e;
    return hipMemcpyAsync(states.p, pl.states.data(), ns * sizeof(ScgState),
                          hipMemcpyHostToDevice, stream);
}

}  // namespace misr

// ------------------------------------------------------------------- checks
static bool finite_pos(double v) { return std::isfinite(v) && v > 0; }

extern "C" const char *misr_last_error(void) { return g_err.c_str(); }

extern "C" void misr_params_default(misr_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->lambda_reg = 0.01;
    p->alpha_btv = 0.4;
    p->eps = 1e-3;
    p->btv_w = 3;
    p->data_p = 2;
    p->eps_data = 1e-3;
    p->scg_sigma = 1e-4;
    p->scg_lambda1 = 1e-6;
    p->n_iter = 50;
    p->img_dtype = MISR_F32;
    p->tile_lr = 0;
    p->halo_lr = 8;
}

static int band_length(const misr_geometry *g) {
    bool frac = false;
    for (int k = 0; k < g->n_frames; ++k)
        for (int a = 0; a < 2; ++a) {
            const double t = g->scale * g->shifts_lr[2 * k + a];
            if (t != std::floor(t)) frac = true;
        }
    return g->scale + g->psf_size - (frac ? 0 : 1);
}

extern "C" misr_status misr_geometry_check(const misr_geometry *g) {
    if (!g) return set_error(MISR_E_INVAL, "geometry is NULL");
    if (g->scale < 1 || g->scale > 4)
        return set_error(MISR_E_INVAL, "scale %d outside [1, 4]", g->scale);
    if (g->hr_h < 1 || g->hr_w < 1 || g->hr_h % g->scale || g->hr_w % g->scale)
        return set_error(MISR_E_INVAL, "HR size %dx%d must be positive and divisible by s=%d",
                         g->hr_h, g->hr_w, g->scale);
    if ((long long)g->hr_h * g->hr_w >= (1LL << 31))
        return set_error(MISR_E_INVAL, "HR image too large (>= 2^31 pixels)");
    if (g->n_frames < 1 || g->n_frames > kMaxK)
        return set_error(MISR_E_INVAL, "n_frames %d outside [1, %d]", g->n_frames, kMaxK);
    if (!g->shifts_lr) return set_error(MISR_E_INVAL, "shifts_lr is NULL");
    for (int i = 0; i < 2 * g->n_frames; ++i)
        if (!std::isfinite(g->shifts_lr[i]) || std::fabs(g->shifts_lr[i]) > 1.0)
            return set_error(MISR_E_INVAL, "shift %d (%g) not finite or |shift| > 1 LR px", i,
                             g->shifts_lr[i]);
    if (g->psf_size < 1 || g->psf_size > 15 || g->psf_size % 2 == 0)
        return set_error(MISR_E_INVAL, "psf_size %d must be odd in [1, 15]", g->psf_size);
    if (!g->psf_1d) return set_error(MISR_E_INVAL, "psf_1d is NULL");
    for (int i = 0; i < g->psf_size; ++i)
        if (!std::isfinite(g->psf_1d[i]))
            return set_error(MISR_E_INVAL, "psf tap %d not finite", i);
    const int L = band_length(g);
    const int Lp = padded_band(g->scale, L);
    if (Lp < 0)
        return set_error(MISR_E_INVAL, "band length %d unsupported at scale %d", L, g->scale);
    // the update/curvature window needs every frame's band start within
    // [-EXT, s-1] relative to the tile (EXT = max(Lp-1, 2))
    const int EXT = Lp - 1 > 2 ? Lp - 1 : 2;
    const int R = (g->psf_size - 1) / 2;
    for (int k = 0; k < g->n_frames; ++k)
        for (int a = 0; a < 2; ++a) {
            const int off = (int)std::floor(g->scale * g->shifts_lr[2 * k + 1 - a]) - R;
            if (off < -EXT || off > g->scale - 1)
                return set_error(MISR_E_INVAL, "frame %d shift moves the band outside the "
                                 "supported window", k);
        }
    return MISR_OK;
}

extern "C" misr_status misr_params_check(const misr_params *p) {
    if (!p) return set_error(MISR_E_INVAL, "params is NULL");
    if (!std::isfinite(p->lambda_reg) || p->lambda_reg < 0)
        return set_error(MISR_E_INVAL, "lambda_reg must be finite and >= 0");
    if (!(p->alpha_btv > 0 && p->alpha_btv < 1))
        return set_error(MISR_E_INVAL, "alpha_btv must lie in (0, 1)");
    if (!std::isfinite(p->eps) || p->eps < 0) return set_error(MISR_E_INVAL, "eps must be >= 0");
    if (p->btv_w < 1 || p->btv_w > 3) return set_error(MISR_E_INVAL, "btv_w must be in [1, 3]");
    if (p->data_p != 1 && p->data_p != 2) return set_error(MISR_E_INVAL, "data_p must be 1 or 2");
    if (!std::isfinite(p->eps_data) || p->eps_data < 0)
        return set_error(MISR_E_INVAL, "eps_data must be >= 0");
    if (!finite_pos(p->scg_sigma)) return set_error(MISR_E_INVAL, "scg_sigma must be > 0");
    if (!finite_pos(p->scg_lambda1)) return set_error(MISR_E_INVAL, "scg_lambda1 must be > 0");
    if (p->n_iter < 0) return set_error(MISR_E_INVAL, "n_iter must be >= 0");
    if (p->img_dtype != MISR_F32 && p->img_dtype != MISR_F16 && p->img_dtype != MISR_BF16)
        return set_error(MISR_E_INVAL, "img_dtype invalid");
    if (p->tile_lr < 0 || p->halo_lr < 0)
        return set_error(MISR_E_INVAL, "tile_lr and halo_lr must be >= 0");
    if (p->x_rounding != 0 && p->x_rounding != 1)
        return set_error(MISR_E_INVAL, "x_rounding must be 0 or 1");
    return MISR_OK;
}

// -------------------------------------------------------------------- ctx
extern "C" misr_status misr_ctx_create(int dev, misr_ctx **out) {
    if (!out) return set_error(MISR_E_INVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) return set_error(MISR_E_HIP, "no HIP device available");
    if (dev < 0 || dev >= n) return set_error(MISR_E_INVAL, "device %d outside [0, %d)", dev, n);
    MISR_HIP(hipSetDevice(dev));
    hipDeviceProp_t prop;
    MISR_HIP(hipGetDeviceProperties(&prop, dev));
    auto *c = new misr_ctx();
    c->dev = dev;
    c->ncu = prop.multiProcessorCount;
    if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming) != hipSuccess) {
        delete c;
        return set_error(MISR_E_HIP, "stream/event creation failed");
    }
    *out = c;
    return MISR_OK;
}

extern "C" misr_status misr_ctx_destroy(misr_ctx *c) {
    if (!c) return set_error(MISR_E_INVAL, "ctx is NULL");
    (void)hipStreamSynchronize(c->stream);
    (void)hipEventDestroy(c->ev_in);
    (void)hipEventDestroy(c->ev_out);
    (void)hipStreamDestroy(c->stream);
    delete c;
    return MISR_OK;
}

static hipError_t set_device(int dev) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    return cur == dev ? hipSuccess : hipSetDevice(dev);
}

// --------------------------------------------------------------------- op
// One axis of A_k = C_y (x) C_x: LR index i reads HR samples
// s*i + off + l, l in [0, Lp).  Built from the three 1-D factors in FP64:
// bilinear translation by t HR px (zero outside [0, N)), "same" convolution
// with the taps (zero padding), mean over s samples.
static void band_weights(int N, int s, double t, int P, const double *psf, int Lp, int off,
                         float *out) {
    const int R = (P - 1) / 2;
    const double fl = std::floor(t), f = t - fl;
    const int ifl = (int)fl;
    std::vector<double> acc((size_t)Lp);
    for (int i = 0; i < N / s; ++i) {
        std::fill(acc.begin(), acc.end(), 0.0);
        for (int b = 0; b < s; ++b) {
            const int u = s * i + b;                // output of the blur, inside [0, N)
            for (int a = -R; a <= R; ++a) {
                const int z = u - a;                // blur input = warp output index
                if (z < 0 || z >= N) continue;      // warp output exists on [0, N) only
                for (int e = 0; e < 2; ++e) {
                    const double wgt = e ? f : 1.0 - f;
                    const int v = z + ifl + e;      // HR sample read by the warp
                    if (wgt == 0.0 || v < 0 || v >= N) continue;
                    acc[v - (s * i + off)] += psf[a + R] * wgt / s;
                }
            }
        }
        for (int l = 0; l < Lp; ++l) out[(size_t)i * Lp + l] = (float)acc[l];
    }
}

extern "C" misr_status misr_op_create(misr_ctx *ctx, const misr_geometry *g, misr_op **out) {
    if (!ctx || !out) return set_error(MISR_E_INVAL, "ctx/out is NULL");
    *out = nullptr;
    misr_status st = misr_geometry_check(g);
    if (st != MISR_OK) return st;
    MISR_HIP(set_device(ctx->dev));
    auto op = std::make_unique<misr_op>();
    op->ctx = ctx;
    op->H = g->hr_h;
    op->W = g->hr_w;
    op->s = g->scale;
    op->K = g->n_frames;
    op->P = g->psf_size;
    op->L = band_length(g);
    op->Lp = padded_band(op->s, op->L);
    op->TH = tile_hr(op->s, op->Lp);
    op->TW = tile_wr(op->s, op->Lp);
    op->shifts.assign(g->shifts_lr, g->shifts_lr + 2 * g->n_frames);
    op->psf.assign(g->psf_1d, g->psf_1d + g->psf_size);
    const int h = op->H / op->s, w = op->W / op->s, R = (op->P - 1) / 2;
    const size_t fy = (size_t)(h + 2 * kPadRows) * op->Lp, fx = (size_t)(w + 2 * kPadRows) * op->Lp;
    std::vector<float> wy((size_t)op->K * fy, 0.f), wx((size_t)op->K * fx, 0.f);
    OpDev &hd = op->host;
    std::memset(&hd, 0, sizeof hd);
    for (int k = 0; k < op->K; ++k) {
        const double tx = op->s * op->shifts[2 * k], ty = op->s * op->shifts[2 * k + 1];
        hd.offy[k] = (int)std::floor(ty) - R;
        hd.offx[k] = (int)std::floor(tx) - R;
        band_weights(op->H, op->s, ty, op->P, op->psf.data(), op->Lp, hd.offy[k],
                     wy.data() + k * fy + (size_t)kPadRows * op->Lp);
        band_weights(op->W, op->s, tx, op->P, op->psf.data(), op->Lp, hd.offx[k],
                     wx.data() + k * fx + (size_t)kPadRows * op->Lp);
    }
    MISR_HIP(op->wy.ensure(wy.size() * 4));
    MISR_HIP(op->wx.ensure(wx.size() * 4));
    MISR_HIP(op->opdev.ensure(sizeof(OpDev)));
    MISR_HIP(hipMemcpy(op->wy.p, wy.data(), wy.size() * 4, hipMemcpyHostToDevice));
    MISR_HIP(hipMemcpy(op->wx.p, wx.data(), wx.size() * 4, hipMemcpyHostToDevice));
    hd.wy = op->wy.as<float>() + (size_t)kPadRows * op->Lp;
    hd.wx = op->wx.as<float>() + (size_t)kPadRows * op->Lp;
    hd.H = op->H;
    hd.W = op->W;
    hd.s = op->s;
    hd.K = op->K;
    hd.L = op->Lp;
    MISR_HIP(hipMemcpy(op->opdev.p, &hd, sizeof hd, hipMemcpyHostToDevice));
    *out = op.release();
    return MISR_OK;
}

extern "C" misr_status misr_op_destroy(misr_op *op) {
    if (!op) return set_error(MISR_E_INVAL, "op is NULL");
    (void)set_device(op->ctx->dev);
    (void)hipStreamSynchronize(op->ctx->stream);
    delete op;
    return MISR_OK;
}

extern "C" int misr_op_band(const misr_op *op) { return op ? op->L : -1; }

// ------------------------------------------------------------- plan build
static void init_state(ScgState &s, const misr_params &p, long long N) {
    std::memset(&s, 0, sizeof s);
    s.lam = p.scg_lambda1;
    s.lam_bar = 0.0;
    s.sigma = p.scg_sigma;
    s.N = N;
    s.n_iter = p.n_iter;
    s.success = 1;
    s.active = 1;
    for (int dy = 0; dy < 3; ++dy)
        for (int dx = 0; dx < 3; ++dx)
            s.wt.gam[dy * 3 + dx] = (dx == 0 && dy == 0) || dx >= p.btv_w || dy >= p.btv_w
                                        ? 0.f
                                        : (float)(p.lambda_reg * std::pow(p.alpha_btv, dx + dy));
    s.wt.eps = (float)p.eps;
    s.wt.eps_data = (float)p.eps_data;
    s.wt.data_p = p.data_p;
    s.wt.x_rounding = p.x_rounding;
}

struct SolveIn {
    const misr_op *op;
    misr_params prm;
    const void *y;
    void *x;
    SolveBufs *bufs;
};

// Builds the work list: solves grouped by kernel class (S, Lp), each solve's
// tiles contiguous so that its partial sums form one range.
static void build_plan(Plan &pl, const std::vector<SolveIn> &in) {
    pl.projs.clear();
    pl.items.clear();
    pl.states.clear();
    pl.classes.clear();
    pl.counts.clear();
    pl.proj_solve.clear();
    pl.item0.assign(in.size(), 0);
    pl.nitems.assign(in.size(), 0);
    std::map<std::pair<int, int>, std::vector<int>> groups;
    std::vector<std::pair<int, int>> order;
    for (int i = 0; i < (int)in.size(); ++i) {
        auto key = std::make_pair(in[i].op->s, in[i].op->Lp);
        if (!groups.count(key)) order.push_back(key);
        groups[key].push_back(i);
    }
    pl.states.resize(in.size());
    for (auto &key : order) {
        Plan::Cls c{key.first, key.second, (int)pl.items.size(), 0};
        for (int i : groups[key]) {
            const SolveIn &s = in[i];
            const misr_op *op = s.op;
            Proj P;
            std::memset(&P, 0, sizeof P);
            P.x[0] = s.x;
            P.x[1] = s.bufs->x1.p;
            P.p[0] = s.bufs->p0.as<float>();
            P.p[1] = s.bufs->p1.as<float>();
            P.g[0] = s.bufs->g0.as<float>();
            P.g[1] = s.bufs->g1.as<float>();
            P.y = s.y;
            P.ld = op->W;
            P.Hb = op->H;
            P.Wb = op->W;
            P.oy1 = op->H;
            P.ox1 = op->W;
            P.ntx = (op->W + op->TW - 1) / op->TW;
            P.op = op->opdev.as<OpDev>();
            const int nty = (op->H + op->TH - 1) / op->TH;
            const int pj = (int)pl.projs.size();
            pl.projs.push_back(P);
            pl.proj_solve.push_back(i);
            init_state(pl.states[i], s.prm, (long long)op->H * op->W);
            pl.item0[i] = (int)pl.items.size();
            for (int ty = 0; ty < nty; ++ty)
                for (int tx = 0; tx < P.ntx; ++tx) pl.items.push_back(Item{pj, ty, tx, 0});
            pl.nitems[i] = (int)pl.items.size() - pl.item0[i];
        }
        c.count = (int)pl.items.size() - c.start;
        pl.classes.push_back(c);
    }
    for (auto &c : pl.classes) pl.counts.push_back(c.count);
    pl.counts.push_back((int)pl.states.size());
}

static std::string plan_key(const Plan &pl, int n_iter, int stype) {
    std::string k = std::to_string(n_iter) + "/" + std::to_string(stype) + "/" +
                     std::to_string(pl.states.size()) + "/" + std::to_string(pl.projs.size());
    for (auto &c : pl.classes)
        k += ":" + std::to_string(c.S) + "," + std::to_string(c.Lp) + "," +
             std::to_string(c.start) + "," + std::to_string(c.count);
    return k;
}

// Enqueues the whole solve (init + n_iter passes + final copy) on `s`.
static hipError_t enqueue_solve(const Plan &pl, PlanDev &pd, int n_iter, int stype,
                                hipStream_t s) {
    const int nc = (int)pl.classes.size();
    const int ns = (int)pl.states.size();
    const int *d_counts = pd.counts.as<int>();
    const int *d_nstates = d_counts + nc;
    auto image = [&](int kind) -> hipError_t {
        for (int c = 0; c < nc; ++c) {
            const Plan::Cls &cl = pl.classes[c];
            hipError_t e = launch_image(cl.S, cl.Lp, cl.count, s, pd.projs.as<Proj>(),
                                        pd.items.as<Item>() + cl.start, d_counts + c,
                                        pd.partials.as<double>() + (size_t)cl.start * kNV, kind,
                                        stype);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    };
    auto scalar = [&](int phase) {
        return launch_scalar(ns, s, pd.refs.as<SolveRef>(), d_nstates, pd.partials.as<double>(),
                             phase);
    };
    hipError_t e;
    if ((e = image(KIND_COSTGRAD)) != hipSuccess) return e;
    if ((e = scalar(PHASE_INIT)) != hipSuccess) return e;
    if ((e = image(KIND_UPCURV)) != hipSuccess) return e;
    for (int it = 0; it < n_iter; ++it) {
        if ((e = scalar(PHASE_A)) != hipSuccess) return e;
        if ((e = image(KIND_TRIAL)) != hipSuccess) return e;
        if ((e = scalar(PHASE_B)) != hipSuccess) return e;
        if ((e = image(KIND_UPCURV)) != hipSuccess) return e;
    }
    return launch_finalize(s, pd.projs.as<Proj>(), (int)pl.projs.size(), stype);
}

// Runs a plan on the context's library stream, ordered after the caller's
// stream and before its later work; the solve is captured into a graph once
// per plan shape and replayed.
static misr_status run_plan(misr_ctx *ctx, Plan &pl, PlanDev &pd, int n_iter, int stype,
                            hipStream_t user) {
    hipStream_t s = ctx->stream;
    MISR_HIP(hipEventRecord(ctx->ev_in, user));
    MISR_HIP(hipStreamWaitEvent(s, ctx->ev_in, 0));
    MISR_HIP(pd.upload(pl, n_iter, s));
    // the graph bakes in the device addresses of the plan arrays
    char ptrs[160];
    snprintf(ptrs, sizeof ptrs, "|%p,%p,%p,%p,%p,%p", pd.projs.p, pd.items.p, pd.counts.p,
             pd.states.p, pd.partials.p, pd.refs.p);
    const std::string key = plan_key(pl, n_iter, stype) + ptrs;
    if (!pd.exec || pd.graph_key != key) {
        if (pd.exec) {
            (void)hipGraphExecDestroy(pd.exec);
            pd.exec = nullptr;
        }
        hipGraph_t graph = nullptr;
        MISR_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        hipError_t e = enqueue_solve(pl, pd, n_iter, stype, s);
        hipError_t e2 = hipStreamEndCapture(s, &graph);
        if (e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return hip_fail(e, "enqueue_solve (capture)");
        }
        if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
        e = hipGraphInstantiate(&pd.exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            pd.exec = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
        pd.graph_key = key;
    }
    MISR_HIP(hipGraphLaunch(pd.exec, s));
    MISR_HIP(hipEventRecord(ctx->ev_out, s));
    MISR_HIP(hipStreamWaitEvent(user, ctx->ev_out, 0));
    return MISR_OK;
}

static misr_status fetch_trace(const Plan &pl, PlanDev &pd, int idx, misr_scg_trace *tr,
                               hipStream_t user) {
    ScgState st;
    MISR_HIP(hipMemcpyAsync(&st, pd.states.as<ScgState>() + idx, sizeof st, hipMemcpyDeviceToHost,
                            user));
    MISR_HIP(hipStreamSynchronize(user));
    tr->n_passes = st.it;
    tr->n_success = st.n_success;
    tr->stop = st.stop;
    tr->E0 = st.E0;
    tr->E_final = st.E;
    if (tr->iters && tr->capacity > 0 && st.it > 0) {
        const int n = st.it < tr->capacity ? st.it : tr->capacity;
        static_assert(sizeof(IterRec) == sizeof(misr_scg_iter), "trace record layout");
        MISR_HIP(hipMemcpy(tr->iters, pd.traces.as<IterRec>() + (size_t)idx * pd.n_iter_max,
                           n * sizeof(IterRec), hipMemcpyDeviceToHost));
    }
    (void)pl;
    return st.stop == 2 ? set_error(MISR_E_NUMERIC, "non-finite cost or curvature at pass %d",
                                    st.it)
                        : MISR_OK;
}

// ------------------------------------------------------------ operators
static misr_status single_view(misr_op *op, const void *x, Plan &pl) {
    SolveIn si{op, {}, nullptr, const_cast<void *>(x), &op->bufs};
    misr_params_default(&si.prm);
    si.prm.n_iter = 0;
    build_plan(pl, {si});
    return MISR_OK;
}

extern "C" misr_status misr_forward(const misr_op *cop, misr_dtype dt, const void *x, void *y,
                                    void *stream) {
    misr_op *op = const_cast<misr_op *>(cop);
    if (!op || !x || !y) return set_error(MISR_E_INVAL, "NULL argument");
    if (dt != MISR_F32 && dt != MISR_F16 && dt != MISR_BF16)
        return set_error(MISR_E_INVAL, "dtype invalid");
    std::lock_guard<std::mutex> lk(op->mu);
    MISR_HIP(set_device(op->ctx->dev));
    Plan &pl = op->plan;
    single_view(op, x, pl);
    PlanDev &pd = op->pdev;
    hipStream_t s = (hipStream_t)stream;
    MISR_HIP(pd.upload(pl, 0, s));
    MISR_HIP(launch_forward(op->s, op->Lp, (int)pl.items.size(), s, pd.projs.as<Proj>(),
                            pd.items.as<Item>(), (int)pl.items.size(), (int)dt, y));
    return MISR_OK;
}

extern "C" misr_status misr_adjoint(const misr_op *cop, misr_dtype dt, const void *r, float *x,
                                    void *stream) {
    misr_op *op = const_cast<misr_op *>(cop);
    if (!op || !x || !r) return set_error(MISR_E_INVAL, "NULL argument");
    if (dt != MISR_F32 && dt != MISR_F16 && dt != MISR_BF16)
        return set_error(MISR_E_INVAL, "dtype invalid");
    std::lock_guard<std::mutex> lk(op->mu);
    MISR_HIP(set_device(op->ctx->dev));
    Plan &pl = op->plan;
    single_view(op, x, pl);
    PlanDev &pd = op->pdev;
    hipStream_t s = (hipStream_t)stream;
    MISR_HIP(pd.upload(pl, 0, s));
    MISR_HIP(launch_adjoint(op->s, op->Lp, (int)pl.items.size(), s, pd.projs.as<Proj>(),
                            pd.items.as<Item>(), (int)pl.items.size(), (int)dt, r, x));
    return MISR_OK;
}

extern "C" misr_status misr_cost_grad(const misr_op *cop, const misr_params *prm, const void *x,
                                      const void *y, float *g, double *cost_dev, void *stream) {
    misr_op *op = const_cast<misr_op *>(cop);
    if (!op || !x || !y || !g || !cost_dev) return set_error(MISR_E_INVAL, "NULL argument");
    misr_status st = misr_params_check(prm);
    if (st != MISR_OK) return st;
    if (prm->tile_lr > 0) return set_error(MISR_E_INVAL, "tiled cost_grad not available");
    std::lock_guard<std::mutex> lk(op->mu);
    MISR_HIP(set_device(op->ctx->dev));
    const size_t es = dtype_size(prm->img_dtype);
    const long long n = (long long)op->H * op->W;
    MISR_HIP(op->bufs.ensure(n, es));
    Plan &pl = op->plan;
    SolveIn si{op, *prm, y, const_cast<void *>(x), &op->bufs};
    si.prm.n_iter = 0;
    build_plan(pl, {si});
    pl.projs[0].g[1] = g;   // the init pass writes g[cur ^ 1] with cur = 0
    PlanDev &pd = op->pdev;
    hipStream_t s = (hipStream_t)stream;
    MISR_HIP(pd.upload(pl, 0, s));
    const Plan::Cls &cl = pl.classes[0];
    MISR_HIP(launch_image(cl.S, cl.Lp, cl.count, s, pd.projs.as<Proj>(), pd.items.as<Item>(),
                          pd.counts.as<int>(), pd.partials.as<double>(), KIND_COSTGRAD,
                          (int)prm->img_dtype));
    MISR_HIP(launch_cost_out(s, pd.partials.as<double>(), cl.count, cost_dev));
    return MISR_OK;
}

// ----------------------------------------------------------------- solves
extern "C" misr_status misr_scg_solve(const misr_op *cop, const misr_params *prm, const void *y,
                                      void *x, misr_scg_trace *trace, void *stream) {
    misr_op *op = const_cast<misr_op *>(cop);
    if (!op || !y || !x) return set_error(MISR_E_INVAL, "NULL argument");
    misr_status st = misr_params_check(prm);
    if (st != MISR_OK) return st;
    if (prm->data_p != 2)
        return set_error(MISR_E_INVAL, "the SCG solve supports the L2 data term (data_p = 2)");
    if (prm->tile_lr > 0) return set_error(MISR_E_INVAL, "tiled solve not available");
    std::lock_guard<std::mutex> lk(op->mu);
    std::lock_guard<std::mutex> lc(op->ctx->mu);
    MISR_HIP(set_device(op->ctx->dev));
    const long long n = (long long)op->H * op->W;
    MISR_HIP(op->bufs.ensure(n, dtype_size(prm->img_dtype)));
    Plan &pl = op->plan;
    build_plan(pl, {SolveIn{op, *prm, y, x, &op->bufs}});
    hipStream_t s = (hipStream_t)stream;
    st = run_plan(op->ctx, pl, op->pdev, prm->n_iter, (int)prm->img_dtype, s);
    if (st != MISR_OK) return st;
    if (trace) return fetch_trace(pl, op->pdev, 0, trace, s);
    return MISR_OK;
}

namespace {
struct BatchCache {
    std::vector<const misr_op *> ops;
    std::vector<std::unique_ptr<SolveBufs>> bufs;
    PlanDev pdev;
    Plan plan;
};
std::mutex g_batch_mu;
BatchCache *g_batch = nullptr;
}  // namespace

extern "C" misr_status misr_scg_solve_batch(int n, const misr_op *const *ops,
                                            const misr_params *prm, const void *const *y,
                                            void *const *x, misr_scg_trace *traces,
                                            void *stream) {
    if (n < 1 || !ops || !prm || !y || !x) return set_error(MISR_E_INVAL, "bad batch arguments");
    misr_ctx *ctx = nullptr;
    for (int i = 0; i < n; ++i) {
        if (!ops[i] || !y[i] || !x[i]) return set_error(MISR_E_INVAL, "NULL entry %d", i);
        misr_status st = misr_params_check(&prm[i]);
        if (st != MISR_OK) return st;
        if (prm[i].data_p != 2 || prm[i].tile_lr > 0)
            return set_error(MISR_E_INVAL, "batch entry %d: L2 data term, untiled only", i);
        if (prm[i].img_dtype != prm[0].img_dtype)
            return set_error(MISR_E_INVAL, "batch entries must share img_dtype");
        if (ctx && ops[i]->ctx != ctx) return set_error(MISR_E_INVAL, "ops span contexts");
        ctx = ops[i]->ctx;
    }
    std::lock_guard<std::mutex> lk(g_batch_mu);
    std::lock_guard<std::mutex> lc(ctx->mu);
    MISR_HIP(set_device(ctx->dev));
    if (!g_batch) g_batch = new BatchCache();
    BatchCache &bc = *g_batch;
    std::vector<const misr_op *> key(ops, ops + n);
    if (bc.ops != key) {
        bc.bufs.clear();
        bc.ops = key;
    }
    int n_iter = 0;
    for (int i = 0; i < n; ++i) n_iter = std::max(n_iter, prm[i].n_iter);
    std::vector<SolveIn> in;
    const size_t es = dtype_size(prm[0].img_dtype);
    for (int i = 0; i < n; ++i) {
        if ((int)bc.bufs.size() <= i) bc.bufs.emplace_back(new SolveBufs());
        MISR_HIP(bc.bufs[i]->ensure((long long)ops[i]->H * ops[i]->W, es));
        in.push_back(SolveIn{ops[i], prm[i], y[i], x[i], bc.bufs[i].get()});
    }
    build_plan(bc.plan, in);
    hipStream_t s = (hipStream_t)stream;
    misr_status st = run_plan(ctx, bc.plan, bc.pdev, n_iter, (int)prm[0].img_dtype, s);
    if (st != MISR_OK) return st;
    misr_status worst = MISR_OK;
    if (traces)
        for (int i = 0; i < n; ++i) {
            misr_status t = fetch_trace(bc.plan, bc.pdev, i, &traces[i], s);
            if (t != MISR_OK) worst = t;
        }
    return worst;
}

// ------------------------------------------------------------- measurement
extern "C" misr_status misr_time_pass(const misr_op *cop, const misr_params *prm, const void *y,
                                      void *x, int which, int reps, double *avg_us,
                                      void *stream) {
    misr_op *op = const_cast<misr_op *>(cop);
    if (!op || !y || !x || !avg_us || reps < 1 || (which != 0 && which != 1))
        return set_error(MISR_E_INVAL, "bad arguments");
    misr_status st = misr_params_check(prm);
    if (st != MISR_OK) return st;
    if (prm->data_p != 2 || prm->tile_lr > 0)
        return set_error(MISR_E_INVAL, "L2 data term, untiled only");
    std::lock_guard<std::mutex> lk(op->mu);
    std::lock_guard<std::mutex> lc(op->ctx->mu);
    MISR_HIP(set_device(op->ctx->dev));
    const long long n = (long long)op->H * op->W;
    MISR_HIP(op->bufs.ensure(n, dtype_size(prm->img_dtype)));
    Plan &pl = op->plan;
    misr_params p1 = *prm;
    p1.n_iter = 1;
    build_plan(pl, {SolveIn{op, p1, y, x, &op->bufs}});
    PlanDev &pd = op->pdev;
    hipStream_t s = op->ctx->stream;
    MISR_HIP(hipEventRecord(op->ctx->ev_in, (hipStream_t)stream));
    MISR_HIP(hipStreamWaitEvent(s, op->ctx->ev_in, 0));
    MISR_HIP(pd.upload(pl, 1, s));
    const Plan::Cls &cl = pl.classes[0];
    const int stype = (int)prm->img_dtype;
    auto image = [&](int kind) {
        return launch_image(cl.S, cl.Lp, cl.count, s, pd.projs.as<Proj>(), pd.items.as<Item>(),
                            pd.counts.as<int>(), pd.partials.as<double>(), kind, stype);
    };
    auto scalar = [&](int phase) {
        return launch_scalar(1, s, pd.refs.as<SolveRef>(), pd.counts.as<int>() + 1,
                             pd.partials.as<double>(), phase);
    };
    MISR_HIP(image(KIND_COSTGRAD));
    MISR_HIP(scalar(PHASE_INIT));
    MISR_HIP(image(KIND_UPCURV));
    MISR_HIP(scalar(PHASE_A));
    hipEvent_t e0, e1;
    MISR_HIP(hipEventCreate(&e0));
    MISR_HIP(hipEventCreate(&e1));
    const int kind = which == 0 ? KIND_TRIAL : KIND_UPCURV;
    hipError_t e = image(kind);   // warm-up launch
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = image(kind);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return hip_fail(e, "misr_time_pass");
    *avg_us = 1e3 * ms / reps;
    return MISR_OK;
}
