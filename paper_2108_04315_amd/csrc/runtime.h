// runtime.h -- host-side runtime of libmisr.so (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <iterator>
#include <map>
#include <cstdarg>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/misr.h"
#include "internal.h"

namespace misr {

// launchers (kernels.hip)
int padded_band(int S, int L);
// tile shape of a kernel key (band length | variant << 8), -1 if none
int tile_hr(int S, int key);
int tile_wr(int S, int key);
// width of the trial kernel's tile (its own, wider shape for variant 0; the
// height is the same)
int tile_wt(int S, int key);
// code = st_code(storage of the views' x, storage of y).  grid must equal the
// item count (*n_items): the trial and update kernels run one workgroup per
// item.
hipError_t launch_image(int S, int Lp, int grid, hipStream_t stream, const Proj *projs,
                        const Item *items, const int *n_items, double *partials, int kind,
                        int code);
hipError_t launch_forward(int S, int Lp, int grid, hipStream_t stream, const Proj *projs,
                          const Item *items, int n, int stype, void *y);
hipError_t launch_adjoint(int S, int Lp, int grid, hipStream_t stream, const Proj *projs,
                          const Item *items, int n, int stype, const void *r, float *x);
// general operators (general_kernels.hip): one pass over a class of general
// items (kind as launch_image), and the standalone FP32 operators
hipError_t launch_general(int grid, hipStream_t stream, const Proj *projs, const Item *items,
                          const int *n_items, double *partials, int kind, int S);
// (mf_tiles > 0: a matrix-free operator, one workgroup per tile)
hipError_t launch_general_forward(hipStream_t stream, const OpDev *op, long long rows,
                                  const float *x, float *y, long long mf_tiles);
hipError_t launch_general_adjoint(hipStream_t stream, const OpDev *op, long long n,
                                  const float *r, float *x, long long mf_tiles);
hipError_t launch_scalar(int grid, hipStream_t stream, const SolveRef *refs, const int *n_refs,
                         const double *partials, const double *partials_u, int phase);
hipError_t launch_halo(hipStream_t stream, const Proj *projs, const HaloCopy *copies,
                       const int *n_copies, int grid);
hipError_t launch_scatter(hipStream_t stream, const Proj *projs, int nproj, int vt, int gt);
hipError_t launch_gather(hipStream_t stream, const Proj *projs, int nproj, int vt, int gt,
                         int which);
hipError_t launch_cost_out(hipStream_t stream, const double *partials, int nitems,
                           double *out);
hipError_t launch_fill(hipStream_t stream, float *p, long long n, float v);
hipError_t launch_finalize(hipStream_t stream, const Proj *projs, int nproj, int stype);
// start point into x (caller storage st): kind 1 bicubic of frame 0, 2 multi-image
// interpolation
hipError_t launch_init(hipStream_t stream, int kind, const InitArgs &a, const void *y, void *x,
                       int st);

enum { KIND_COSTGRAD = 0, KIND_TRIAL = 1, KIND_UPCURV = 2 };
enum { PHASE_INIT = 0, PHASE_A = 1, PHASE_B = 2 };

misr_status set_error(misr_status st, const char *fmt, ...);
misr_status hip_fail(hipError_t e, const char *what);
#define MISR_HIP(call)                                         \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return misr::hip_fail(e_, #call); \
    } while (0)

size_t dtype_size(misr_dtype dt);

// A device allocation owned by the library.
// Cache of device blocks for a stream-ordered user (the server): blocks are
// handed back instead of freed, so that requests of recurring sizes reuse
// them without hipMalloc / hipFree (hipFree waits for the whole device).
// Reuse is safe because every user of a pool enqueues on one stream.
struct MemPool {
    std::multimap<size_t, void *> free_;
    size_t held = 0;
    size_t limit = 0;   // bytes kept beyond which the largest blocks are freed
    static size_t round(size_t n) { return ((n ? n : 16) + (1u << 20) - 1) & ~(size_t)((1u << 20) - 1); }
    hipError_t get(void **p, size_t n) {
        n = round(n);
        auto it = free_.find(n);
        if (it != free_.end()) {
            *p = it->second;
            free_.erase(it);
            held -= n;
            return hipSuccess;
        }
        hipError_t e = hipMalloc(p, n);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            trim(0);
            e = hipMalloc(p, n);
        }
        return e;
    }
    void put(void *p, size_t n) {
        n = round(n);
        free_.emplace(n, p);
        held += n;
        if (held > limit) trim(limit);
    }
    void trim(size_t to) {
        while (held > to && !free_.empty()) {
            auto it = std::prev(free_.end());
            (void)hipFree(it->second);
            held -= it->first;
            free_.erase(it);
        }
    }
    ~MemPool() { trim(0); }
};

struct DevMem {
    void *p = nullptr;
    size_t n = 0;
    MemPool *pool = nullptr;   // blocks come from / go back to this cache if set
    DevMem() = default;
    DevMem(const DevMem &) = delete;
    DevMem &operator=(const DevMem &) = delete;
    ~DevMem() { release(); }
    void release() {
        if (p) {
            if (pool)
                pool->put(p, n);
            else
                (void)hipFree(p);
        }
        p = nullptr;
        n = 0;
    }
    hipError_t ensure(size_t bytes) {
        if (bytes <= n && p) return hipSuccess;
        release();
        hipError_t e = pool ? pool->get(&p, bytes) : hipMalloc(&p, bytes ? bytes : 16);
        if (e == hipSuccess) n = pool ? MemPool::round(bytes) : bytes;
        else p = nullptr;
        return e;
    }
    template <typename T>
    T *as() const { return (T *)p; }
};

// Work list and device state for a set of solves advanced together.  The
// trial pass walks `items` (owned tiles), the update pass `items_u` (owned
// plus halo; the same list when no view has a halo).
struct Plan {
    struct Cls {
        int S, Lp, start, count;
    };
    std::vector<Proj> projs;
    std::vector<Item> items, items_u;
    std::vector<ScgState> states;
    std::vector<Cls> classes, classes_u;
    std::vector<int> counts;          // trial classes, update classes, then n_states
    std::vector<int> proj_solve;      // solve index of each view
    std::vector<int> item0, nitems;   // per solve: its range of trial items
    std::vector<int> item0u, nitemsu; // per solve: its range of update items
    std::vector<SolveRef> refs;       // device-side references (filled by upload)
    std::vector<HaloCopy> halos;      // halo exchanges after each trial pass
    struct Init {                     // start points computed on the device
        int kind;
        InitArgs a;
        const void *y;
        void *x;
        int st;
    };
    std::vector<Init> inits;
    bool tiled = false;               // some solve is split into tiles
    bool staged = false;              // some solve's iterate lives in library views
                                      // (tiled, or FP32 over a 16-bit caller image)
    int vt = ST_F32, gt = ST_F32;     // storage of the views' x and of the caller's x
    int yt = ST_F32;                  // storage of the frames
    int code() const { return st_code(vt, yt); }
    void finish_counts() {
        counts.clear();
        for (auto &c : classes) counts.push_back(c.count);
        for (auto &c : classes_u) counts.push_back(c.count);
        counts.push_back((int)refs.size() > 0 ? (int)refs.size() : (int)states.size());
        counts.push_back((int)halos.size());
    }
    int n_states_idx() const { return (int)(classes.size() + classes_u.size()); }
};

// The iterate is FP32 in library buffers while the caller's x is 16-bit.
inline bool iterate_fp32(const misr_params &p) {
    return p.img_dtype != MISR_F32 && p.x_work == 0;
}
// Storage type of the views' x.
inline int view_stype(const misr_params &p) {
    return iterate_fp32(p) ? (int)ST_F32 : (int)p.img_dtype;
}
inline size_t view_esize(const misr_params &p) { return view_stype(p) == ST_F32 ? 4 : 2; }
// Storage type of the frames y.
inline int frame_stype(const misr_params &p) {
    return p.y_u16 ? (int)ST_U16 : (int)p.img_dtype;
}

// Per-solve image buffers owned by the library (x1, p0, p1, g0, g1; x0w is
// the FP32 copy of x0 when a 16-bit caller image is solved with an FP32
// iterate).
struct SolveBufs {
    DevMem x1, p0, p1, g0, g1, x0w;
    DevMem res;   // general operators: the residual term per LR row, then
                  // A x[0], A x[1], A p[0], A p[1] (kGenVecs LR vectors)
    void set_pool(MemPool *pl) {
        x1.pool = p0.pool = p1.pool = g0.pool = g1.pool = x0w.pool = res.pool = pl;
    }
    hipError_t ensure(long long n, size_t es) {
        hipError_t e;
        if ((e = x1.ensure(n * es)) != hipSuccess) return e;
        if ((e = p0.ensure(n * 4)) != hipSuccess) return e;
        if ((e = p1.ensure(n * 4)) != hipSuccess) return e;
        if ((e = g0.ensure(n * 4)) != hipSuccess) return e;
        return g1.ensure(n * 4);
    }
    // an untiled solve with parameters p over n HR pixels
    hipError_t ensure_view(long long n, const misr_params &p) {
        hipError_t e = ensure(n, view_esize(p));
        if (e == hipSuccess && iterate_fp32(p)) e = x0w.ensure(n * 4);
        return e;
    }
};

// Per-tile buffers of a tiled solve (x pair, p pair, g pair per tile).
struct TileSet {
    int tile_lr = 0, halo_lr = 0;
    size_t es = 0;
    MemPool *pool = nullptr;   // for the tile buffers, if set
    std::vector<std::unique_ptr<SolveBufs>> bufs;
    std::vector<std::unique_ptr<DevMem>> x0;
};

// Device mirrors of a Plan plus an instantiated graph of the whole solve.
struct PlanDev {
    DevMem projs, items, items_u, counts, states, partials, partials_u, traces, refs, halos;
    int n_iter_max = 0;
    size_t trace_ns = 0;
    hipGraphExec_t exec = nullptr;
    std::string graph_key;
    ~PlanDev() {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
    hipError_t upload(Plan &pl, int n_iter_max, hipStream_t stream);
};

}  // namespace misr

struct misr_ctx {
    int dev;
    int ncu;
    std::atomic<int> users{0};   // live ops and servers; the ctx outlives them
    hipStream_t stream;     // library stream that runs captured solves
    hipEvent_t ev_in, ev_out;
    std::mutex mu;
};

struct misr_op {
    misr_ctx *ctx;
    int H, W, s, K, P, L, Lp, TH, TW;  // TH x TW: HR tile of the image kernels
    int TWt = 0;                       // TH x TWt: the trial kernel's tile
    int tv = 0;                        // tile variant (set by misr_op_tune)
    // key of the image kernels: band length and tile variant
    int kernel_key() const { return Lp | (tv << 8); }
    std::vector<double> shifts;
    std::vector<double> psf;           // [K][2][P]: each frame's vertical, horizontal taps
    misr::DevMem wy, wx, opdev;
    // general operator (affine warps or non-separable PSFs): A and A^T as ELL
    // matrices (L = Lp = TH = TW = 0; the work-list class key is (s, 0))
    bool general = false;
    misr::DevMem a_col, a_val, t_col, t_val;
    misr::DevMem gker;                 // matrix-free: blur-and-bin kernels (K x Q x Q)
    misr::OpDev host;
    std::mutex mu;
    // final SCG state of the last misr_scg_solve (read by misr_scg_status)
    misr::DevMem last_state;
    bool have_last = false;
    // cached workspace of the single-image entry points
    misr::SolveBufs bufs;
    misr::TileSet tiles;
    misr::PlanDev pdev;
    misr::Plan plan;
};

namespace misr {

// SCG state of a new solve from its parameters (N = HR pixels).
void init_state(ScgState &s, const misr_params &p, long long N);
// Looks up, on device dev (current), the address of the workspace of
// misr_cost_grad_noalloc; once per device (noalloc.hip).
hipError_t scratch_init(int dev);
// Band length L of a translational geometry's 1-D factors (before rounding
// up to a compiled length).
int band_length(const misr_geometry *g);
// Zero weight rows after each frame's row (pad_y) and column (pad_x) tables
// of a banded operator of scale S and compiled band Lp.
void band_pad_after(int S, int Lp, int &pad_y, int &pad_x);
// General geometry: whether the matrix-free kernels take it (every frame's
// warp invertible and its adjoint windows within the LDS) unless
// general_ell asks for the stored form; with hd non-NULL also fills its
// matrix-free fields (mf, P, Q, gm, gi, eu, ev, ncu, ncv, ru, rv) and, with
// ker non-NULL, the blur-and-bin kernels (K x Q x Q).
bool general_mf_plan(const misr_geometry *g, OpDev *hd, std::vector<float> *ker);
// Work items of a matrix-free general operator: groups of kMfLRG LR tiles
// over all frames, HR tiles.
long long mf_lr_tiles(int H, int W, int s, int K);
long long mf_hr_tiles(int H, int W);


// Tile grid of a tiled solve: tile t = (a, b) owns HR rows [a T, (a+1) T) and
// columns [b T, (b+1) T) (clipped); its buffer adds a halo of Hh on interior
// sides.
struct TileGrid {
    int T, Hh, ny, nx;
};
TileGrid tile_grid(const misr_op *op, const misr_params &p);
// E_INVAL when the halo is below the reach of the operator and the prior.
misr_status check_tiling(const misr_op *op, const misr_params &p);
// Per-tile buffers (halo included) of a tiled solve.
hipError_t ensure_tiles(const misr_op *op, const misr_params &p, TileSet &ts);
// Grid and integer HR frame offsets of an operator for the start-point kernels.
InitArgs init_args(const misr_op *op);

// Appends one solve's views (one untiled view, or one per tile plus the halo
// copies between them) with their trial and update items; Proj::st is left
// for the caller.
void add_views(const misr_op *op, const misr_params &prm, const void *y, void *x,
               SolveBufs *bufs, TileSet *tiles, std::vector<Proj> &projs,
               std::vector<Item> &items, std::vector<Item> &items_u,
               std::vector<HaloCopy> &halos);

}  // namespace misr
