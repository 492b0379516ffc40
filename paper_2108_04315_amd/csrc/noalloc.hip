// noalloc.hip -- misr_cost_grad_noalloc: J(x) and grad J(x) for callers that
// cannot allocate device memory (code under graph capture, tight serving
// loops, harnesses that forbid allocation).
//
// misr_cost_grad keeps its work list, solver state and partial sums in
// workspace it allocates on the operator.  This variant runs the same kernels
// (the fused cost + gradient pass in its init mode, then the reduction of the
// partial sums) with that workspace in `scratch`, a fixed array in device
// memory of every GPU the library runs on, held until the process ends.  Its
// address on each device is looked up once, when a context is created on that
// device; the entry point itself allocates nothing and copies nothing from
// host memory: one small kernel writes the work list and state (passed by
// value as launch arguments) into the array.
//
// Every call on a device shares that device's array: calls that overlap on
// one device (on different streams, or from different threads) race.
#include <cstring>
#include <mutex>

#include "runtime.h"

namespace misr {
// Bytes of the no-allocation workspace per device.
constexpr size_t kScratchBytes = 2u << 20;
constexpr int kMaxDevices = 64;
}  // namespace misr

using namespace misr;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices];   // device address of `scratch` on each device

// Offsets inside the workspace: state, view, item count, items, partial sums.
struct Layout {
    size_t st, proj, cnt, items, part, end;
};

size_t up256(size_t v) { return (v + 255) & ~(size_t)255; }

Layout layout(long long n_items) {
    Layout l;
    l.st = 0;
    l.proj = up256(l.st + sizeof(ScgState));
    l.cnt = up256(l.proj + sizeof(Proj));
    l.items = up256(l.cnt + sizeof(int));
    l.part = up256(l.items + (size_t)n_items * sizeof(Item));
    l.end = l.part + (size_t)n_items * kNV * sizeof(double);
    return l;
}

// Writes the solver state (objective weights), the view (pointing at that
// state) and the item list of one untiled image into the workspace: item i
// is tile strip_tile(i), the order of the library's own work lists.
__global__ void k_noalloc_setup(Proj P, ScgState S, int nty, int ntx, unsigned char *base,
                                Layout l) {
    const int n = nty * ntx;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0) {
        ScgState *st = (ScgState *)(base + l.st);
        *st = S;
        P.st = st;
        *(Proj *)(base + l.proj) = P;
        *(int *)(base + l.cnt) = n;
    }
    if (i < n) {
        int ty, tx;
        strip_tile(i, nty, ntx, ty, tx);
        ((Item *)(base + l.items))[i] = Item{0, ty, tx, 0};
    }
}

}  // namespace

// Looks up the workspace's address on device dev (the current device); once
// per device.
hipError_t misr::scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[dev]) return hipSuccess;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch[dev] = p;
    return hipSuccess;
}

extern "C" size_t misr_cost_grad_noalloc_max_bytes(void) { return kScratchBytes; }

extern "C" misr_status misr_cost_grad_noalloc(const misr_op *op, const misr_params *prm,
                                              const void *x, const void *y, float *g,
                                              double *cost_dev, void *stream) {
    if (!op || !prm || !x || !y || !g || !cost_dev) return set_error(MISR_E_INVAL, "NULL argument");
    misr_status st = misr_params_check(prm);
    if (st != MISR_OK) return st;
    if (op->general)
        return set_error(MISR_E_INVAL, "misr_cost_grad_noalloc takes banded (translational, "
                         "separable-PSF) operators");
    if (prm->tile_lr > 0)
        return set_error(MISR_E_INVAL, "misr_cost_grad_noalloc evaluates untiled images "
                         "(tile_lr = 0)");
    const int dev = op->ctx->dev;
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = (dev >= 0 && dev < kMaxDevices) ? g_scratch[dev] : nullptr;
    }
    if (!base) return set_error(MISR_E_HIP, "no-allocation workspace of device %d not set up", dev);
    const int nty = (op->H + op->TH - 1) / op->TH, ntx = (op->W + op->TWt - 1) / op->TWt;
    const long long n_items = (long long)nty * ntx;
    const Layout l = layout(n_items);
    if (l.end > kScratchBytes)
        return set_error(MISR_E_INVAL, "%lld tiles need %zu bytes of workspace, more than the "
                         "%zu the no-allocation entry point holds (at most %lld tiles of "
                         "%d x %d HR px)", n_items, l.end, kScratchBytes,
                         (long long)((kScratchBytes - layout(0).end) /
                                     (sizeof(Item) + kNV * sizeof(double))),
                         op->TH, op->TWt);
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e == hipSuccess && cur != dev) e = hipSetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    // the state of misr_cost_grad's evaluation: x as stored, g written to
    // g[cur ^ 1] with cur = 0, no direction buffer
    misr_params p = *prm;
    p.n_iter = 0;
    p.x_work = 1;
    p.x_init = 0;
    ScgState S;
    init_state(S, p, (long long)op->H * op->W);
    Proj P;
    std::memset(&P, 0, sizeof P);
    P.x[0] = const_cast<void *>(x);
    P.g[1] = g;
    P.y = y;
    P.op = op->opdev.as<OpDev>();
    P.ld = P.Wb = op->W;
    P.Hb = op->H;
    P.oy1 = P.uy1 = op->H;
    P.ox1 = P.ux1 = op->W;
    P.ntx = (op->W + op->TW - 1) / op->TW;
    hipStream_t s = (hipStream_t)stream;
    unsigned char *b = (unsigned char *)base;
    const int blocks = (int)((n_items + 255) / 256);
    hipLaunchKernelGGL(k_noalloc_setup, dim3(blocks), dim3(256), 0, s, P, S, nty, ntx, b, l);
    MISR_HIP(hipGetLastError());
    MISR_HIP(launch_image(op->s, op->kernel_key(), (int)n_items, s, (const Proj *)(b + l.proj),
                          (const Item *)(b + l.items), (const int *)(b + l.cnt),
                          (double *)(b + l.part), KIND_COSTGRAD,
                          st_code(view_stype(p), frame_stype(p))));
    MISR_HIP(launch_cost_out(s, (const double *)(b + l.part), (int)n_items, cost_dev));
    return MISR_OK;
}
