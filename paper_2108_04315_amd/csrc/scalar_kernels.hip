// scalar_kernels.hip -- the device-resident SCG state machine (Moller's
// scalar steps in FP64), small helper kernels, and the dispatch from a
// geometry's (scale, band length) to the image-kernel instances.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace misr {

// ------------------------------------------------------------ scalar kernels
// One workgroup per solve: sums that solve's partials in a fixed order, then
// thread 0 runs Moller's scalar steps in FP64.
enum Phase { PH_INIT = 0, PH_A = 1, PH_B = 2 };

__device__ void scg_init(ScgState &s, const double *v) {
    s.E = v[0] + v[1];
    s.E0 = s.E;
    s.rr = v[2];
    s.pi = v[2];
    s.mu = v[2];
    s.alpha = 0.0;
    s.beta = 0.0;
    s.alpha_f = 0.f;
    s.beta_f = 0.f;
    s.lam_bar = 0.0;
    s.k = 1;
    s.it = 0;
    s.n_success = 0;
    s.stop = 0;
    if (!isfinite(s.E) || !isfinite(s.rr)) {
        s.active = 0;
        s.stop = 2;
        s.do_update = 0;
        return;
    }
    s.active = (s.n_iter > 0);
    s.success = 1;
    s.cur ^= 1;          // the gradient at x0 went to g[cur ^ 1]
    s.upd_src = s.xc;    // p[xc] is zero: the update pass sets p = -g0, x unchanged
    s.xc ^= 1;
    s.do_update = 1;
    s.sigk = (s.pi > 0.0) ? s.sigma / sqrt(s.pi) : 0.0;
    s.sigk_f = (float)s.sigk;
}

// steps 1-5 of the pass
__device__ void scg_phase_a(ScgState &s, const double *v) {
    if (!s.active) return;
    if (s.success) {
        s.delta = v[0] + v[1];
        s.pi = v[2];
        s.mu = v[3];
    }
    if (s.rr == 0.0) {
        s.active = 0;
        s.stop = 1;
        return;
    }
    if (!isfinite(s.delta)) {
        s.active = 0;
        s.stop = 2;
        return;
    }
    double d = s.delta + (s.lam - s.lam_bar) * s.pi;
    if (d <= 0.0) {
        s.lam_bar = 2.0 * (s.lam - d / s.pi);
        d = -d + s.lam * s.pi;
        s.lam = s.lam_bar;
    }
    s.delta = d;
    s.alpha = s.mu / d;
    if (!isfinite(s.alpha)) {
        s.active = 0;
        s.stop = 2;
        return;
    }
    s.alpha_f = (float)s.alpha;
    s.rseed = mix32(0x51ed270bu + (unsigned)s.it);
}

// steps 6-9 of the pass
__device__ void scg_phase_b(ScgState &s, const double *v, IterRec *trace) {
    s.do_update = 0;
    if (!s.active) return;
    const double rr0 = s.rr;   // |r|^2 at the pass's start (mu = p . r used this r)
    const double Et = v[0] + v[1];
    s.E_t = Et;
    if (!isfinite(Et)) {
        s.active = 0;
        s.stop = 2;
        s.Delta = 0.0;
    } else {
        const double Delta = 2.0 * s.delta * (s.E - Et) / (s.mu * s.mu);
        s.Delta = Delta;
        if (Delta >= 0.0) {
            const double gg = v[2], ggk = v[3], gp = v[4];
            s.E = Et;
            s.lam_bar = 0.0;
            s.success = 1;
            s.n_success++;
            s.beta = (s.k % s.N == 0) ? 0.0 : (gg - ggk) / s.mu;
            s.rr = gg;
            s.cur ^= 1;
            s.upd_src = s.xc;
            s.xc ^= 1;
            s.do_update = 1;
            s.beta_f = (float)s.beta;
            const double pn = gg - 2.0 * s.beta * gp + s.beta * s.beta * s.pi;
            s.sigk = (pn > 0.0) ? s.sigma / sqrt(pn) : 0.0;
            s.sigk_f = (float)s.sigk;
            if (Delta >= 0.75) s.lam *= 0.25;
        } else {
            s.lam_bar = s.lam;
            s.success = 0;
        }
        if (Delta < 0.25) s.lam += s.delta * (1.0 - Delta) / s.pi;
    }
    if (trace) {
        IterRec &r = trace[s.it];
        r.E = s.E;
        r.E_t = s.E_t;
        r.delta = s.delta;
        r.mu = s.mu;
        r.alpha = s.alpha;
        r.Delta = s.Delta;
        r.lam = s.lam;
        r.pi = s.pi;
        r.rr = rr0;
        r.success = (s.do_update != 0);
        r.pad_ = 0;
    }
    s.k++;
    s.it++;
    if (s.it >= s.n_iter) s.active = 0;
}

// partials: per-item sums of the trial pass (init, phase B); partials_u: of
// the update pass (phase A).
// The solve's state is copied into LDS by 8-byte words while its partial
// sums are loaded (both only need the SolveRef), updated there by thread 0
// and copied back, so the kernel waits on global memory twice per solve
// rather than once per dependent access.
constexpr int kStW = (int)(sizeof(ScgState) / 8);
static_assert(sizeof(ScgState) % 8 == 0 && kStW <= kNT, "state copied by 8-byte words");
// Threads of the scalar kernel (a solve's partial sums, one row per work
// item, four loads each in flight per round; 1024 threads measured slower).
constexpr int kST = kNT;

__global__ void __launch_bounds__(kST) k_scalar(const SolveRef *refs, const int *n_refs,
                                                const double *__restrict__ partials,
                                                const double *__restrict__ partials_u,
                                                int phase) {
    __shared__ double red[kNV * (kST / 64)];
    __shared__ double tot[kNV];
    __shared__ ScgState sst;
    unsigned long long *sw = reinterpret_cast<unsigned long long *>(&sst);
    const int ns = *n_refs;
    // the launch grid never exceeds the SolveRef array, so the first ref is
    // read without waiting for the count
    SolveRef ref = refs[blockIdx.x];
    for (int sv = blockIdx.x; sv < ns; sv += gridDim.x) {
        if (sv != (int)blockIdx.x) ref = refs[sv];
        unsigned long long *gw = reinterpret_cast<unsigned long long *>(ref.st);
        if (threadIdx.x < kStW) sw[threadIdx.x] = gw[threadIdx.x];
        const double *pt = (phase == PH_A) ? partials_u : partials;
        const int i0 = (phase == PH_A) ? ref.item0u : ref.item0;
        const int ni = (phase == PH_A) ? ref.nitemsu : ref.nitems;
        // four items per step, all their loads issued before the additions
        // (a solve may hold thousands of items); past the end an item is
        // loaded from a valid address and counted as zero, so each thread
        // adds its items in the same order whatever the count, and in one
        // memory round trip per kSU x kST items
        constexpr int kSU = 4;   // (eight measured slower)
        double v[kNV] = {0, 0, 0, 0, 0, 0};
        const int end = i0 + ni;
        for (int i = i0 + threadIdx.x; i < end; i += kSU * kST) {
            double t[kSU][kNV];
#pragma unroll
            for (int a = 0; a < kSU; ++a) {
                const int j = (i + a * kST < end) ? i + a * kST : i;
#pragma unroll
                for (int q = 0; q < kNV; ++q) t[a][q] = pt[(long long)j * kNV + q];
            }
#pragma unroll
            for (int a = 0; a < kSU; ++a)
#pragma unroll
                for (int q = 0; q < kNV; ++q) v[q] += (i + a * kST < end) ? t[a][q] : 0.0;
        }
        // the sums are used only where the phase needs them (scg_phase_a
        // reads them after an accepted pass only)
        block_sum_store<kNV, kST>(v, tot, red);   // its barriers also publish sst
        if (threadIdx.x == 0) {
            if (phase == PH_INIT)
                scg_init(sst, tot);
            else if (phase == PH_A)
                scg_phase_a(sst, tot);
            else
                scg_phase_b(sst, tot, ref.trace);
        }
        __syncthreads();
        if (threadIdx.x < kStW) gw[threadIdx.x] = sw[threadIdx.x];
        __syncthreads();
    }
}

// Sums one solve's partials into out[0..3) = {J, E_data, E_reg} (cost only).
__global__ void __launch_bounds__(kNT) k_cost_out(const double *__restrict__ partials,
                                                  int nitems, double *out) {
    __shared__ double red[kNV * (kNT / 64)];
    __shared__ double tot[kNV];
    double v[kNV] = {0, 0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < nitems; i += kNT)
#pragma unroll
        for (int q = 0; q < kNV; ++q) v[q] += partials[(long long)i * kNV + q];
    block_sum_store<kNV, kNT>(v, tot, red);
    if (threadIdx.x == 0) {
        out[0] = tot[0] + tot[1];
        out[1] = tot[0];
        out[2] = tot[1];
    }
}

// ----------------------------------------------------------- small kernels
__global__ void k_fill_f32(float *p, long long n, float v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

// Copies x[1] into x[0] for every view whose current iterate sits in the
// workspace buffer (decided on the device).
__global__ void k_finalize(const Proj *__restrict__ projs, int nproj, int stype) {
    for (int j = 0; j < nproj; ++j) {
        const Proj &P = projs[j];
        if (P.st->xc == 0) continue;
        const long long n = (long long)P.Hb * P.ld;
        const int es = (stype == ST_F32) ? 4 : 2;
        if (es == 4) {
            const float *a = (const float *)P.x[1];
            float *b = (float *)P.x[0];
            for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
                 i += (long long)gridDim.x * blockDim.x)
                b[i] = a[i];
        } else {
            const unsigned short *a = (const unsigned short *)P.x[1];
            unsigned short *b = (unsigned short *)P.x[0];
            for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
                 i += (long long)gridDim.x * blockDim.x)
                b[i] = a[i];
        }
    }
}

// ---------------------------------------------------- tiled-solve helpers
// Halo exchange: each copy moves a rectangle of the trial gradient g[cur^1]
// from the view that owns it into another view's halo.
__global__ void k_halo(const Proj *__restrict__ projs, const HaloCopy *__restrict__ copies,
                       const int *n_copies) {
    const int n = *n_copies;
    for (int c = blockIdx.x; c < n; c += gridDim.x) {
        const HaloCopy hc = copies[c];
        const Proj &A = projs[hc.src];
        const Proj &B = projs[hc.dst];
        const int g = A.st->cur ^ 1;
        const float *src = A.g[g];
        float *dst = B.g[g];
        for (int q = threadIdx.x; q < hc.rows * hc.cols; q += blockDim.x) {
            const int r = q / hc.cols, cc = q - r * hc.cols;
            const int gy = hc.gy + r, gx = hc.gx + cc;
            dst[(long long)(gy - B.gy0) * B.ld + gx - B.gx0] =
                src[(long long)(gy - A.gy0) * A.ld + gx - A.gx0];
        }
    }
}

// Element conversions between the storage types (round to nearest even
// into 16-bit; widening is exact).
__device__ __forceinline__ float ld_any(const void *b, long long i, int t) {
    if (t == ST_F32) return ((const float *)b)[i];
    if (t == ST_BF16) return __uint_as_float((unsigned)((const unsigned short *)b)[i] << 16);
    return (float)((const _Float16 *)b)[i];
}
__device__ __forceinline__ void st_any(void *b, long long i, int t, float v) {
    if (t == ST_F32) {
        ((float *)b)[i] = v;
    } else if (t == ST_BF16) {
        unsigned u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) {
            u = 0x7fc00000u;
        } else {
            u += 0x7fffu + ((u >> 16) & 1u);
        }
        ((unsigned short *)b)[i] = (unsigned short)(u >> 16);
    } else {
        ((_Float16 *)b)[i] = (_Float16)v;
    }
}

// Whole-image x (the solve's xglob, storage gt) into every view's x[0]
// (storage vt), halo included; p[0] cleared so that the first update starts
// from a zero direction.
__global__ void k_scatter(const Proj *__restrict__ projs, int nproj, int vt, int gt) {
    for (int j = blockIdx.y; j < nproj; j += gridDim.y) {
        const Proj &P = projs[j];
        const ScgState &st = *P.st;
        const long long n = (long long)P.Hb * P.Wb;
        for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
             q += (long long)gridDim.x * blockDim.x) {
            const int r = (int)(q / P.Wb), c = (int)(q - (long long)r * P.Wb);
            const long long src = (long long)(P.gy0 + r) * st.ldg + P.gx0 + c;
            const long long dst = (long long)r * P.ld + c;
            st_any(P.x[0], dst, vt, ld_any(st.xglob, src, gt));
            P.p[0][dst] = 0.f;
        }
    }
}

// Owned part of every view's current x (which = 0; storage vt, written as
// gt) or trial gradient g[cur^1] (which = 1; FP32) back into the whole-image
// buffer.
__global__ void k_gather(const Proj *__restrict__ projs, int nproj, int vt, int gt, int which) {
    for (int j = blockIdx.y; j < nproj; j += gridDim.y) {
        const Proj &P = projs[j];
        const ScgState &st = *P.st;
        const int oh = P.oy1 - P.oy0, ow = P.ox1 - P.ox0;
        const long long n = (long long)oh * ow;
        const void *srcb = which ? (const void *)P.g[st.cur ^ 1] : P.x[st.xc];
        void *dstb = which ? (void *)st.gglob : st.xglob;
        const int ts = which ? (int)ST_F32 : vt, td = which ? (int)ST_F32 : gt;
        for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
             q += (long long)gridDim.x * blockDim.x) {
            const int r = (int)(q / ow) + P.oy0, c = (int)(q % ow) + P.ox0;
            const long long src = (long long)r * P.ld + c;
            const long long dst = (long long)(P.gy0 + r) * st.ldg + P.gx0 + c;
            st_any(dstb, dst, td, ld_any(srcb, src, ts));
        }
    }
}

// ------------------------------------------------------- start points
// Multi-image interpolation: frame k's pixel (i, j) lands on HR
// (s i + ty_k, s j + tx_k); mean of the samples landing on a pixel, in frame
// order; frame 0's covering pixel where none lands.
__global__ void k_interpolate(InitArgs a, const void *y, void *x, int st) {
    const int h = a.H / a.s, w = a.W / a.s;
    const long long n = (long long)a.H * a.W;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        const int u = (int)(q / a.W), v = (int)(q - (long long)u * a.W);
        float acc = 0.f;
        int cnt = 0;
        for (int k = 0; k < a.K; ++k) {
            const int r = u - a.ty[k], c = v - a.tx[k];
            if (r < 0 || c < 0 || r % a.s != 0 || c % a.s != 0) continue;
            const int i = r / a.s, j = c / a.s;
            if (i >= h || j >= w) continue;
            acc += ld_any(y, ((long long)k * h + i) * w + j, st);
            ++cnt;
        }
        st_any(x, q, st, cnt ? acc / (float)cnt : ld_any(y, (long long)(u / a.s) * w + v / a.s, st));
    }
}

// Keys cubic convolution weight (a = -1/2).
__device__ __forceinline__ float keys_w(float t) {
    t = fabsf(t);
    if (t <= 1.f) return (1.5f * t - 2.5f) * t * t + 1.f;
    if (t < 2.f) return ((-0.5f * t + 2.5f) * t - 4.f) * t + 2.f;
    return 0.f;
}

// Bicubic upsampling of frame 0: HR pixel u at LR coordinate (u + 1/2)/s - 1/2,
// 4 x 4 taps clamped to the frame.
__global__ void k_upsample(InitArgs a, const void *y, void *x, int st) {
    const int h = a.H / a.s, w = a.W / a.s;
    const long long n = (long long)a.H * a.W;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        const int u = (int)(q / a.W), v = (int)(q - (long long)u * a.W);
        const double cy = (u + 0.5) / a.s - 0.5, cx = (v + 0.5) / a.s - 0.5;
        const int iy = (int)floor(cy), ix = (int)floor(cx);
        const float fy = (float)(cy - iy), fx = (float)(cx - ix);
        float wy[4], wx[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            wy[t] = keys_w(fy - (t - 1));
            wx[t] = keys_w(fx - (t - 1));
        }
        float acc = 0.f;
#pragma unroll
        for (int ta = 0; ta < 4; ++ta) {
            const int i = min(max(iy + ta - 1, 0), h - 1);
            float row = 0.f;
#pragma unroll
            for (int tb = 0; tb < 4; ++tb) {
                const int j = min(max(ix + tb - 1, 0), w - 1);
                row = fmaf(wx[tb], ld_any(y, (long long)i * w + j, st), row);
            }
            acc = fmaf(wy[ta], row, acc);
        }
        st_any(x, q, st, acc);
    }
}

// ------------------------------------------------------------- dispatching
#define MISR_SCALES(X) X(1) X(2) X(3) X(4)
#define X(s)                                                                                   \
    int tile_dims_s##s(int Lp, int *th, int *tw);                                              \
    int tile_dims_trial_s##s(int Lp, int *th, int *tw);                                        \
    hipError_t launch_trial_s##s(int Lp, int stype, int grid, hipStream_t st, const Proj *projs, \
                                 const Item *items, const int *n_items, double *partials,      \
                                 int mode);                                                    \
    hipError_t launch_upcurv_s##s(int Lp, int stype, int grid, hipStream_t st,                 \
                                  const Proj *projs, const Item *items, const int *n_items,    \
                                  double *partials);                                           \
    hipError_t launch_forward_s##s(int Lp, int stype, int grid, hipStream_t st,                \
                                   const Proj *projs, const Item *items, int n, void *y);      \
    hipError_t launch_adjoint_s##s(int Lp, int stype, int grid, hipStream_t st,                \
                                   const Proj *projs, const Item *items, int n, const void *r, \
                                   float *x);
MISR_SCALES(X)
#undef X

// Band lengths instantiated per scale; an operator's L is rounded up to one.
static const int kBands[5][6] = {{0}, {4, 8, 16, 0}, {6, 8, 9, 12, 16, 0},
                                 {6, 9, 10, 12, 16, 0}, {12, 16, 0}};

int padded_band(int S, int L) {
    if (S < 1 || S > 4) return -1;
    for (int i = 0; kBands[S][i]; ++i)
        if (kBands[S][i] >= L) return kBands[S][i];
    return -1;
}

static int tile_dims(int S, int Lp, int *th, int *tw) {
    switch (S) {
    case 1: return tile_dims_s1(Lp, th, tw);
    case 2: return tile_dims_s2(Lp, th, tw);
    case 3: return tile_dims_s3(Lp, th, tw);
    case 4: return tile_dims_s4(Lp, th, tw);
    }
    return 0;
}

int tile_hr(int S, int Lp) {
    int th = -1, tw = -1;
    return tile_dims(S, Lp, &th, &tw) ? th : -1;
}

int tile_wr(int S, int Lp) {
    int th = -1, tw = -1;
    return tile_dims(S, Lp, &th, &tw) ? tw : -1;
}

int tile_wt(int S, int key) {
    int th = -1, tw = -1, ok = 0;
    switch (S) {
    case 1: ok = tile_dims_trial_s1(key, &th, &tw); break;
    case 2: ok = tile_dims_trial_s2(key, &th, &tw); break;
    case 3: ok = tile_dims_trial_s3(key, &th, &tw); break;
    case 4: ok = tile_dims_trial_s4(key, &th, &tw); break;
    }
    return ok ? tw : -1;
}

hipError_t launch_image(int S, int Lp, int grid, hipStream_t stream, const Proj *projs,
                        const Item *items, const int *n_items, double *partials, int kind,
                        int stype) {
#define X(s)                                                                                  \
    if (S == s)                                                                               \
        return kind == 2 ? launch_upcurv_s##s(Lp, stype, grid, stream, projs, items, n_items, \
                                              partials)                                       \
                         : launch_trial_s##s(Lp, stype, grid, stream, projs, items, n_items,  \
                                             partials, kind);
    MISR_SCALES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_forward(int S, int Lp, int grid, hipStream_t stream, const Proj *projs,
                          const Item *items, int n, int stype, void *y) {
#define X(s) \
    if (S == s) return launch_forward_s##s(Lp, stype, grid, stream, projs, items, n, y);
    MISR_SCALES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint(int S, int Lp, int grid, hipStream_t stream, const Proj *projs,
                          const Item *items, int n, int stype, const void *r, float *x) {
#define X(s) \
    if (S == s) return launch_adjoint_s##s(Lp, stype, grid, stream, projs, items, n, r, x);
    MISR_SCALES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_scalar(int grid, hipStream_t stream, const SolveRef *refs, const int *n_refs,
                         const double *partials, const double *partials_u, int phase) {
    hipLaunchKernelGGL(k_scalar, dim3(grid), dim3(kST), 0, stream, refs, n_refs, partials,
                       partials_u, phase);
    return hipGetLastError();
}

hipError_t launch_halo(hipStream_t stream, const Proj *projs, const HaloCopy *copies,
                       const int *n_copies, int grid) {
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_halo, dim3(grid), dim3(256), 0, stream, projs, copies, n_copies);
    return hipGetLastError();
}

hipError_t launch_scatter(hipStream_t stream, const Proj *projs, int nproj, int vt, int gt) {
    hipLaunchKernelGGL(k_scatter, dim3(256, nproj < 65535 ? nproj : 65535), dim3(256), 0, stream,
                       projs, nproj, vt, gt);
    return hipGetLastError();
}

hipError_t launch_gather(hipStream_t stream, const Proj *projs, int nproj, int vt, int gt,
                         int which) {
    hipLaunchKernelGGL(k_gather, dim3(256, nproj < 65535 ? nproj : 65535), dim3(256), 0, stream,
                       projs, nproj, vt, gt, which);
    return hipGetLastError();
}

hipError_t launch_cost_out(hipStream_t stream, const double *partials, int nitems,
                           double *out) {
    hipLaunchKernelGGL(k_cost_out, dim3(1), dim3(kNT), 0, stream, partials, nitems, out);
    return hipGetLastError();
}

hipError_t launch_fill(hipStream_t stream, float *p, long long n, float v) {
    if (n <= 0) return hipSuccess;
    long long blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)blocks), dim3(256), 0, stream, p, n, v);
    return hipGetLastError();
}

hipError_t launch_init(hipStream_t stream, int kind, const InitArgs &a, const void *y, void *x,
                       int st) {
    const long long n = (long long)a.H * a.W;
    long long blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (kind == 1)
        hipLaunchKernelGGL(k_upsample, dim3((unsigned)blocks), dim3(256), 0, stream, a, y, x, st);
    else
        hipLaunchKernelGGL(k_interpolate, dim3((unsigned)blocks), dim3(256), 0, stream, a, y, x,
                           st);
    return hipGetLastError();
}

hipError_t launch_finalize(hipStream_t stream, const Proj *projs, int nproj, int stype) {
    hipLaunchKernelGGL(k_finalize, dim3(1024), dim3(256), 0, stream, projs, nproj, stype);
    return hipGetLastError();
}

}  // namespace misr
