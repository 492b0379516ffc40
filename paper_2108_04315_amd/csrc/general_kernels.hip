// general_kernels.hip -- the SCG hot path for general operators: per-frame
// affine warps M_k and non-separable PSFs B_k (A_k = D B_k M_k of Eq. sisr
// with general factors), where A_k is not a Kronecker product of two banded
// 1-D operators and the tile kernels do not apply.
//
// A = [A_0; ...; A_{K-1}] is held as an ELL matrix over the K h w LR rows and
// its transpose over the H W HR rows (built once per operator on the host,
// entry q of row r at [q * rows + r], so a wave reads each entry slot of 64
// consecutive rows in one coalesced access).  One thread per row, kGenRows
// rows per work item.  A pass is two launches over the same item list, each
// taking the items of its role (item.tx): the trial evaluates the LR rows
// (forward at x + alpha p, residual, data cost) and then the HR rows
// (adjoint of the residual, BTV prior, gradient and inner products); the
// update pass takes the HR rows (x, p update, prior curvature) and then the
// LR rows (data curvature along the new p).  Views are FP32 and untiled.
#include <hip/hip_runtime.h>

#include "device_common.h"

namespace misr {

// The 8 BTV offsets d = (dx, dy) in [0, 2]^2 minus the origin (Eq. prior).
__device__ constexpr int kGX[8] = {1, 2, 0, 1, 2, 0, 1, 2};
__device__ constexpr int kGY[8] = {0, 0, 1, 1, 1, 2, 2, 2};

// (A v)_r for ELL row r of `rows`, with v(c) given by f(c)
// (entries in groups of four, every load of a group issued before its
// arithmetic, so that a thread keeps several HBM requests in flight)
template <class F>
FI float ell_row(const AS1 int *col, const AS1 float *val, int width, i64 rows, i64 r, F f) {
    float acc = 0.f;
    int q = 0;
    for (; q + 4 <= width; q += 4) {
        int c[4];
        float v[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const i64 at = (i64)(q + e) * rows + r;
            c[e] = col[at];
            v[e] = val[at];
        }
        float g[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) g[e] = f(c[e]);
#pragma unroll
        for (int e = 0; e < 4; ++e) acc = fmaf(v[e], g[e], acc);
    }
    for (; q < width; ++q) {
        const i64 at = (i64)q * rows + r;
        acc = fmaf(val[at], f(col[at]), acc);
    }
    return acc;
}

// trial / cost+gradient, LR rows: r = A x_t - y per row, its data cost, and
// the residual term the adjoint consumes (2 r, or psi(r) for the L1 term)
__global__ void __launch_bounds__(kGenRows) k_gen_trial_lr(const Proj *projs, const Item *items,
                                                           const int *n_items, double *partials,
                                                           int mode) {
    __shared__ double red[kNV * (kGenRows / 64)];
    const int it = blockIdx.x;
    if (it >= *n_items) return;
    const Item itm = items[it];
    if (itm.tx != 0) return;
    const Proj &P = projs[itm.proj];
    const ScgState &st = *P.st;
    if (mode == 1 && !st.active) return;
    const OpDev &op = *P.op;
    const i64 rows = (i64)op.K * (op.H / op.s) * (op.W / op.s);
    const i64 r = (i64)itm.ty * kGenRows + threadIdx.x;
    const int xc = st.xc;
    const AS1 float *x = glb((const float *)P.x[xc]);
    const AS1 float *p = glb(P.p[xc]);
    const float af = (mode == 1) ? st.alpha_f : 0.f;
    double e = 0.0;
    if (r < rows) {
        // mode 0 reads x alone: p is not yet initialised there
        const float ax = ell_row(glb(op.a_col), glb(op.a_val), op.a_w, rows, r, [&](int c) {
            return mode == 1 ? fmaf(af, p[c], x[c]) : x[c];
        });
        const float rr = ax - glb((const float *)P.y)[r] * st.wt.y_scale;
        float rv;
        if (st.wt.data_p == 2) {
            e = (double)rr * (double)rr;
            rv = 2.f * rr;
        } else {
            const float epsd = st.wt.eps_data;
            float ph, ps;
            phi_psi(rr, epsd, epsd * epsd, ph, ps);
            e = (double)ph;
            rv = ps;
        }
        glbw(P.res)[r] = rv;
    }
    double v[5] = {e, 0.0, 0.0, 0.0, 0.0};
    block_sum_store<5, kGenRows>(v, partials + (i64)it * kNV, red);
}

// trial / cost+gradient, HR rows: g_t = A^T (residual term) + the BTV
// gradient at x_t; writes g_t to g[cur ^ 1] with {E_reg, |g_t|^2, g_t.g_k,
// g_t.p} (mode 0: p[xc] = 0, the start direction buffer)
__global__ void __launch_bounds__(kGenRows) k_gen_trial_hr(const Proj *projs, const Item *items,
                                                           const int *n_items, double *partials,
                                                           int mode) {
    __shared__ double red[kNV * (kGenRows / 64)];
    const int it = blockIdx.x;
    if (it >= *n_items) return;
    const Item itm = items[it];
    if (itm.tx != 1) return;
    const Proj &P = projs[itm.proj];
    const ScgState &st = *P.st;
    if (mode == 1 && !st.active) return;
    const OpDev &op = *P.op;
    const int H = op.H, W = op.W;
    const i64 n = (i64)H * W;
    const i64 u = (i64)itm.ty * kGenRows + threadIdx.x;
    const int xc = st.xc, cur = st.cur;
    const AS1 float *x = glb((const float *)P.x[xc]);
    const AS1 float *p = glb(P.p[xc]);
    const float af = (mode == 1) ? st.alpha_f : 0.f;
    double er = 0.0, gg = 0.0, ggk = 0.0, gp = 0.0;
    if (u < n) {
        const AS1 float *res = glb((const float *)P.res);
        float g = ell_row(glb(op.t_col), glb(op.t_val), op.t_w, n, u,
                          [&](int c) { return res[c]; });
        const int ui = (int)(u / W), vi = (int)(u - (i64)ui * W);
        auto xt = [&](i64 c) { return mode == 1 ? fmaf(af, p[c], x[c]) : x[c]; };
        const float x0 = xt(u), eps = st.wt.eps, e2 = eps * eps;
        float eb = 0.f;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const int dx = kGX[d], dy = kGY[d];
            const float gam = st.wt.gam[dy * 3 + dx];
            float ph, ps;
            if (ui + dy < H && vi + dx < W) {   // pair (i, i + d), owned by i
                phi_psi(x0 - xt(u + (i64)dy * W + dx), eps, e2, ph, ps);
                g = fmaf(gam, ps, g);
                eb = fmaf(gam, ph, eb);
            }
            if (ui - dy >= 0 && vi - dx >= 0) {   // pair (i - d, i)
                phi_psi(xt(u - (i64)dy * W - dx) - x0, eps, e2, ph, ps);
                g = fmaf(-gam, ps, g);
            }
        }
        er = (double)eb;
        glbw(P.g[cur ^ 1])[u] = g;
        gg = (double)g * (double)g;
        if (mode == 1) {
            ggk = (double)g * (double)glb(P.g[cur])[u];
            gp = (double)g * (double)p[u];
        } else {
            glbw(P.p[xc])[u] = 0.f;
        }
    }
    double v[5] = {0.0, er, gg, ggk, gp};
    block_sum_store<5, kGenRows>(v, partials + (i64)it * kNV, red);
}

// update, HR rows: x <- x + alpha p, p <- -g_t + beta p (into the other
// buffer of each pair), with {prior curvature, |p|^2, p.r}: the prior part of
// Moller's curvature at the new (x, p), lambda sum gamma q^2 Q(z, sigma_k q)
// over the pairs (i, i + d) owned by i
__global__ void __launch_bounds__(kGenRows) k_gen_upd_hr(const Proj *projs, const Item *items,
                                                         const int *n_items, double *partials) {
    __shared__ double red[kNV * (kGenRows / 64)];
    const int it = blockIdx.x;
    if (it >= *n_items) return;
    const Item itm = items[it];
    if (itm.tx != 1) return;
    const Proj &P = projs[itm.proj];
    const ScgState &st = *P.st;
    if (!st.do_update) return;
    const OpDev &op = *P.op;
    const int H = op.H, W = op.W;
    const i64 n = (i64)H * W;
    const i64 u = (i64)itm.ty * kGenRows + threadIdx.x;
    const int src = st.upd_src, dst = src ^ 1;
    const AS1 float *x = glb((const float *)P.x[src]);
    const AS1 float *p = glb(P.p[src]);
    const AS1 float *gt = glb(P.g[st.cur]);
    const float af = st.alpha_f, bf = st.beta_f;
    double dreg = 0.0, pp = 0.0, pr = 0.0;
    if (u < n) {
        auto xn = [&](i64 c) { return fmaf(af, p[c], x[c]); };
        auto pn = [&](i64 c) { return fmaf(bf, p[c], -gt[c]); };
        const float x0 = xn(u), p0 = pn(u);
        glbw((float *)P.x[dst])[u] = x0;
        glbw(P.p[dst])[u] = p0;
        pp = (double)p0 * (double)p0;
        pr = -(double)p0 * (double)gt[u];
        const int ui = (int)(u / W), vi = (int)(u - (i64)ui * W);
        const float eps = st.wt.eps, e2 = eps * eps, sk = st.sigk_f;
        float a = 0.f;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const int dx = kGX[d], dy = kGY[d];
            if (ui + dy < H && vi + dx < W) {
                const i64 c = u + (i64)dy * W + dx;
                const float z = x0 - xn(c), q = p0 - pn(c);
                a += st.wt.gam[dy * 3 + dx] * q * q * psi_quot(z, sk * q, eps, e2);
            }
        }
        dreg = (double)a;
    }
    double v[4] = {0.0, dreg, pp, pr};
    block_sum_store<4, kGenRows>(v, partials + (i64)it * kNV, red);
}

// update, LR rows: the data part of the curvature along the new p,
// 2 (A_k p)^2 for the L2 term, (A_k p)^2 Q(A_k x - y_k, sigma_k A_k p) for the
// Charbonnier L1 term (x, p the new iterate and direction)
__global__ void __launch_bounds__(kGenRows) k_gen_upd_lr(const Proj *projs, const Item *items,
                                                         const int *n_items, double *partials) {
    __shared__ double red[kNV * (kGenRows / 64)];
    const int it = blockIdx.x;
    if (it >= *n_items) return;
    const Item itm = items[it];
    if (itm.tx != 0) return;
    const Proj &P = projs[itm.proj];
    const ScgState &st = *P.st;
    if (!st.do_update) return;
    const OpDev &op = *P.op;
    const i64 rows = (i64)op.K * (op.H / op.s) * (op.W / op.s);
    const i64 r = (i64)itm.ty * kGenRows + threadIdx.x;
    const int dst = st.upd_src ^ 1;
    const AS1 float *xn = glb((const float *)P.x[dst]);
    const AS1 float *pn = glb(P.p[dst]);
    double dd = 0.0;
    if (r < rows) {
        const float ap = ell_row(glb(op.a_col), glb(op.a_val), op.a_w, rows, r,
                                 [&](int c) { return pn[c]; });
        if (st.wt.data_p == 2) {
            dd = 2.0 * (double)ap * (double)ap;
        } else {
            const float ax = ell_row(glb(op.a_col), glb(op.a_val), op.a_w, rows, r,
                                     [&](int c) { return xn[c]; });
            const float rr = ax - glb((const float *)P.y)[r] * st.wt.y_scale;
            const float epsd = st.wt.eps_data;
            dd = (double)(ap * ap * psi_quot(rr, st.sigk_f * ap, epsd, epsd * epsd));
        }
    }
    double v[4] = {dd, 0.0, 0.0, 0.0};
    block_sum_store<4, kGenRows>(v, partials + (i64)it * kNV, red);
}

// standalone operators (FP32): y = A x over the LR rows, x = A^T r over the HR rows
__global__ void __launch_bounds__(kGenRows) k_gen_forward(const OpDev *opp, const float *x,
                                                          float *y) {
    const OpDev &op = *opp;
    const i64 rows = (i64)op.K * (op.H / op.s) * (op.W / op.s);
    for (i64 r = (i64)blockIdx.x * kGenRows + threadIdx.x; r < rows;
         r += (i64)gridDim.x * kGenRows)
        y[r] = ell_row(glb(op.a_col), glb(op.a_val), op.a_w, rows, r,
                       [&](int c) { return x[c]; });
}

__global__ void __launch_bounds__(kGenRows) k_gen_adjoint(const OpDev *opp, const float *r,
                                                          float *x) {
    const OpDev &op = *opp;
    const i64 n = (i64)op.H * op.W;
    for (i64 u = (i64)blockIdx.x * kGenRows + threadIdx.x; u < n;
         u += (i64)gridDim.x * kGenRows)
        x[u] = ell_row(glb(op.t_col), glb(op.t_val), op.t_w, n, u,
                       [&](int c) { return r[c]; });
}

// A pass over one class of general items: the trial and the cost+gradient
// run the LR rows then the HR rows, the update the HR rows then the LR rows.
hipError_t launch_general(int grid, hipStream_t stream, const Proj *projs, const Item *items,
                          const int *n_items, double *partials, int kind) {
    if (grid <= 0) return hipSuccess;
    if (kind == 2) {
        hipLaunchKernelGGL(k_gen_upd_hr, dim3(grid), dim3(kGenRows), 0, stream, projs, items,
                           n_items, partials);
        hipLaunchKernelGGL(k_gen_upd_lr, dim3(grid), dim3(kGenRows), 0, stream, projs, items,
                           n_items, partials);
    } else {
        const int mode = kind == 1 ? 1 : 0;
        hipLaunchKernelGGL(k_gen_trial_lr, dim3(grid), dim3(kGenRows), 0, stream, projs, items,
                           n_items, partials, mode);
        hipLaunchKernelGGL(k_gen_trial_hr, dim3(grid), dim3(kGenRows), 0, stream, projs, items,
                           n_items, partials, mode);
    }
    return hipGetLastError();
}

hipError_t launch_general_forward(hipStream_t stream, const OpDev *op, long long rows,
                                  const float *x, float *y) {
    long long blocks = (rows + kGenRows - 1) / kGenRows;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_gen_forward, dim3((unsigned)blocks), dim3(kGenRows), 0, stream, op, x,
                       y);
    return hipGetLastError();
}

hipError_t launch_general_adjoint(hipStream_t stream, const OpDev *op, long long n,
                                  const float *r, float *x) {
    long long blocks = (n + kGenRows - 1) / kGenRows;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_gen_adjoint, dim3((unsigned)blocks), dim3(kGenRows), 0, stream, op, r,
                       x);
    return hipGetLastError();
}

}  // namespace misr
