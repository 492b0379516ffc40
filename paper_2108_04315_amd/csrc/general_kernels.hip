// general_kernels.hip -- the SCG hot path for general operators: per-frame
// affine warps M_k and non-separable PSFs B_k (A_k = D B_k M_k of Eq. sisr
// with general factors), where A_k is not a Kronecker product of two banded
// 1-D operators and the band kernels do not apply.
//
// Matrix-free form (OpDev::mf): A_k is applied from its factors.  Forward,
// per LR tile: the warped image z = M_k v on the HR window the tile's outputs
// read is built in LDS (bilinear samples of v, zero off the grid), then each
// LR pixel takes its Q x Q window of z times the frame's blur-and-bin kernel
// C_k (B_k's P x P PSF convolved with D's s x s box, over s^2).  Adjoint, per
// HR tile: per frame the residual window is staged in LDS, the
// back-projection w = B_k^T D^T r_k is formed on the HR window the tile's
// pixels gather from (the preimage of the tile under the warp), and each
// pixel sums w over the positions whose warped coordinates lie within one
// pixel of it, times the bilinear (tent) weights: the transpose of the
// forward's sampling, gathered rather than scattered, so each output is a
// fixed-order sum.  Per pass and HR pixel this reads x, p (and the frames)
// once instead of the sparse matrices' entries.
//
// Stored form (warps whose windows exceed the LDS, or on request):
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

#include <type_traits>

#include "device_common.h"

namespace misr {

// The 8 BTV offsets d = (dx, dy) in [0, 2]^2 minus the origin (Eq. prior).
__device__ constexpr int kGX[8] = {1, 2, 0, 1, 2, 0, 1, 2};
__device__ constexpr int kGY[8] = {0, 0, 1, 1, 1, 2, 2, 2};

// ------------------------------------------------------------ matrix-free

// (M_k v)(u, v) from the warped coordinate (r, c) of HR pixel (u, v): the
// bilinear sample of v; zero off the grid, corners off the grid weigh
// nothing.
template <class V>
FI float mf_sample(int H, int W, int u, int v, double r, double c, V vec) {
    if (u < 0 || u >= H || v < 0 || v >= W) return 0.f;
    const double r0 = floor(r), c0 = floor(c);
    const float fa = (float)(r - r0), fb = (float)(c - c0);
    // clamped before the conversion: a corner beyond the grid weighs nothing
    const int ir = (int)fmin(fmax(r0, -2.0), (double)H + 1.0);
    const int ic = (int)fmin(fmax(c0, -2.0), (double)W + 1.0);
    const bool r0k = ir >= 0 && ir < H, r1k = ir + 1 >= 0 && ir + 1 < H;
    const bool c0k = ic >= 0 && ic < W, c1k = ic + 1 >= 0 && ic + 1 < W;
    const i64 b = (i64)ir * W + ic;
    float acc = 0.f;
    if (r0k && c0k) acc = fmaf((1.f - fa) * (1.f - fb), vec(b), acc);
    if (r0k && c1k) acc = fmaf((1.f - fa) * fb, vec(b + 1), acc);
    if (r1k && c0k) acc = fmaf(fa * (1.f - fb), vec(b + W), acc);
    if (r1k && c1k) acc = fmaf(fa * fb, vec(b + W + 1), acc);
    return acc;
}

// Tile q of LR item t: an item takes kMfLRG consecutive tiles of one frame
// (frames in turn, tiles row-major); frame, tile row and column, or false
// past the frame's last tile.
FI bool mf_lr_tile(const AS4 OpDev &op, int t, int q, int &k, int &ti, int &tj) {
    const int h = op.H / op.s, w = op.W / op.s, TI = mf_ti(op.s);
    const int nti = (h + TI - 1) / TI, ntj = (w + kMfTJ - 1) / kMfTJ;
    const int ng = (nti * ntj + kMfLRG - 1) / kMfLRG;
    k = t / ng;
    const int c = (t - k * ng) * kMfLRG + q;
    if (c >= nti * ntj) return false;
    ti = c / ntj;
    tj = c - ti * ntj;
    return true;
}

// e / d for 0 <= e < 2^21, d >= 1, through the float reciprocal inv = 1 / d:
// (e + 1/2) / d lies at least 1/(2 d) from an integer, well above the
// product's rounding error, so the truncation is exact.
FI int mf_div(int e, float inv) { return (int)(((float)e + 0.5f) * inv); }

// (A_k v) at this thread's LR pixels of LR tile (ti, tj) of frame k: row i,
// columns j + 32 c, c < kMfCPT, into out[c] (pixels past the frame are
// computed and not used: the caller checks i < h, j + 32 c < w).  zs: the
// warped window, free again on return.
template <int S, class V>
FI void mf_forward(const AS4 OpDev &op, int k, int ti, int tj, V vec, float *zs, int &i, int &j,
                   float (&out)[kMfCPT]) {
    constexpr int TI = mf_ti(S);
    const int H = op.H, W = op.W, Q = op.Q, R = (op.P - 1) / 2;
    const int i0 = ti * TI, j0 = tj * kMfTJ;
    const int ZR = S * (TI - 1) + Q, ZC = S * (kMfTJ - 1) + Q;
    const int u0 = S * i0 - R, v0 = S * j0 - R;
    const double m0 = op.gm[k][0], m1 = op.gm[k][1], m2 = op.gm[k][2];
    const double m3 = op.gm[k][3], m4 = op.gm[k][4], m5 = op.gm[k][5];
    const float izc = 1.f / (float)ZC;
    for (int e = threadIdx.x; e < ZR * ZC; e += kGenRows) {
        const int a = mf_div(e, izc), b = e - a * ZC;
        const double u = u0 + a, v = v0 + b;
        zs[e] = mf_sample(H, W, u0 + a, v0 + b, fma(m0, u, fma(m1, v, m2)),
                          fma(m3, u, fma(m4, v, m5)), vec);
    }
    __syncthreads();
    const int il = threadIdx.x / 32, jl = threadIdx.x % 32;
    const AS4 float *ck = cst(op.gker) + (i64)k * Q * Q;
    const float *zb = zs + S * il * ZC + S * jl;
    float acc[kMfCPT];
#pragma unroll
    for (int c = 0; c < kMfCPT; ++c) acc[c] = 0.f;
    for (int a = 0; a < Q; ++a) {
#pragma unroll 4
        for (int b = 0; b < Q; ++b) {
            const float cw = ck[a * Q + b];
#pragma unroll
            for (int c = 0; c < kMfCPT; ++c) acc[c] = fmaf(cw, zb[a * ZC + b + S * 32 * c], acc[c]);
        }
    }
    __syncthreads();
    i = i0 + il;
    j = j0 + jl;
#pragma unroll
    for (int c = 0; c < kMfCPT; ++c) out[c] = acc[c];
}

// Clamped conversion of a window bound (the operator's windows are small,
// the clamp only keeps the conversion defined).
FI int mf_int(double v) { return (int)fmin(fmax(v, -1073741824.0), 1073741824.0); }

// acc[t] += sum_k (A_k^T r_k)(pixel) for this thread's four pixels of HR
// tile (tu, tv) (rows tu kMfTU + threadIdx.x / 64 + 4 t, column
// tv kMfTV + threadIdx.x % 64); res(k, i, j) gives r_k.  lds: kMfWin floats
// plus kMfQP^2, free again on return.
//
// Per frame: the back-projection window [ua, ub] x [va, vb] holds every
// candidate position of every pixel of the tile (a pixel's candidates start
// at floor(u(p) - eu) + 1, ncu of them), so the gathers need no bounds
// checks; positions off the grid hold 0.  Position (u, v) takes the residual
// of LR pixels i = floor((u + R) / s) - t, t < NT = ceil(Q / s), with kernel
// row (u + R) mod s + s t (rows from Q on are zero in the padded copy), so
// every position runs the same NT x NT taps.
template <int S, class Rf>
FI void mf_adjoint(const AS4 OpDev &op, int tu, int tv, Rf res, float *lds, float (&acc)[4]) {
    const int H = op.H, W = op.W, Q = op.Q, R = (op.P - 1) / 2;
    const int h = H / S, w = W / S;
    const int NT = (Q + S - 1) / S, QP = S * NT;
    const int U0 = tu * kMfTU, V0 = tv * kMfTV;
    const int U1 = min(U0 + kMfTU, H) - 1, V1 = min(V0 + kMfTV, W) - 1;
    const int row = threadIdx.x >> 6, lane = threadIdx.x & 63;
    float *cpl = lds + kMfWin;
    for (int k = 0; k < op.K; ++k) {
        const double g0 = op.gi[k][0], g1 = op.gi[k][1], g2 = op.gi[k][2];
        const double g3 = op.gi[k][3], g4 = op.gi[k][4], g5 = op.gi[k][5];
        const double eu = op.eu[k], ev = op.ev[k];
        double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double pr = (q & 1) ? U1 : U0, pc = (q & 2) ? V1 : V0;
            const double uc = fma(g0, pr, fma(g1, pc, g2)), vc = fma(g3, pr, fma(g4, pc, g5));
            umin = fmin(umin, uc);
            umax = fmax(umax, uc);
            vmin = fmin(vmin, vc);
            vmax = fmax(vmax, vc);
        }
        const int ua = mf_int(floor(umin - eu)) + 1, va = mf_int(floor(vmin - ev)) + 1;
        const int ub = min(mf_int(floor(umax + eu)) + 1, ua + op.ru[k] - 1);
        const int vb = min(mf_int(floor(vmax + ev)) + 1, va + op.rv[k] - 1);
        // the tile's pixels gather from nothing on the grid: skip (uniform)
        if (ub < 0 || ua > H - 1 || vb < 0 || va > W - 1) continue;
        const int RU = ub - ua + 1, RV = vb - va + 1;
        const int i0 = fdiv(ua + R, S) - NT + 1, j0 = fdiv(va + R, S) - NT + 1;
        const int NI = fdiv(ub + R, S) - i0 + 1, NJ = fdiv(vb + R, S) - j0 + 1;
        float *rsm = lds, *wt = lds + NI * NJ;
        const float inj = 1.f / (float)NJ, irv = 1.f / (float)RV;
        for (int e = threadIdx.x; e < NI * NJ; e += kGenRows) {
            const int a = mf_div(e, inj), i = i0 + a, j = j0 + e - a * NJ;
            rsm[e] = (i >= 0 && i < h && j >= 0 && j < w) ? res(k, i, j) : 0.f;
        }
        const AS4 float *ck = cst(op.gker) + (i64)k * Q * Q;
        for (int a = threadIdx.x >> 5; a < QP; a += kGenRows / 32) {
            const int b = threadIdx.x & 31;
            if (b < QP) cpl[a * QP + b] = (a < Q && b < Q) ? ck[a * Q + b] : 0.f;
        }
        __syncthreads();
        // the taps, with their count fixed at compile time where it is small
        auto backproj = [&](auto ntc) {
            constexpr int NTC = decltype(ntc)::value;
            const int nt = NTC > 0 ? NTC : NT;
            for (int e = threadIdx.x; e < RU * RV; e += kGenRows) {
                const int a = mf_div(e, irv);
                const int u = ua + a, v = va + e - a * RV;
                float sum = 0.f;
                if (u >= 0 && u < H && v >= 0 && v < W) {
                    const int qu = fdiv(u + R, S), qv = fdiv(v + R, S);
                    const float *cr = cpl + (u + R - S * qu) * QP + (v + R - S * qv);
                    const float *rr = rsm + (qu - i0) * NJ + (qv - j0);
#pragma unroll 6
                    for (int t = 0; t < nt; ++t)
#pragma unroll 6
                        for (int t2 = 0; t2 < nt; ++t2)
                            sum = fmaf(cr[S * (t * QP + t2)], rr[-t * NJ - t2], sum);
                }
                wt[e] = sum;
            }
        };
        switch (NT) {   // uniform
        case 2: backproj(std::integral_constant<int, 2>{}); break;
        case 3: backproj(std::integral_constant<int, 3>{}); break;
        case 4: backproj(std::integral_constant<int, 4>{}); break;
        case 5: backproj(std::integral_constant<int, 5>{}); break;
        default: backproj(std::integral_constant<int, 0>{}); break;
        }
        __syncthreads();
        const double m0 = op.gm[k][0], m1 = op.gm[k][1], m2 = op.gm[k][2];
        const double m3 = op.gm[k][3], m4 = op.gm[k][4], m5 = op.gm[k][5];
        const float m0f = (float)m0, m1f = (float)m1, m3f = (float)m3, m4f = (float)m4;
        const int ncu = op.ncu[k], ncv = op.ncv[k];
        const bool c33 = ncu == 3 && ncv == 3;   // the near-identity warps (uniform)
        // tile-relative coordinates in FP32 (magnitudes of the tile's extent):
        // the preimage of the tile's corner pixel (U0, V0) less the window's
        // origin, and the warped coordinate of the window's origin less the
        // corner pixel, both from FP64 once per tile.  A rounding that moves a
        // pixel's first candidate by one position changes only candidates at
        // the edge of its support, whose tent weights are zero to rounding.
        const float ub0 = (float)(fma(g0, (double)U0, fma(g1, (double)V0, g2)) - ua);
        const float vb0 = (float)(fma(g3, (double)U0, fma(g4, (double)V0, g5)) - va);
        const float rb0 = (float)(fma(m0, (double)ua, fma(m1, (double)va, m2)) - U0);
        const float cb0 = (float)(fma(m3, (double)ua, fma(m4, (double)va, m5)) - V0);
        const float g0f = (float)g0, g1f = (float)g1, g3f = (float)g3, g4f = (float)g4;
        const float euf = (float)eu, evf = (float)ev;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int dr = row + 4 * t, dc = lane;
            if (U0 + dr > U1 || V0 + dc > V1) continue;
            // first candidate, relative to the window's origin, kept inside
            // the window (a rounding at the edge moves it by one)
            const float uq = fmaf((float)dr, g0f, fmaf((float)dc, g1f, ub0)) - euf;
            const float vq = fmaf((float)dr, g3f, fmaf((float)dc, g4f, vb0)) - evf;
            const int ous = min(max(0, (int)floorf(uq) + 1), RU - ncu);
            const int ovs = min(max(0, (int)floorf(vq) + 1), RV - ncv);
            // its warped coordinate relative to the pixel
            const float d0r = fmaf((float)ous, m0f, fmaf((float)ovs, m1f, rb0)) - (float)dr;
            const float d0c = fmaf((float)ous, m3f, fmaf((float)ovs, m4f, cb0)) - (float)dc;
            const float *wb = wt + ous * RV + ovs;
            float a_t = 0.f;
            auto cand = [&](int a, int b) {
                const float dr = fmaf((float)b, m1f, fmaf((float)a, m0f, d0r));
                const float dc = fmaf((float)b, m4f, fmaf((float)a, m3f, d0c));
                const float wgt = fmaxf(0.f, 1.f - fabsf(dr)) * fmaxf(0.f, 1.f - fabsf(dc));
                a_t = fmaf(wgt, wb[a * RV + b], a_t);
            };
            if (c33) {
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int b = 0; b < 3; ++b) cand(a, b);
            } else {
                for (int a = 0; a < ncu; ++a)
                    for (int b = 0; b < ncv; ++b) cand(a, b);
            }
            acc[t] += a_t;
        }
        __syncthreads();
    }
}

// Runs f with the scale as a compile-time constant (uniform branch).
template <class F>
FI void mf_by_scale(int s, F f) {
    switch (s) {
    case 1: f(std::integral_constant<int, 1>{}); break;
    case 2: f(std::integral_constant<int, 2>{}); break;
    case 3: f(std::integral_constant<int, 3>{}); break;
    default: f(std::integral_constant<int, 4>{}); break;
    }
}

// ------------------------------------------------------------ stored form

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

// Residual term of LR row r (frame value y[r]) at forward value ax: the
// data cost of the row and the term the adjoint consumes (2 r, or psi(r)
// for the Charbonnier L1 term), stored to res[r].
FI double gen_residual(const ScgState &st, const Proj &P, i64 r, float ax) {
    const float rr = ax - glb((const float *)P.y)[r] * st.wt.y_scale;
    float rv;
    double e;
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
    return e;
}

// BTV prior at HR pixel (ui, vi) of x_t, given at offsets (dy, dx) from the
// pixel by xo(dy, dx): adds its gradient to g and returns its cost over the
// pairs (i, i + d) owned by the pixel.
template <class X>
FI float gen_prior(const ScgState &st, int H, int W, int ui, int vi, X xo, float &g) {
    const float x0 = xo(0, 0), eps = st.wt.eps, e2 = eps * eps;
    float eb = 0.f;
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const int dx = kGX[d], dy = kGY[d];
        const float gam = st.wt.gam[dy * 3 + dx];
        float ph, ps;
        if (ui + dy < H && vi + dx < W) {   // pair (i, i + d), owned by i
            phi_psi(x0 - xo(dy, dx), eps, e2, ph, ps);
            g = fmaf(gam, ps, g);
            eb = fmaf(gam, ph, eb);
        }
        if (ui - dy >= 0 && vi - dx >= 0) {   // pair (i - d, i)
            phi_psi(xo(-dy, -dx) - x0, eps, e2, ph, ps);
            g = fmaf(-gam, ps, g);
        }
    }
    return eb;
}

// Prior part of Moller's curvature at the new (x, p) over the pairs owned by
// HR pixel (ui, vi): lambda sum gamma q^2 Q(z, sigma_k q), the new x and p
// at offsets (dy, dx) given by xo, po.
template <class X, class Pf>
FI float gen_prior_curv(const ScgState &st, int H, int W, int ui, int vi, X xo, Pf po) {
    const float x0 = xo(0, 0), p0 = po(0, 0);
    const float eps = st.wt.eps, e2 = eps * eps, sk = st.sigk_f;
    float a = 0.f;
#pragma unroll
    for (int d = 0; d < 8; ++d) {
        const int dx = kGX[d], dy = kGY[d];
        if (ui + dy < H && vi + dx < W) {
            const float z = x0 - xo(dy, dx), q = p0 - po(dy, dx);
            a += st.wt.gam[dy * 3 + dx] * q * q * psi_quot(z, sk * q, eps, e2);
        }
    }
    return a;
}

// Update at HR pixel u = (ui, vi) of the stored form: x <- x + alpha p,
// p <- -g_t + beta p into the other buffers; returns the prior part of the
// curvature at the new (x, p), with |p|^2 and p.r.
FI float gen_update(const ScgState &st, const Proj &P, int H, int W, i64 u, int ui, int vi,
                    double &pp, double &pr) {
    const int src = st.upd_src, dst = src ^ 1;
    const AS1 float *x = glb((const float *)P.x[src]);
    const AS1 float *p = glb(P.p[src]);
    const AS1 float *gt = glb(P.g[st.cur]);
    const float af = st.alpha_f, bf = st.beta_f;
    auto xn = [&](int dy, int dx) {
        const i64 c = u + (i64)dy * W + dx;
        return fmaf(af, p[c], x[c]);
    };
    auto pn = [&](int dy, int dx) {
        const i64 c = u + (i64)dy * W + dx;
        return fmaf(bf, p[c], -gt[c]);
    };
    const float x0 = xn(0, 0), p0 = pn(0, 0);
    glbw((float *)P.x[dst])[u] = x0;
    glbw(P.p[dst])[u] = p0;
    pp += (double)p0 * (double)p0;
    pr += -(double)p0 * (double)gt[u];
    return gen_prior_curv(st, H, W, ui, vi, xn, pn);
}

// Data part of the curvature of one LR row at A p (ap) and A x (ax) of the
// new iterate: 2 (A_k p)^2 for the L2 term, (A_k p)^2 Q(A_k x - y_k,
// sigma_k A_k p) for the Charbonnier L1 term.
FI double gen_data_curv(const ScgState &st, const Proj &P, i64 r, float ap, float ax) {
    if (st.wt.data_p == 2) return 2.0 * (double)ap * (double)ap;
    const float rr = ax - glb((const float *)P.y)[r] * st.wt.y_scale;
    const float epsd = st.wt.eps_data;
    return (double)(ap * ap * psi_quot(rr, st.sigk_f * ap, epsd, epsd * epsd));
}

// trial / cost+gradient, LR rows (an LR tile, or kGenRows ELL rows): the
// forward at x_t = x + alpha p (mode 1) or x (mode 0), the residual term and
// the data cost.  Matrix-free: mode 0 applies A to x and keeps A x (and
// A p = 0 for the zero start direction); mode 1 takes A x + alpha A p from
// the kept vectors (A is linear), with no forward.
__global__ void __launch_bounds__(kGenRows) k_gen_trial_lr(const Proj *projs, const Item *items,
                                                           const int *n_items, double *partials,
                                                           int mode) {
    __shared__ double red[kNV * (kGenRows / 64)];
    // the warped window of the matrix-free forward (mode 0 only: the launch
    // sizes it, so the elementwise mode 1 runs at full occupancy)
    extern __shared__ float zs[];
    const int it = blockIdx.x;
    if (it >= *n_items) return;
    const Item itm = items[it];
    if (itm.tx != 0) return;
    const Proj &P = projs[itm.proj];
    const ScgState &st = *P.st;
    if (mode == 1 && !st.active) return;
    const AS4 OpDev &op = *cst(P.op);
    const int h = op.H / op.s, w = op.W / op.s;
    const int xc = st.xc;
    const AS1 float *x = glb((const float *)P.x[xc]);
    const AS1 float *p = glb(P.p[xc]);
    const float af = (mode == 1) ? st.alpha_f : 0.f;
    // mode 0 reads x alone: p is not yet initialised there
    auto xt = [&](i64 c) { return mode == 1 ? fmaf(af, p[c], x[c]) : x[c]; };
    double e = 0.0;
    if (op.mf && mode == 1) {
        // elementwise: item t takes LR rows [t B, (t + 1) B), B = kGenRows
        // kMfCPT (there are at least as many LR items as such blocks)
#pragma unroll
        for (int c = 0; c < kMfCPT; ++c) {
            const i64 r = ((i64)itm.ty * kMfCPT + c) * kGenRows + threadIdx.x;
            if (r < (i64)op.K * h * w)
                e += gen_residual(st, P, r, fmaf(af, glb(P.ap[xc])[r], glb(P.ax[xc])[r]));
        }
    } else if (op.mf) {
        int k, ti, tj, i, j;
        mf_by_scale(op.s, [&](auto S) {
            for (int q = 0; q < kMfLRG && mf_lr_tile(op, itm.ty, q, k, ti, tj); ++q) {
                float ax[kMfCPT];
                mf_forward<S.value>(op, k, ti, tj, xt, zs, i, j, ax);
#pragma unroll
                for (int c = 0; c < kMfCPT; ++c)
                    if (i < h && j + 32 * c < w) {
                        const i64 row = ((i64)k * h + i) * w + j + 32 * c;
                        e += gen_residual(st, P, row, ax[c]);
                        glbw(P.ax[xc])[row] = ax[c];
                        glbw(P.ap[xc])[row] = 0.f;
                    }
            }
        });
    } else {
        const i64 rows = (i64)op.K * h * w;
        const i64 r = (i64)itm.ty * kGenRows + threadIdx.x;
        if (r < rows) e = gen_residual(st, P, r, ell_row(glb(op.a_col), glb(op.a_val), op.a_w,
                                                          rows, r, xt));
    }
    double v[5] = {e, 0.0, 0.0, 0.0, 0.0};
    block_sum_store<5, kGenRows>(v, partials + (i64)it * kNV, red);
}

// trial / cost+gradient, HR rows (an HR tile, or kGenRows ELL rows):
// g_t = A^T (residual term) + the BTV gradient at x_t; writes g_t to
// g[cur ^ 1] with {E_reg, |g_t|^2, g_t.g_k, g_t.p} (mode 0: p[xc] = 0, the
// start direction buffer)
__global__ void __launch_bounds__(kGenRows) k_gen_trial_hr(const Proj *projs, const Item *items,
                                                           const int *n_items, double *partials,
                                                           int mode) {
    __shared__ double red[kNV * (kGenRows / 64)];
    __shared__ float lds[kMfWin + kMfQP * kMfQP];
    const int it = blockIdx.x;
    if (it >= *n_items) return;
    const Item itm = items[it];
    if (itm.tx != 1) return;
    const Proj &P = projs[itm.proj];
    const ScgState &st = *P.st;
    if (mode == 1 && !st.active) return;
    const AS4 OpDev &op = *cst(P.op);
    const int H = op.H, W = op.W, h = H / op.s, w = W / op.s;
    const i64 n = (i64)H * W;
    const int xc = st.xc, cur = st.cur;
    const AS1 float *x = glb((const float *)P.x[xc]);
    const AS1 float *p = glb(P.p[xc]);
    const AS1 float *res = glb((const float *)P.res);
    const float af = (mode == 1) ? st.alpha_f : 0.f;
    auto xt = [&](i64 c) { return mode == 1 ? fmaf(af, p[c], x[c]) : x[c]; };
    double er = 0.0, gg = 0.0, ggk = 0.0, gp = 0.0;
    // gradient of one pixel from its data part: prior (x_t at offsets from
    // the pixel given by xo), store, inner products
    auto finish = [&](i64 u, int ui, int vi, float g, auto xo) {
        er += (double)gen_prior(st, H, W, ui, vi, xo, g);
        glbw(P.g[cur ^ 1])[u] = g;
        gg += (double)g * (double)g;
        if (mode == 1) {
            ggk += (double)g * (double)glb(P.g[cur])[u];
            gp += (double)g * (double)p[u];
        } else {
            glbw(P.p[xc])[u] = 0.f;
        }
    };
    if (op.mf) {
        const int ntv = (W + kMfTV - 1) / kMfTV;
        const int tu = itm.ty / ntv, tv = itm.ty - tu * ntv;
        float acc[4] = {0.f, 0.f, 0.f, 0.f};
        mf_by_scale(op.s, [&](auto S) {
            mf_adjoint<S.value>(op, tu, tv,
                                [&](int k, int i, int j) { return res[((i64)k * h + i) * w + j]; },
                                lds, acc);
        });
        // x_t on the tile and two pixels around it, for the prior's pairs
        constexpr int WR = kMfTU + 4, WC = kMfTV + 4;
        const int U0 = tu * kMfTU - 2, V0 = tv * kMfTV - 2;
        for (int e = threadIdx.x; e < WR * WC; e += kGenRows) {
            const int a = e / WC, u = U0 + a, v = V0 + e - a * WC;
            lds[e] = (u >= 0 && u < H && v >= 0 && v < W) ? xt((i64)u * W + v) : 0.f;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int a = (threadIdx.x >> 6) + 4 * t, b = threadIdx.x & 63;
            const int pr = tu * kMfTU + a, pc = tv * kMfTV + b;
            const float *wp = lds + (a + 2) * WC + b + 2;
            if (pr < H && pc < W)
                finish((i64)pr * W + pc, pr, pc, acc[t],
                       [&](int dy, int dx) { return wp[dy * WC + dx]; });
        }
    } else {
        const i64 u = (i64)itm.ty * kGenRows + threadIdx.x;
        if (u < n) {
            const int ui = (int)(u / W), vi = (int)(u - (i64)ui * W);
            finish(u, ui, vi, ell_row(glb(op.t_col), glb(op.t_val), op.t_w, n, u,
                                      [&](int c) { return res[c]; }),
                   [&](int dy, int dx) { return xt(u + (i64)dy * W + dx); });
        }
    }
    double v[5] = {0.0, er, gg, ggk, gp};
    block_sum_store<5, kGenRows>(v, partials + (i64)it * kNV, red);
}

// update, HR rows (an HR tile, or kGenRows rows): x <- x + alpha p,
// p <- -g_t + beta p (into the other buffer of each pair), with {prior
// curvature, |p|^2, p.r}: the prior part of Moller's curvature at the new
// (x, p), lambda sum gamma q^2 Q(z, sigma_k q) over the pairs (i, i + d)
// owned by i
__global__ void __launch_bounds__(kGenRows) k_gen_upd_hr(const Proj *projs, const Item *items,
                                                         const int *n_items, double *partials) {
    __shared__ double red[kNV * (kGenRows / 64)];
    __shared__ float upd_lds[2 * (kMfTU + 2) * (kMfTV + 2)];
    const int it = blockIdx.x;
    if (it >= *n_items) return;
    const Item itm = items[it];
    if (itm.tx != 1) return;
    const Proj &P = projs[itm.proj];
    const ScgState &st = *P.st;
    if (!st.do_update) return;
    const AS4 OpDev &op = *cst(P.op);
    const int H = op.H, W = op.W;
    double dreg = 0.0, pp = 0.0, pr = 0.0;
    if (op.mf) {
        // the new x and p on the tile and the two pixels below and right of
        // it (the pairs a pixel owns), each formed once
        constexpr int WR = kMfTU + 2, WC = kMfTV + 2;
        float *xw = upd_lds, *pw = upd_lds + WR * WC;
        const int ntv = (W + kMfTV - 1) / kMfTV;
        const int tu = itm.ty / ntv, tv = itm.ty - tu * ntv;
        const int src = st.upd_src, dst = src ^ 1;
        const AS1 float *x = glb((const float *)P.x[src]);
        const AS1 float *p = glb(P.p[src]);
        const AS1 float *gt = glb(P.g[st.cur]);
        const float af = st.alpha_f, bf = st.beta_f;
        for (int e = threadIdx.x; e < WR * WC; e += kGenRows) {
            const int a = e / WC, u = tu * kMfTU + a, v = tv * kMfTV + e - a * WC;
            float xv = 0.f, pv = 0.f;
            if (u < H && v < W) {
                const i64 c = (i64)u * W + v;
                xv = fmaf(af, p[c], x[c]);
                pv = fmaf(bf, p[c], -gt[c]);
            }
            xw[e] = xv;
            pw[e] = pv;
        }
        __syncthreads();
        float a = 0.f;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int ra = (threadIdx.x >> 6) + 4 * t, cb = threadIdx.x & 63;
            const int ui = tu * kMfTU + ra, vi = tv * kMfTV + cb;
            if (ui >= H || vi >= W) continue;
            const i64 u = (i64)ui * W + vi;
            const int o = ra * WC + cb;
            const float x0 = xw[o], p0 = pw[o];
            glbw((float *)P.x[dst])[u] = x0;
            glbw(P.p[dst])[u] = p0;
            pp += (double)p0 * (double)p0;
            pr += -(double)p0 * (double)gt[u];
            a += gen_prior_curv(st, H, W, ui, vi,
                                [&](int dy, int dx) { return xw[o + dy * WC + dx]; },
                                [&](int dy, int dx) { return pw[o + dy * WC + dx]; });
        }
        dreg = (double)a;
    } else {
        const i64 u = (i64)itm.ty * kGenRows + threadIdx.x;
        if (u < (i64)H * W) {
            const int ui = (int)(u / W), vi = (int)(u - (i64)ui * W);
            dreg = (double)gen_update(st, P, H, W, u, ui, vi, pp, pr);
        }
    }
    double v[4] = {0.0, dreg, pp, pr};
    block_sum_store<4, kGenRows>(v, partials + (i64)it * kNV, red);
}

// update, LR rows (an LR tile, or kGenRows ELL rows): the data part of the
// curvature along the new p (x, p the new iterate and direction).
// Matrix-free: A p of the new direction by the forward, A x of the new
// iterate as A x + alpha A p of the old one; both kept for the next trial.
__global__ void __launch_bounds__(kGenRows) k_gen_upd_lr(const Proj *projs, const Item *items,
                                                         const int *n_items, double *partials) {
    __shared__ double red[kNV * (kGenRows / 64)];
    extern __shared__ float zs[];   // the forward's warped window, sized by the launch
    const int it = blockIdx.x;
    if (it >= *n_items) return;
    const Item itm = items[it];
    if (itm.tx != 0) return;
    const Proj &P = projs[itm.proj];
    const ScgState &st = *P.st;
    if (!st.do_update) return;
    const AS4 OpDev &op = *cst(P.op);
    const int h = op.H / op.s, w = op.W / op.s;
    const int dst = st.upd_src ^ 1;
    const AS1 float *xn = glb((const float *)P.x[dst]);
    const AS1 float *pn = glb(P.p[dst]);
    auto fx = [&](i64 c) { return xn[c]; };
    auto fp = [&](i64 c) { return pn[c]; };
    const bool l1 = st.wt.data_p != 2;
    double dd = 0.0;
    if (op.mf) {
        int k, ti, tj, i, j;
        const int src = st.upd_src;
        const float af = st.alpha_f;
        mf_by_scale(op.s, [&](auto S) {
            for (int q = 0; q < kMfLRG && mf_lr_tile(op, itm.ty, q, k, ti, tj); ++q) {
                float ap[kMfCPT];
                mf_forward<S.value>(op, k, ti, tj, fp, zs, i, j, ap);
#pragma unroll
                for (int c = 0; c < kMfCPT; ++c)
                    if (i < h && j + 32 * c < w) {
                        const i64 row = ((i64)k * h + i) * w + j + 32 * c;
                        const float ax = fmaf(af, glb(P.ap[src])[row], glb(P.ax[src])[row]);
                        glbw(P.ax[dst])[row] = ax;
                        glbw(P.ap[dst])[row] = ap[c];
                        dd += gen_data_curv(st, P, row, ap[c], ax);
                    }
            }
        });
    } else {
        const i64 rows = (i64)op.K * h * w;
        const i64 r = (i64)itm.ty * kGenRows + threadIdx.x;
        if (r < rows) {
            const float ap = ell_row(glb(op.a_col), glb(op.a_val), op.a_w, rows, r, fp);
            const float ax = l1 ? ell_row(glb(op.a_col), glb(op.a_val), op.a_w, rows, r, fx) : 0.f;
            dd = gen_data_curv(st, P, r, ap, ax);
        }
    }
    double v[4] = {dd, 0.0, 0.0, 0.0};
    block_sum_store<4, kGenRows>(v, partials + (i64)it * kNV, red);
}

// standalone operators (FP32): y = A x over the LR rows, x = A^T r over the
// HR rows; matrix-free: one tile per workgroup
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

__global__ void __launch_bounds__(kGenRows) k_mf_forward(const OpDev *opp, const float *x,
                                                         float *y) {
    __shared__ float zs[kMfZ];
    const AS4 OpDev &op = *cst(opp);
    const int h = op.H / op.s, w = op.W / op.s;
    const AS1 float *xg = glb(x);
    int k, ti, tj, i, j;
    mf_by_scale(op.s, [&](auto S) {
        for (int q = 0; q < kMfLRG && mf_lr_tile(op, blockIdx.x, q, k, ti, tj); ++q) {
            float ax[kMfCPT];
            mf_forward<S.value>(op, k, ti, tj, [&](i64 c) { return xg[c]; }, zs, i, j, ax);
#pragma unroll
            for (int c = 0; c < kMfCPT; ++c)
                if (i < h && j + 32 * c < w) y[((i64)k * h + i) * w + j + 32 * c] = ax[c];
        }
    });
}

__global__ void __launch_bounds__(kGenRows) k_mf_adjoint(const OpDev *opp, const float *r,
                                                         float *x) {
    __shared__ float lds[kMfWin + kMfQP * kMfQP];
    const AS4 OpDev &op = *cst(opp);
    const int H = op.H, W = op.W, h = H / op.s, w = W / op.s;
    const AS1 float *rg = glb(r);
    const int ntv = (W + kMfTV - 1) / kMfTV;
    const int tu = blockIdx.x / ntv, tv = blockIdx.x - tu * ntv;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    mf_by_scale(op.s, [&](auto S) {
        mf_adjoint<S.value>(op, tu, tv,
                            [&](int k, int i, int j) { return rg[((i64)k * h + i) * w + j]; }, lds,
                            acc);
    });
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int pr = tu * kMfTU + (threadIdx.x >> 6) + 4 * t;
        const int pc = tv * kMfTV + (threadIdx.x & 63);
        if (pr < H && pc < W && (threadIdx.x >> 6) + 4 * t < kMfTU) x[(i64)pr * W + pc] = acc[t];
    }
}

// A pass over one class of general items: the trial and the cost+gradient
// run the LR rows then the HR rows, the update the HR rows then the LR rows.
hipError_t launch_general(int grid, hipStream_t stream, const Proj *projs, const Item *items,
                          const int *n_items, double *partials, int kind, int S) {
    if (grid <= 0) return hipSuccess;
    // the forward's warped window for the class's scale (any P)
    const size_t zb = (size_t)mf_zwin(S) * sizeof(float);
    if (kind == 2) {
        hipLaunchKernelGGL(k_gen_upd_hr, dim3(grid), dim3(kGenRows), 0, stream, projs, items,
                           n_items, partials);
        hipLaunchKernelGGL(k_gen_upd_lr, dim3(grid), dim3(kGenRows), zb, stream, projs, items,
                           n_items, partials);
    } else {
        const int mode = kind == 1 ? 1 : 0;
        hipLaunchKernelGGL(k_gen_trial_lr, dim3(grid), dim3(kGenRows), mode == 0 ? zb : 0, stream,
                           projs, items, n_items, partials, mode);
        hipLaunchKernelGGL(k_gen_trial_hr, dim3(grid), dim3(kGenRows), 0, stream, projs, items,
                           n_items, partials, mode);
    }
    return hipGetLastError();
}

hipError_t launch_general_forward(hipStream_t stream, const OpDev *op, long long rows,
                                  const float *x, float *y, long long mf_tiles) {
    if (mf_tiles > 0) {
        hipLaunchKernelGGL(k_mf_forward, dim3((unsigned)mf_tiles), dim3(kGenRows), 0, stream, op,
                           x, y);
        return hipGetLastError();
    }
    long long blocks = (rows + kGenRows - 1) / kGenRows;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_gen_forward, dim3((unsigned)blocks), dim3(kGenRows), 0, stream, op, x,
                       y);
    return hipGetLastError();
}

hipError_t launch_general_adjoint(hipStream_t stream, const OpDev *op, long long n,
                                  const float *r, float *x, long long mf_tiles) {
    if (mf_tiles > 0) {
        hipLaunchKernelGGL(k_mf_adjoint, dim3((unsigned)mf_tiles), dim3(kGenRows), 0, stream, op,
                           r, x);
        return hipGetLastError();
    }
    long long blocks = (n + kGenRows - 1) / kGenRows;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_gen_adjoint, dim3((unsigned)blocks), dim3(kGenRows), 0, stream, op, r,
                       x);
    return hipGetLastError();
}

}  // namespace misr
