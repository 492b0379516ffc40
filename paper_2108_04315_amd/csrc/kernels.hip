// kernels.hip -- gfx950 kernels of the MISR SCG hot path.
//
// Work decomposition: every image kernel walks a work list of (view, tile)
// items; a tile is TH x TW owned HR pixels (TH = S*TLY).  A workgroup stages
// the tile's window (owned pixels plus EXT = max(L-1, 2) on each side) into
// LDS once and runs every frame's separable band passes from there:
//
//   forward   A_k x  : pass 1 rows   (HR rows -> LR columns, L taps, stride S)
//                      pass 2 columns (HR rows -> LR rows,   L taps, stride S)
//   adjoint   A_k^T r: pass 3 columns (LR rows -> HR rows, gather, <= ceil(L/S) taps)
//                      pass 4 rows    (LR cols -> HR cols, gather)
//
// A_k = C_y,k (x) C_x,k holds exactly because the warp, the PSF and the
// binning of Eq. sisr are all separable (zero padding included), so one 2-D
// operator becomes two 1-D banded ones.  Inner products are accumulated in
// FP64 per thread and reduced per workgroup in a fixed order (deterministic).
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "internal.h"

namespace misr {

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ int fdiv(int a, int b) {
    int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}
__device__ __forceinline__ int cdiv(int a, int b) { return -fdiv(-a, b); }

__device__ __forceinline__ float ld_st(const void *base, long long i, int st) {
    if (st == ST_F32) return ((const float *)base)[i];
    if (st == ST_F16) return __half2float(((const __half *)base)[i]);
    return __bfloat162float(((const __hip_bfloat16 *)base)[i]);
}
__device__ __forceinline__ float round_st(float v, int st) {
    if (st == ST_F32) return v;
    if (st == ST_F16) return __half2float(__float2half(v));
    return __bfloat162float(__float2bfloat16(v));
}
__device__ __forceinline__ void st_st(void *base, long long i, float v, int st) {
    if (st == ST_F32)
        ((float *)base)[i] = v;
    else if (st == ST_F16)
        ((__half *)base)[i] = __float2half(v);
    else
        ((__hip_bfloat16 *)base)[i] = __float2bfloat16(v);
}

__device__ __forceinline__ float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Charbonnier penalty phi(z) = sqrt(z^2+e^2) - e, written z^2/(sqrt(z^2+e^2)+e)
// so that it has no cancellation; derivative psi(z) = z / sqrt(z^2+e^2).
__device__ __forceinline__ void phi_psi(float z, float eps, float e2, float &phi,
                                        float &psi) {
    if (eps == 0.f) {
        phi = fabsf(z);
        psi = (z > 0.f) ? 1.f : ((z < 0.f) ? -1.f : 0.f);
        return;
    }
    const float d = fmaf(z, z, e2);
    const float r = rsq(d);
    psi = z * r;
    phi = z * psi * rcp(fmaf(eps, r, 1.f));
}
__device__ __forceinline__ float psi_only(float z, float eps, float e2) {
    if (eps == 0.f) return (z > 0.f) ? 1.f : ((z < 0.f) ? -1.f : 0.f);
    return z * rsq(fmaf(z, z, e2));
}

// (psi(b + h) - psi(b)) / h, the finite-difference quotient Moller's curvature
// takes along one BTV pair.  Closed form without cancellation:
//   (e^2 + C) / (A B (A + B)),  A = |(a, e)|, B = |(b, e)|, C = A B - a b,
// with C = (e^2 (a^2 + b^2) + e^4) / (A B + a b) when a b > 0.  When |h| is
// below 1e-3 B the third-order Taylor series in h is used instead (remainder
// below float32 rounding).
__device__ __forceinline__ float psi_quot(float b, float h, float eps, float e2) {
    if (eps == 0.f) {
        if (h == 0.f) return 0.f;
        const float a = b + h;
        const float sa = (a > 0.f) ? 1.f : ((a < 0.f) ? -1.f : 0.f);
        const float sb = (b > 0.f) ? 1.f : ((b < 0.f) ? -1.f : 0.f);
        return (sa - sb) / h;
    }
    const float bb = fmaf(b, b, e2);
    const float rB = rsq(bb);
    const float rB2 = rB * rB;
    const float t = h * rB2;
    if (fabsf(h * rB) < 1e-3f) {
        const float poly = fmaf(0.5f * t * t, fmaf(4.f * b, b, -e2), fmaf(-1.5f * t, b, 1.f));
        return e2 * rB * rB2 * poly;
    }
    const float a = b + h;
    const float aa = fmaf(a, a, e2);
    const float rA = rsq(aa);
    const float A = aa * rA, B = bb * rB;
    const float AB = A * B, ab = a * b;
    const float C = (ab > 0.f) ? (e2 * (a * a + b * b) + e2 * e2) / (AB + ab) : AB - ab;
    return (e2 + C) * rA * rB / (A + B);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sums N per-thread values over the workgroup in a fixed order and stores them
// to out[0..N) (thread 0..N-1 write).  red: LDS scratch of N * kNT/64 doubles.
template <int N>
__device__ __forceinline__ void block_sum_store(double (&v)[N], double *out, double *red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) red[wid * N + i] = v[i];
    __syncthreads();
    if (threadIdx.x < N) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kNT / 64; ++w) s += red[w * N + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

// ------------------------------------------------------------ tile geometry
template <int S, int L>
struct Cfg {
    static constexpr int TL = (L > 10) ? ((32 / S) > 4 ? 32 / S : 4) : (S == 3 ? 16 : 64 / S);
    static constexpr int TH = S * TL, TW = S * TL;
    static constexpr int EXT = (L - 1 > 2) ? L - 1 : 2;
    static constexpr int WR = TH + 2 * EXT, WC = TW + 2 * EXT;
    static constexpr int WCP = WC + 1;
    static constexpr int NI = (TH + L - 2) / S + 1;
    static constexpr int NJ = (TW + L - 2) / S + 1;
    static constexpr int NR = S * (NI - 1) + L;
    static constexpr int NPX = (TH * TW + kNT - 1) / kNT;
    static constexpr int XS = WR * WCP;
    static constexpr int HX = (NR * NJ > TH * NJ) ? NR * NJ : TH * NJ;
    static constexpr int RS = NI * NJ;
    static constexpr int WY = NI * L, WX = NJ * L;
    // floats; +2*kNV*4 doubles of reduction scratch
    static constexpr int SMEM_TRIAL = XS + HX + RS + WY + WX;
    static constexpr int SMEM_UPD = 2 * XS + HX + WY + WX;
    static constexpr int SMEM = (SMEM_TRIAL > SMEM_UPD ? SMEM_TRIAL : SMEM_UPD);
    static_assert(NR <= WR, "window too small");
    static_assert(SMEM * 4 + 4 * kNV * 8 * 2 <= 160 * 1024, "LDS budget (gfx950: 160 KB per CU)");
};

// Stage frame k's band weights for LR rows [iA, iA+NI) and columns [jA, jA+NJ).
template <int L>
__device__ __forceinline__ void stage_weights(const OpDev &op, int k, int iA, int NI, int jA,
                                              int NJ, float *wys, float *wxs) {
    const int h = op.H / op.s, w = op.W / op.s;
    const float *gy = op.wy + ((long long)k * h + iA) * L;
    const float *gx = op.wx + ((long long)k * w + jA) * L;
    for (int q = threadIdx.x; q < NI * L; q += kNT) wys[q] = gy[q];
    for (int q = threadIdx.x; q < NJ * L; q += kNT) wxs[q] = gx[q];
}

// pass 1: hx[rr][jj] = sum_l wx[jj][l] * win[wr0 + rr][wc0 + S*jj + l]
template <int S, int L, int WCP>
__device__ __forceinline__ void pass_rows(const float *win, int wr0, int wc0, int NR, int NJ,
                                          const float *wxs, float *hx) {
    for (int q = threadIdx.x; q < NR * NJ; q += kNT) {
        const int rr = q / NJ, jj = q - rr * NJ;
        const float *xr = win + (wr0 + rr) * WCP + wc0 + S * jj;
        const float *wv = wxs + jj * L;
        float a = 0.f;
#pragma unroll
        for (int l = 0; l < L; ++l) a = fmaf(wv[l], xr[l], a);
        hx[q] = a;
    }
}

// ------------------------------------------------------------------ k_trial
// Fused cost + gradient at x_t = x + alpha p (mode 1) or at x (mode 0):
// every frame's forward, residual, data cost, adjoint; BTV cost and gradient;
// writes g_t = grad J(x_t) to g[cur^1] for the owned pixels and the partial
// sums {E_data, E_reg, |g_t|^2, g_t.g_k, g_t.p}.
template <int S, int L>
__device__ void tile_trial(const Proj &P, const ScgState &st, int ty, int tx, int mode,
                           int stype, float *sm, double *red, double *part) {
    using C = Cfg<S, L>;
    const OpDev &op = *P.op;
    const int tid = threadIdx.x;
    const int u0 = P.oy0 + ty * C::TH, v0 = P.ox0 + tx * C::TW;
    const int u1 = min(u0 + C::TH, P.oy1), v1 = min(v0 + C::TW, P.ox1);
    const int U0 = P.gy0 + u0, V0 = P.gx0 + v0;
    const int H = op.H, W = op.W, h = H / S, w = W / S;
    float *xs = sm;
    float *hx = xs + C::XS;
    float *rs = hx + C::HX;
    float *wys = rs + C::RS;
    float *wxs = wys + C::WY;

    const void *xb = P.x[st.xc];
    const float *pb = P.p[st.xc];
    const float af = (mode == 1) ? st.alpha_f : 0.f;
    for (int q = tid; q < C::WR * C::WC; q += kNT) {
        const int r = q / C::WC, c = q - r * C::WC;
        const int ub = u0 - C::EXT + r, vb = v0 - C::EXT + c;
        float val = 0.f;
        if (ub >= 0 && ub < P.Hb && vb >= 0 && vb < P.Wb) {
            const long long idx = (long long)ub * P.ld + vb;
            val = ld_st(xb, idx, stype);
            if (mode == 1) val = fmaf(af, pb[idx], val);
        }
        xs[r * C::WCP + c] = val;
    }
    float gacc[C::NPX];
#pragma unroll
    for (int m = 0; m < C::NPX; ++m) gacc[m] = 0.f;
    double e_data = 0.0;
    const int data_p = st.wt.data_p;
    const float epsd = st.wt.eps_data, e2d = epsd * epsd;
    __syncthreads();

    for (int k = 0; k < op.K; ++k) {
        const int offy = op.offy[k], offx = op.offx[k];
        const int iA = max(0, cdiv(U0 - L + 1 - offy, S));
        const int iB = min(h - 1, fdiv(U0 + C::TH - 1 - offy, S));
        const int jA = max(0, cdiv(V0 - L + 1 - offx, S));
        const int jB = min(w - 1, fdiv(V0 + C::TW - 1 - offx, S));
        const int NI = iB - iA + 1, NJ = jB - jA + 1;
        if (NI <= 0 || NJ <= 0) continue;
        stage_weights<L>(op, k, iA, NI, jA, NJ, wys, wxs);
        __syncthreads();
        const int NR = S * (NI - 1) + L;
        pass_rows<S, L, C::WCP>(xs, S * iA + offy - U0 + C::EXT, S * jA + offx - V0 + C::EXT,
                                NR, NJ, wxs, hx);
        __syncthreads();
        // pass 2 + residual + data cost (owned LR pixels only)
        const long long ybase = (long long)k * h * w;
        for (int q = tid; q < NI * NJ; q += kNT) {
            const int ii = q / NJ, jj = q - ii * NJ;
            const float *wv = wys + ii * L;
            float a = 0.f;
#pragma unroll
            for (int l = 0; l < L; ++l) a = fmaf(wv[l], hx[(S * ii + l) * NJ + jj], a);
            const int gi = iA + ii, gj = jA + jj;
            const float r = a - ld_st(P.y, ybase + (long long)gi * w + gj, stype);
            const bool own = (S * gi >= U0) && (S * gi < P.gy0 + u1) && (S * gj >= V0) &&
                             (S * gj < P.gx0 + v1);
            float rv;
            if (data_p == 2) {
                if (own) e_data += (double)r * (double)r;
                rv = 2.f * r;
            } else {
                float ph, ps;
                phi_psi(r, epsd, e2d, ph, ps);
                if (own) e_data += (double)ph;
                rv = ps;
            }
            rs[q] = rv;
        }
        __syncthreads();
        // pass 3: tt[uu][jj] = sum_i wy[i][U - S i - offy] * rs[i][jj]
        float *tt = hx;
        for (int q = tid; q < C::TH * NJ; q += kNT) {
            const int uu = q / NJ, jj = q - uu * NJ;
            const int U = U0 + uu;
            const int ilo = max(iA, cdiv(U - offy - L + 1, S)), ihi = min(iB, fdiv(U - offy, S));
            float a = 0.f;
            for (int i = ilo; i <= ihi; ++i)
                a = fmaf(wys[(i - iA) * L + (U - S * i - offy)], rs[(i - iA) * NJ + jj], a);
            tt[q] = a;
        }
        __syncthreads();
        // pass 4: g[uu][vv] += sum_j wx[j][V - S j - offx] * tt[uu][j]
#pragma unroll
        for (int m = 0; m < C::NPX; ++m) {
            const int q = tid + m * kNT;
            if (q >= C::TH * C::TW) break;
            const int uu = q / C::TW, vv = q - uu * C::TW;
            const int V = V0 + vv;
            const int jlo = max(jA, cdiv(V - offx - L + 1, S)), jhi = min(jB, fdiv(V - offx, S));
            float a = 0.f;
            for (int j = jlo; j <= jhi; ++j)
                a = fmaf(wxs[(j - jA) * L + (V - S * j - offx)], tt[uu * NJ + (j - jA)], a);
            gacc[m] += a;
        }
        __syncthreads();
    }

    // BTV prior (Eq. prior) at x_t: owned pairs (i, i+d) give the cost, both
    // pair directions give the gradient.
    const float eps = st.wt.eps, e2 = eps * eps;
    double e_reg = 0.0, gg = 0.0, ggk = 0.0, gp = 0.0;
    float *gout = P.g[st.cur ^ 1];
    const float *gk = P.g[st.cur];
#pragma unroll
    for (int m = 0; m < C::NPX; ++m) {
        const int q = tid + m * kNT;
        if (q >= C::TH * C::TW) break;
        const int uu = q / C::TW, vv = q - uu * C::TW;
        if (u0 + uu >= u1 || v0 + vv >= v1) continue;
        const int U = U0 + uu, V = V0 + vv;
        const float *c = xs + (uu + C::EXT) * C::WCP + vv + C::EXT;
        const float xi = c[0];
        float gb = 0.f, eb = 0.f;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                if (dx == 0 && dy == 0) continue;
                const float gam = st.wt.gam[dy * 3 + dx];
                if (gam == 0.f) continue;
                if (U + dy < H && V + dx < W) {
                    float ph, ps;
                    phi_psi(xi - c[dy * C::WCP + dx], eps, e2, ph, ps);
                    gb = fmaf(gam, ps, gb);
                    eb = fmaf(gam, ph, eb);
                }
                if (U - dy >= 0 && V - dx >= 0) {
                    gb = fmaf(-gam, psi_only(c[-dy * C::WCP - dx] - xi, eps, e2), gb);
                }
            }
        const float gv = gacc[m] + gb;
        e_reg += (double)eb;
        const long long idx = (long long)(u0 + uu) * P.ld + v0 + vv;
        gout[idx] = gv;
        gg += (double)gv * (double)gv;
        if (mode == 0) P.p[st.xc][idx] = 0.f;   // start direction buffer for the init pass
        if (mode == 1) {
            ggk += (double)gv * (double)gk[idx];
            gp += (double)gv * (double)pb[idx];
        }
    }
    double v[5] = {e_data, e_reg, gg, ggk, gp};
    block_sum_store<5>(v, part, red);
}

// ----------------------------------------------------------------- k_upcurv
// Accepted step: x <- x + alpha p, p <- -g_t + beta p (into the other buffer
// of each pair), then Moller's curvature at the new (x, p) without forming
// x + sigma_k p: data part 2 sum_k |A_k p|^2 (exact, the data term is
// quadratic), prior part lambda sum gamma q^2 Q(z, sigma_k q).  Partial sums
// {2 |A p|^2, prior part, |p|^2, p.r}.
template <int S, int L>
__device__ void tile_upcurv(const Proj &P, const ScgState &st, int ty, int tx, int stype,
                            float *sm, double *red, double *part) {
    using C = Cfg<S, L>;
    const OpDev &op = *P.op;
    const int tid = threadIdx.x;
    const int u0 = P.oy0 + ty * C::TH, v0 = P.ox0 + tx * C::TW;
    const int u1 = min(u0 + C::TH, P.oy1), v1 = min(v0 + C::TW, P.ox1);
    const int U0 = P.gy0 + u0, V0 = P.gx0 + v0;
    const int H = op.H, W = op.W;
    float *xs = sm;
    float *ps = xs + C::XS;
    float *hx = ps + C::XS;
    float *wys = hx + C::HX;
    float *wxs = wys + C::WY;

    const int src = st.upd_src, dst = src ^ 1;
    const void *xb = P.x[src];
    const float *pb = P.p[src];
    const float *gt = P.g[st.cur];
    const float af = st.alpha_f, bf = st.beta_f;
    for (int q = tid; q < C::WR * C::WC; q += kNT) {
        const int r = q / C::WC, c = q - r * C::WC;
        const int ub = u0 - C::EXT + r, vb = v0 - C::EXT + c;
        float xv = 0.f, pv = 0.f;
        if (ub >= 0 && ub < P.Hb && vb >= 0 && vb < P.Wb) {
            const long long idx = (long long)ub * P.ld + vb;
            const float p0 = pb[idx];
            xv = round_st(fmaf(af, p0, ld_st(xb, idx, stype)), stype);
            pv = fmaf(bf, p0, -gt[idx]);
        }
        xs[r * C::WCP + c] = xv;
        ps[r * C::WCP + c] = pv;
    }
    __syncthreads();
    // write the owned part of the new iterate; |p|^2 and p.r
    double pp = 0.0, pr = 0.0;
    void *xo = P.x[dst];
    float *po = P.p[dst];
    for (int q = tid; q < C::TH * C::TW; q += kNT) {
        const int uu = q / C::TW, vv = q - uu * C::TW;
        if (u0 + uu >= u1 || v0 + vv >= v1) continue;
        const long long idx = (long long)(u0 + uu) * P.ld + v0 + vv;
        const int wi = (uu + C::EXT) * C::WCP + vv + C::EXT;
        st_st(xo, idx, xs[wi], stype);
        const float pv = ps[wi];
        po[idx] = pv;
        pp += (double)pv * (double)pv;
        pr -= (double)pv * (double)gt[idx];
    }
    // data part: |A_k p|^2 over the owned LR pixels
    double ap2 = 0.0;
    const int NIo = (u1 - u0) / S, NJo = (v1 - v0) / S;
    const int iA = U0 / S, jA = V0 / S;
    if (NIo > 0 && NJo > 0) {
        for (int k = 0; k < op.K; ++k) {
            const int offy = op.offy[k], offx = op.offx[k];
            stage_weights<L>(op, k, iA, NIo, jA, NJo, wys, wxs);
            __syncthreads();
            const int NR = S * (NIo - 1) + L;
            pass_rows<S, L, C::WCP>(ps, offy + C::EXT, offx + C::EXT, NR, NJo, wxs, hx);
            __syncthreads();
            for (int q = tid; q < NIo * NJo; q += kNT) {
                const int ii = q / NJo, jj = q - ii * NJo;
                const float *wv = wys + ii * L;
                float a = 0.f;
#pragma unroll
                for (int l = 0; l < L; ++l) a = fmaf(wv[l], hx[(S * ii + l) * NJo + jj], a);
                ap2 += (double)a * (double)a;
            }
            __syncthreads();
        }
    }
    // prior part over owned pairs (i, i+d)
    const float eps = st.wt.eps, e2 = eps * eps, sk = st.sigk_f;
    double dreg = 0.0;
    for (int q = tid; q < C::TH * C::TW; q += kNT) {
        const int uu = q / C::TW, vv = q - uu * C::TW;
        if (u0 + uu >= u1 || v0 + vv >= v1) continue;
        const int U = U0 + uu, V = V0 + vv;
        const int wi = (uu + C::EXT) * C::WCP + vv + C::EXT;
        const float xi = xs[wi], pi = ps[wi];
        float acc = 0.f;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy)
#pragma unroll
            for (int dx = 0; dx < 3; ++dx) {
                if (dx == 0 && dy == 0) continue;
                const float gam = st.wt.gam[dy * 3 + dx];
                if (gam == 0.f || U + dy >= H || V + dx >= W) continue;
                const int o = dy * C::WCP + dx;
                const float z = xi - xs[wi + o];
                const float qd = pi - ps[wi + o];
                acc = fmaf(gam * qd * qd, psi_quot(z, sk * qd, eps, e2), acc);
            }
        dreg += (double)acc;
    }
    double v[4] = {2.0 * ap2, dreg, pp, pr};
    block_sum_store<4>(v, part, red);
}

// -------------------------------------------------------- standalone passes
// y[k] = A_k x on the owned LR pixels of one tile.
template <int S, int L>
__device__ void tile_forward(const Proj &P, int ty, int tx, int stype, void *yout, float *sm) {
    using C = Cfg<S, L>;
    const OpDev &op = *P.op;
    const int tid = threadIdx.x;
    const int u0 = P.oy0 + ty * C::TH, v0 = P.ox0 + tx * C::TW;
    const int u1 = min(u0 + C::TH, P.oy1), v1 = min(v0 + C::TW, P.ox1);
    const int U0 = P.gy0 + u0, V0 = P.gx0 + v0;
    const int h = op.H / S, w = op.W / S;
    float *xs = sm;
    float *hx = xs + C::XS;
    float *wys = hx + C::HX;
    float *wxs = wys + C::WY;
    for (int q = tid; q < C::WR * C::WC; q += kNT) {
        const int r = q / C::WC, c = q - r * C::WC;
        const int ub = u0 - C::EXT + r, vb = v0 - C::EXT + c;
        float val = 0.f;
        if (ub >= 0 && ub < P.Hb && vb >= 0 && vb < P.Wb)
            val = ld_st(P.x[0], (long long)ub * P.ld + vb, stype);
        xs[r * C::WCP + c] = val;
    }
    __syncthreads();
    const int NIo = (u1 - u0) / S, NJo = (v1 - v0) / S;
    const int iA = U0 / S, jA = V0 / S;
    if (NIo <= 0 || NJo <= 0) return;
    for (int k = 0; k < op.K; ++k) {
        const int offy = op.offy[k], offx = op.offx[k];
        stage_weights<L>(op, k, iA, NIo, jA, NJo, wys, wxs);
        __syncthreads();
        pass_rows<S, L, C::WCP>(xs, offy + C::EXT, offx + C::EXT, S * (NIo - 1) + L, NJo, wxs,
                                hx);
        __syncthreads();
        for (int q = tid; q < NIo * NJo; q += kNT) {
            const int ii = q / NJo, jj = q - ii * NJo;
            const float *wv = wys + ii * L;
            float a = 0.f;
#pragma unroll
            for (int l = 0; l < L; ++l) a = fmaf(wv[l], hx[(S * ii + l) * NJo + jj], a);
            st_st(yout, (long long)k * h * w + (long long)(iA + ii) * w + jA + jj, a, stype);
        }
        __syncthreads();
    }
}

// x = sum_k A_k^T r_k on the owned HR pixels of one tile (r staged per frame).
template <int S, int L>
__device__ void tile_adjoint(const Proj &P, int ty, int tx, int stype, const void *r,
                             float *xout, float *sm) {
    using C = Cfg<S, L>;
    const OpDev &op = *P.op;
    const int tid = threadIdx.x;
    const int u0 = P.oy0 + ty * C::TH, v0 = P.ox0 + tx * C::TW;
    const int u1 = min(u0 + C::TH, P.oy1), v1 = min(v0 + C::TW, P.ox1);
    const int U0 = P.gy0 + u0, V0 = P.gx0 + v0;
    const int h = op.H / S, w = op.W / S;
    float *tt = sm;
    float *rs = tt + C::HX;
    float *wys = rs + C::RS;
    float *wxs = wys + C::WY;
    float gacc[C::NPX];
#pragma unroll
    for (int m = 0; m < C::NPX; ++m) gacc[m] = 0.f;
    for (int k = 0; k < op.K; ++k) {
        const int offy = op.offy[k], offx = op.offx[k];
        const int iA = max(0, cdiv(U0 - L + 1 - offy, S));
        const int iB = min(h - 1, fdiv(U0 + C::TH - 1 - offy, S));
        const int jA = max(0, cdiv(V0 - L + 1 - offx, S));
        const int jB = min(w - 1, fdiv(V0 + C::TW - 1 - offx, S));
        const int NI = iB - iA + 1, NJ = jB - jA + 1;
        if (NI <= 0 || NJ <= 0) continue;
        stage_weights<L>(op, k, iA, NI, jA, NJ, wys, wxs);
        for (int q = tid; q < NI * NJ; q += kNT) {
            const int ii = q / NJ, jj = q - ii * NJ;
            rs[q] = ld_st(r, (long long)k * h * w + (long long)(iA + ii) * w + jA + jj, stype);
        }
        __syncthreads();
        for (int q = tid; q < C::TH * NJ; q += kNT) {
            const int uu = q / NJ, jj = q - uu * NJ;
            const int U = U0 + uu;
            const int ilo = max(iA, cdiv(U - offy - L + 1, S)), ihi = min(iB, fdiv(U - offy, S));
            float a = 0.f;
            for (int i = ilo; i <= ihi; ++i)
                a = fmaf(wys[(i - iA) * L + (U - S * i - offy)], rs[(i - iA) * NJ + jj], a);
            tt[q] = a;
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < C::NPX; ++m) {
            const int q = tid + m * kNT;
            if (q >= C::TH * C::TW) break;
            const int uu = q / C::TW, vv = q - uu * C::TW;
            const int V = V0 + vv;
            const int jlo = max(jA, cdiv(V - offx - L + 1, S)), jhi = min(jB, fdiv(V - offx, S));
            float a = 0.f;
            for (int j = jlo; j <= jhi; ++j)
                a = fmaf(wxs[(j - jA) * L + (V - S * j - offx)], tt[uu * NJ + (j - jA)], a);
            gacc[m] += a;
        }
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < C::NPX; ++m) {
        const int q = tid + m * kNT;
        if (q >= C::TH * C::TW) break;
        const int uu = q / C::TW, vv = q - uu * C::TW;
        if (u0 + uu >= u1 || v0 + vv >= v1) continue;
        xout[(long long)(u0 + uu) * P.ld + v0 + vv] = gacc[m];
    }
}

// -------------------------------------------------------------- the kernels
// Image kernels walk the work list with a grid stride; n_items is read from
// device memory so that one captured launch can serve a changing list.
enum Kind { K_COSTGRAD = 0, K_TRIAL = 1, K_UPCURV = 2 };

template <int S, int L>
__global__ void __launch_bounds__(kNT) k_image(const Proj *__restrict__ projs,
                                               const Item *__restrict__ items,
                                               const int *__restrict__ n_items,
                                               const ScgState *__restrict__ states,
                                               double *__restrict__ partials, int kind,
                                               int stype) {
    __shared__ float sm[Cfg<S, L>::SMEM];
    __shared__ double red[kNV * (kNT / 64)];
    const int n = *n_items;
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const Item itm = items[it];
        const Proj &P = projs[itm.proj];
        const ScgState &st = states[P.req];
        double *part = partials + (long long)it * kNV;
        if (kind == K_UPCURV) {
            if (!st.do_update) continue;
            tile_upcurv<S, L>(P, st, itm.ty, itm.tx, stype, sm, red, part);
        } else {
            if (kind == K_TRIAL && !st.active) continue;
            tile_trial<S, L>(P, st, itm.ty, itm.tx, kind, stype, sm, red, part);
        }
        __syncthreads();
    }
}

template <int S, int L>
__global__ void __launch_bounds__(kNT) k_forward(const Proj *__restrict__ projs,
                                                 const Item *__restrict__ items, int n,
                                                 int stype, void *yout) {
    __shared__ float sm[Cfg<S, L>::SMEM];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const Item itm = items[it];
        tile_forward<S, L>(projs[itm.proj], itm.ty, itm.tx, stype, yout, sm);
        __syncthreads();
    }
}

template <int S, int L>
__global__ void __launch_bounds__(kNT) k_adjoint(const Proj *__restrict__ projs,
                                                 const Item *__restrict__ items, int n,
                                                 int stype, const void *r, float *xout) {
    __shared__ float sm[Cfg<S, L>::SMEM];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const Item itm = items[it];
        tile_adjoint<S, L>(projs[itm.proj], itm.ty, itm.tx, stype, r, xout, sm);
        __syncthreads();
    }
}

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
}

// steps 6-9 of the pass
__device__ void scg_phase_b(ScgState &s, const double *v, IterRec *trace) {
    s.do_update = 0;
    if (!s.active) return;
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
        r.success = (s.do_update != 0);
        r.pad_ = 0;
    }
    s.k++;
    s.it++;
    if (s.it >= s.n_iter) s.active = 0;
}

__global__ void __launch_bounds__(kNT) k_scalar(ScgState *states, const int *n_states,
                                                const double *__restrict__ partials,
                                                IterRec *const *traces, int phase) {
    __shared__ double red[kNV * (kNT / 64)];
    __shared__ double tot[kNV];
    const int ns = *n_states;
    for (int sv = blockIdx.x; sv < ns; sv += gridDim.x) {
        ScgState &s = states[sv];
        bool need;
        if (phase == PH_INIT)
            need = true;
        else if (phase == PH_A)
            need = s.active && s.success;
        else
            need = s.active;
        __syncthreads();   // every thread has read the state before thread 0 writes it
        if (need) {
            double v[kNV] = {0, 0, 0, 0, 0, 0};
            for (int i = s.item0 + threadIdx.x; i < s.item0 + s.nitems; i += kNT)
#pragma unroll
                for (int q = 0; q < kNV; ++q) v[q] += partials[(long long)i * kNV + q];
            block_sum_store<kNV>(v, tot, red);
        }
        if (threadIdx.x == 0) {
            if (phase == PH_INIT)
                scg_init(s, tot);
            else if (phase == PH_A)
                scg_phase_a(s, tot);
            else
                scg_phase_b(s, tot, traces ? traces[sv] : nullptr);
        }
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
    block_sum_store<kNV>(v, tot, red);
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
__global__ void k_finalize(const Proj *__restrict__ projs, int nproj,
                           const ScgState *__restrict__ states, int stype) {
    for (int j = 0; j < nproj; ++j) {
        const Proj &P = projs[j];
        if (states[P.req].xc == 0) continue;
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

// ------------------------------------------------------------- dispatching
// Supported (S, L) instances; L is the operator's band length rounded up.
#define MISR_INSTANCES(X) \
    X(1, 2) X(1, 4) X(1, 8) X(1, 16) \
    X(2, 4) X(2, 6) X(2, 8) X(2, 9) X(2, 12) X(2, 16) \
    X(3, 6) X(3, 9) X(3, 10) X(3, 12) X(3, 16) \
    X(4, 8) X(4, 12) X(4, 16)

int padded_band(int S, int L) {
    static const int tab[5][7] = {{0}, {2, 4, 8, 16, 0}, {4, 6, 8, 9, 12, 16, 0},
                                  {6, 9, 10, 12, 16, 0}, {8, 12, 16, 0}};
    if (S < 1 || S > 4) return -1;
    for (int i = 0; tab[S][i]; ++i)
        if (tab[S][i] >= L) return tab[S][i];
    return -1;
}

int tile_hr(int S, int Lp) {
#define X(s, l) \
    if (S == s && Lp == l) return Cfg<s, l>::TH;
    MISR_INSTANCES(X)
#undef X
    return -1;
}

hipError_t launch_image(int S, int Lp, int grid, hipStream_t stream, const Proj *projs,
                        const Item *items, const int *n_items, const ScgState *states,
                        double *partials, int kind, int stype) {
#define X(s, l)                                                                           \
    if (S == s && Lp == l) {                                                              \
        hipLaunchKernelGGL((k_image<s, l>), dim3(grid), dim3(kNT), 0, stream, projs, items, \
                           n_items, states, partials, kind, stype);                       \
        return hipGetLastError();                                                         \
    }
    MISR_INSTANCES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_forward(int S, int Lp, int grid, hipStream_t stream, const Proj *projs,
                          const Item *items, int n, int stype, void *y) {
#define X(s, l)                                                                             \
    if (S == s && Lp == l) {                                                                \
        hipLaunchKernelGGL((k_forward<s, l>), dim3(grid), dim3(kNT), 0, stream, projs, items, \
                           n, stype, y);                                                    \
        return hipGetLastError();                                                           \
    }
    MISR_INSTANCES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_adjoint(int S, int Lp, int grid, hipStream_t stream, const Proj *projs,
                          const Item *items, int n, int stype, const void *r, float *x) {
#define X(s, l)                                                                             \
    if (S == s && Lp == l) {                                                                \
        hipLaunchKernelGGL((k_adjoint<s, l>), dim3(grid), dim3(kNT), 0, stream, projs, items, \
                           n, stype, r, x);                                                 \
        return hipGetLastError();                                                           \
    }
    MISR_INSTANCES(X)
#undef X
    return hipErrorInvalidValue;
}

hipError_t launch_scalar(int grid, hipStream_t stream, ScgState *states, const int *n_states,
                         const double *partials, IterRec *const *traces, int phase) {
    hipLaunchKernelGGL(k_scalar, dim3(grid), dim3(kNT), 0, stream, states, n_states, partials,
                       traces, phase);
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

hipError_t launch_finalize(hipStream_t stream, const Proj *projs, int nproj,
                           const ScgState *states, int stype) {
    hipLaunchKernelGGL(k_finalize, dim3(1024), dim3(256), 0, stream, projs, nproj, states,
                       stype);
    return hipGetLastError();
}

}  // namespace misr
