// image_kernels.hip -- gfx950 image kernels of the MISR SCG hot path, for one
// scale factor S (compiled once per S with -DMISR_SCALE=S).
//
// Work decomposition: every kernel walks a work list of (view, tile) items;
// a tile is TH x TW owned HR pixels.  A 512-thread workgroup stages the tile's
// window (owned pixels plus EXT = max(L-1, 2) on each side) into LDS once and
// runs every frame's separable band passes from there:
//
//   forward  A_k x  : pass 1 along rows    (HR rows -> LR columns, L taps, stride S)
//                     pass 2 along columns (HR rows -> LR rows,    L taps, stride S)
//   adjoint A_k^T r : pass 3 along columns (LR rows -> HR rows, ceil(L/S) taps)
//                     pass 4 along rows    (LR cols -> HR cols)
//
// A_k = C_y,k (x) C_x,k holds exactly because the warp, the PSF and the
// binning of the observation model (Sec. 3.1, Eq. sisr) are all separable,
// zero padding included, so each 2-D operator becomes two 1-D banded ones.
// Band weights are read per LR row/column from the operator's tables with
// wave-uniform (scalar) loads: every pass maps one weight row to one wave.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device_common.h"

#ifndef MISR_SCALE
#error "compile with -DMISR_SCALE=<s>"
#endif

namespace misr {

constexpr int kNTI = 512;          // threads per workgroup of the image kernels
constexpr int kNWI = kNTI / 64;    // waves per workgroup

// Tile shapes: variant 0 is the widest tile for which one 64-lane wave spans
// every tile dimension a pass maps to lanes and two workgroups fit a CU's LDS
// in both the trial and the update pass; variant 1 is about half as wide;
// variant 2 is a trial-kernel shape as wide as the trial pass's LDS alone
// allows (the update pass stages two windows), paired with variant 0's
// update shape.
template <int S, int L, int TV>
struct Tile {
    static constexpr int EXT = (L - 1 > 2) ? L - 1 : 2;   // window margin (HR px)
    static constexpr int NTAP = (L + S - 1) / S;         // adjoint taps per output
    static constexpr int CJ = 4;                         // pass 1 LR columns per wave step
    static constexpr int CI = 4;                         // pass 2 LR rows per wave step
    static constexpr int CU = (S == 4) ? 8 : 6;          // pass 3 HR rows per wave step
    static constexpr int calc_th() {
        int best = S;
        for (int th = S; th + 2 <= 64; th += S)
            if (S * ((th + L - 2) / S) + L <= 64) best = th;
        return best;
    }
    static constexpr int TH = calc_th();
    static constexpr int NIM = (TH + L - 2) / S + 1;     // LR rows touching the tile
    static constexpr int NRM = S * (NIM - 1) + L;        // HR rows those read
    static constexpr int odd(int v) { return (v % 2) ? v : v + 1; }
    // LDS floats of a tile tw wide: the trial pass's, and the update pass's
    // unless the shape is the trial kernel's own (variant 2)
    static constexpr int lds_floats(int tw) {
        const int wcp = odd(tw + 2 * EXT);
        const int njp = odd((tw + L - 2) / S + 1);
        const int xs = (TH + 2 * EXT) * wcp + S * CJ + 8;
        const int hx = NRM * njp + S * CI * njp;
        const int hr = hx + NIM * njp;
        const int gs = TH * (tw + 1);
        const int trial = xs + (hr > gs ? hr : gs) + TH * tw;   // + the owned p
        const int upd = 2 * xs + hx + NIM * njp;                // + A_k x for p = 1
        return (TV == 2 || trial > upd) ? trial : upd;
    }
    static constexpr int calc_tw() {
        int best = kNWI * S;
        for (int tw = kNWI * S; tw <= 1024; tw += kNWI * S)
            if ((tw + L - 2) / S + 1 <= 64 && lds_floats(tw) * 4 <= 79 * 1024) best = tw;
        // variant 1: about half as wide (more workgroups for small images)
        if (TV == 1) {
            const int half = best / 2 / (kNWI * S) * (kNWI * S);
            best = half > kNWI * S ? half : kNWI * S;
        }
        return best;
    }
    static constexpr int TW = calc_tw();
    static constexpr int WR = TH + 2 * EXT, WC = TW + 2 * EXT, WCP = odd(WC);
    static constexpr int NJM = (TW + L - 2) / S + 1;
    static constexpr int NJP = odd(NJM);
    static constexpr int CV = TW / kNWI;                 // pass 4 / prior columns per wave
    static constexpr int XS = WR * WCP + S * CJ + 8;
    static constexpr int HXS = NRM * NJP + S * CI * NJP;
    static constexpr int RSS = NIM * NJP;
    static constexpr int GP = TW + 1;                    // row stride of the LDS gradient
    static constexpr int SMEM = lds_floats(TW);
    static_assert(NRM <= 64 && TH + 2 <= 64 && NJM <= 64, "a wave spans a tile dimension");
    static_assert(CV % S == 0 && CU % S == 0, "phase-aligned groups");
    static constexpr int PO = XS + ((HXS + RSS > TH * GP) ? HXS + RSS : TH * GP);
    static_assert(TH * GP <= SMEM - XS && TH <= NRM, "LDS aliasing");
    static_assert(PO + TH * TW <= SMEM, "LDS: owned p of the trial pass");
};

// pass 1: hx[r][j] = sum_l wx[jA+j][l] win[wr0+r][wc0+S j+l], r < NR, j < NJ.
// Waves take groups of CJ LR columns (their weights are scalar loads), lanes
// take rows; each lane keeps the S(CJ-1)+L window samples it needs in
// registers.
template <int S, int L, int TV>
FI void pass1(const float *win, int wr0, int wc0, int NR, int NJ, const AS4 float *wxk, int jA,
              int jlast, float *hx) {
    using T = Tile<S, L, TV>;
    constexpr int CJ = T::CJ, NX = S * (CJ - 1) + L;
    const int lane = threadIdx.x & 63, wv = uni(threadIdx.x >> 6);
    for (int jg = wv; jg * CJ < NJ; jg += kNWI) {
        const int j0 = jg * CJ;
        // rows past the end of the table read its zero padding
        const AS4 float *wb = wxk + (jA + j0) * L;
        float wgt[CJ][L];
#pragma unroll
        for (int c = 0; c < CJ; ++c)
#pragma unroll
            for (int l = 0; l < L; ++l) wgt[c][l] = wb[c * L + l];
        if (lane < NR) {
            const float *src = win + (wr0 + lane) * T::WCP + wc0 + S * j0;
            float xv[NX];
#pragma unroll
            for (int t = 0; t < NX; ++t) xv[t] = src[t];
#pragma unroll
            for (int c = 0; c < CJ; ++c) {
                float a = 0.f;
#pragma unroll
                for (int l = 0; l < L; ++l) a = fmaf(wgt[c][l], xv[S * c + l], a);
                if (j0 + c < NJ) hx[lane * T::NJP + j0 + c] = a;
            }
        }
    }
}

// pass 2: a = sum_l wy[iA+i][l] hx[S i + l][j]; waves take groups of CI LR
// rows, lanes take LR columns; out(i, j, a) consumes each result.
template <int S, int L, int TV, class F>
FI void pass2(const float *hx, int NI, int NJ, const AS4 float *wyk, int iA, int ilast, F out) {
    using T = Tile<S, L, TV>;
    constexpr int CI = T::CI, NH = S * (CI - 1) + L;
    const int lane = threadIdx.x & 63, wv = uni(threadIdx.x >> 6);
    for (int ig = wv; ig * CI < NI; ig += kNWI) {
        const int i0 = ig * CI;
        const AS4 float *wb = wyk + (iA + i0) * L;
        float wgt[CI][L];
#pragma unroll
        for (int c = 0; c < CI; ++c)
#pragma unroll
            for (int l = 0; l < L; ++l) wgt[c][l] = wb[c * L + l];
        if (lane < NJ) {
            float hv[NH];
#pragma unroll
            for (int t = 0; t < NH; ++t) hv[t] = hx[(S * i0 + t) * T::NJP + lane];
            float av[CI];
#pragma unroll
            for (int c = 0; c < CI; ++c) {
                float a = 0.f;
#pragma unroll
                for (int l = 0; l < L; ++l) a = fmaf(wgt[c][l], hv[S * c + l], a);
                av[c] = a;
            }
            out(i0, lane, av);
        }
    }
}

// pass 3: tt[u][j] = sum_i wy[i][U - S i - offy] rs[i][j] for the TH rows.
// PH = (U0 - offy) mod S fixes every tap offset at compile time.
template <int S, int L, int TV, int PH>
FI void pass3_ph(const float *rs, float *tt, int U0, int offy, int iA, int iB, int NJ,
                 const AS4 float *wyk) {
    using T = Tile<S, L, TV>;
    constexpr int CU = T::CU, NTAP = T::NTAP;
    constexpr int NIG = (PH + CU - 1) / S + NTAP;
    const int lane = threadIdx.x & 63, wv = uni(threadIdx.x >> 6);
    for (int ug = wv; ug * CU < T::TH; ug += kNWI) {
        const int u0 = ug * CU;
        const int q0 = fdiv(U0 + u0 - offy, S);
        const int ib = q0 - (NTAP - 1);
        // LR rows outside [0, h) read the zero padding of the table (the
        // rows of a last tile past the image edge included: the padding
        // after each frame covers the widest compiled tile)
        const AS4 float *wb = wyk + ib * L;
        float wg[CU][NTAP];
#pragma unroll
        for (int c = 0; c < CU; ++c) {
            const int dq = (PH + c) / S, ph = (PH + c) % S;
#pragma unroll
            for (int m = 0; m < NTAP; ++m) {
                const int l = ph + S * m;
                wg[c][m] = (l < L) ? wb[(dq - m + NTAP - 1) * L + l] : 0.f;
            }
        }
        if (lane < NJ) {
            float rv[NIG];
#pragma unroll
            for (int t = 0; t < NIG; ++t) {
                const int i = ib + t;
                const float v = rs[(min(max(i, iA), iB) - iA) * T::NJP + lane];
                rv[t] = (i >= iA && i <= iB) ? v : 0.f;
            }
#pragma unroll
            for (int c = 0; c < CU; ++c) {
                const int dq = (PH + c) / S;
                float a = 0.f;
#pragma unroll
                for (int m = 0; m < NTAP; ++m) a = fmaf(wg[c][m], rv[dq - m + NTAP - 1], a);
                if (u0 + c < T::TH) tt[(u0 + c) * T::NJP + lane] = a;
            }
        }
    }
}

// pass 4: g[u][v] += sum_j wx[j][V - S j - offx] tt[u][j] for the wave's CV
// columns; lanes take rows (u = lane - 2).
template <int S, int L, int TV, int PH>
FI void pass4_ph(const float *tt, float (&gacc)[Tile<S, L, TV>::CV], int V0, int offx, int jA,
                 int jB, const AS4 float *wxk) {
    using T = Tile<S, L, TV>;
    constexpr int CV = T::CV, NTAP = T::NTAP;
    constexpr int NJG = (PH + CV - 1) / S + NTAP;
    const int lane = threadIdx.x & 63, wv = uni(threadIdx.x >> 6);
    const int u = lane - 2;
    const int cv0 = wv * CV;
    const int q0 = fdiv(V0 + cv0 - offx, S);
    const int jb = q0 - (NTAP - 1);
    const AS4 float *wb = wxk + jb * L;
    const int ur = min(max(u, 0), T::TH - 1);
    float tv[NJG];
#pragma unroll
    for (int t = 0; t < NJG; ++t) {
        const int j = jb + t;
        const float v = tt[ur * T::NJP + (min(max(j, jA), jB) - jA)];
        tv[t] = (j >= jA && j <= jB) ? v : 0.f;
    }
#pragma unroll
    for (int c = 0; c < CV; ++c) {
        const int dq = (PH + c) / S, ph = (PH + c) % S;
        float a = 0.f;
#pragma unroll
        for (int m = 0; m < NTAP; ++m) {
            const int l = ph + S * m;
            if (l < L) a = fmaf(wb[(dq - m + NTAP - 1) * L + l], tv[dq - m + NTAP - 1], a);
        }
        gacc[c] += a;
    }
}

template <int S, int L, int TV>
FI void pass3(int ph, const float *rs, float *tt, int U0, int offy, int iA, int iB, int NJ,
              const AS4 float *wyk) {
    if (ph == 0) pass3_ph<S, L, TV, 0>(rs, tt, U0, offy, iA, iB, NJ, wyk);
    if constexpr (S > 1) if (ph == 1) pass3_ph<S, L, TV, 1>(rs, tt, U0, offy, iA, iB, NJ, wyk);
    if constexpr (S > 2) if (ph == 2) pass3_ph<S, L, TV, 2>(rs, tt, U0, offy, iA, iB, NJ, wyk);
    if constexpr (S > 3) if (ph == 3) pass3_ph<S, L, TV, 3>(rs, tt, U0, offy, iA, iB, NJ, wyk);
}

template <int S, int L, int TV>
FI void pass4(int ph, const float *tt, float (&gacc)[Tile<S, L, TV>::CV], int V0, int offx, int jA,
              int jB, const AS4 float *wxk) {
    if (ph == 0) pass4_ph<S, L, TV, 0>(tt, gacc, V0, offx, jA, jB, wxk);
    if constexpr (S > 1) if (ph == 1) pass4_ph<S, L, TV, 1>(tt, gacc, V0, offx, jA, jB, wxk);
    if constexpr (S > 2) if (ph == 2) pass4_ph<S, L, TV, 2>(tt, gacc, V0, offx, jA, jB, wxk);
    if constexpr (S > 3) if (ph == 3) pass4_ph<S, L, TV, 3>(tt, gacc, V0, offx, jA, jB, wxk);
}

// The 8 BTV offsets d = (dx, dy) in [0, 2]^2 minus the origin (Eq. prior, w = 3).
__device__ constexpr int kDX[8] = {1, 2, 0, 1, 2, 0, 1, 2};
__device__ constexpr int kDY[8] = {0, 0, 1, 1, 1, 2, 2, 2};

// BTV prior on the window, swept left to right over the wave's CV columns
// with lanes on rows (u = lane - 2, two rows of halo).  Each pair (i, i+d)
// is evaluated once, by the lane of i; the pixel i+d takes the share back
// from the same lane's history (same row, dx columns earlier) or, for rows
// below, from the lane dy above through DPP lane shifts of the per-dy sums.
// The 3-column window and the 2-step history rotate through three register
// slots, so the loop is unrolled by three and nothing is moved.  Steps 0
// and 1 (columns cv0-2, cv0-1) only fill the history.  The gradient
// accumulates into gs (LDS, row stride GP).
template <int S, int L, int TV, bool EPS0, bool CHECK>
FI void btv_sweep(const float *xs, float *gs, const float (&gam)[8], float eps, int U0, int V0,
                  int H, int W, int th_own, int tw_own, double &e_reg) {
    using T = Tile<S, L, TV>;
    constexpr int NSTEP = T::CV + 2;
    const int lane = threadIdx.x & 63, wv = uni(threadIdx.x >> 6);
    const int u = lane - 2;
    const int cv0 = wv * T::CV;
    const int U = U0 + u;
    const int ur = min(u, T::TH - 1);
    const float e2 = eps * eps;
    const bool row_tile = u >= 0 && u < T::TH;
    const bool own_row = u >= 0 && u < (CHECK ? th_own : T::TH);
    // pair validity per row offset (both pixels inside the image)
    bool rok[3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) rok[dy] = !CHECK || (U >= 0 && U + dy < H);
    const float *base = xs + (T::EXT + ur) * T::WCP + T::EXT + cv0 - 2;
    float *grow = gs + max(u, 0) * T::GP + cv0 - 2;
    float win[3][3];    // win[dy][slot]: window column c (from cv0 - 2) sits in slot (c + 1) % 3
    float hist[3][8];   // hist[slot][d]: the step's lambda gamma_d psi(z_d), slot t % 3
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) {
        win[dy][1] = base[dy * T::WCP + 0];
        win[dy][2] = base[dy * T::WCP + 1];
    }
#pragma unroll
    for (int q = 0; q < 3; ++q)
#pragma unroll
        for (int d = 0; d < 8; ++d) hist[q][d] = 0.f;
    float gam_sum = 0.f;
#pragma unroll
    for (int d = 0; d < 8; ++d) gam_sum += gam[d];
    double eacc = 0.0;
    // step t handles column cv0 + t - 2 and loads window column t + 2 (slot t % 3)
    auto step = [&](auto slot_c, auto out_c, int t) {
        constexpr int Q = decltype(slot_c)::value;
        constexpr bool OUT = decltype(out_c)::value;
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) win[dy][Q] = base[dy * T::WCP + t + 2];
        const int v = cv0 + t - 2, V = V0 + v;
        bool cok[3];
#pragma unroll
        for (int dx = 0; dx < 3; ++dx) cok[dx] = !CHECK || (V >= 0 && V + dx < W);
        const float x0 = win[0][(Q + 1) % 3];
        // the prior's cost of the column; for interior tiles (every pair
        // valid) the sum of gamma_d B_d, B_d = |(z_d, eps)|, less eps times
        // the sum of the gamma_d, which shares gamma_d / B_d with the gradient
        float eb = 0.f;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const int dx = kDX[d], dy = kDY[d];
            const float z = x0 - win[dy][(Q + 1 + dx) % 3];
            if (EPS0) {
                const float ps = (z > 0.f) ? 1.f : ((z < 0.f) ? -1.f : 0.f);
                const bool valid = rok[dy] && cok[dx];
                hist[Q][d] = valid ? gam[d] * ps : 0.f;
                eb = fmaf(valid ? gam[d] : 0.f, fabsf(z), eb);
            } else if (CHECK) {
                const bool valid = rok[dy] && cok[dx];
                const float dd = fmaf(z, z, e2);
                const float r = rsq(dd);
                hist[Q][d] = valid ? gam[d] * (z * r) : 0.f;
                eb = fmaf(valid ? gam[d] : 0.f, fmaf(dd, r, -eps), eb);
            } else {
                const float dd = fmaf(z, z, e2);
                const float gr = gam[d] * rsq(dd);
                hist[Q][d] = gr * z;
                eb = fmaf(gr, dd, eb);
            }
        }
        if (!EPS0 && !CHECK) eb = fmaf(-eps, gam_sum, eb);
        if (OUT) {
            // shares of the pairs (i - d, i): from dx steps back, dy lanes up
            float own = 0.f, back[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const int dx = kDX[d], dy = kDY[d];
                own += hist[Q][d];
                back[dy] += hist[(Q + 3 - dx) % 3][d];
            }
            const float up = wave_shr1(back[1] + wave_shr1(back[2]));
            const float gsum = own - back[0] - up;
            if (row_tile) grow[t] += gsum;
            if (own_row && (!CHECK || v < tw_own)) eacc += (double)eb;
        }
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using F = std::false_type;
    using Tr = std::true_type;
    step(I0{}, F{}, 0);
    step(I1{}, F{}, 1);
    step(I2{}, Tr{}, 2);
#pragma unroll 1
    for (int t = 3; t + 2 < NSTEP; t += 3) {
        step(I0{}, Tr{}, t);
        step(I1{}, Tr{}, t + 1);
        step(I2{}, Tr{}, t + 2);
    }
    constexpr int REM = NSTEP % 3;   // steps after the last full group of three
    if constexpr (REM >= 1) step(I0{}, Tr{}, NSTEP - REM);
    if constexpr (REM >= 2) step(I1{}, Tr{}, NSTEP - REM + 1);
    e_reg += eacc;
}

// Curvature of the prior along p (Moller's step 2 without forming x + sk p):
// sum over owned pairs of gamma q^2 Q(z, sk q), z, q the pair differences of
// x and p.  Same sweep as btv_sweep (lanes on rows, waves on CV columns,
// 3-slot rotating windows, unrolled by three); [ru0,ru1) x [rv0,rv1) is the
// owned part of the tile.  With eps > 0 every pair first takes the
// first-order series of psi_quot, Q(z, h) = eps^2 / B^3 (1 - 3/2 h z / B^2),
// B = |(z, eps)|: in u = q / B the term is gamma eps^2 u^2 / B times
// (1 - 3/2 sk u z / B).  The next term of the series is at most 2 (h / B)^2
// relative, so for |h| / B = sk |u| < kCurvTau = 1e-4 the truncation stays
// below FP32 rounding; a lane with a pair beyond that recomputes its column
// with the closed form, so the common case takes one branch per column.
template <int S, int L, int TV, bool CHECK, bool EPS0>
FI void curv_sweep(const float *xs, const float *ps, const float (&gam)[8], float eps, float sk,
                   int U0, int V0, int H, int W, int ru0, int ru1, int rv0, int rv1,
                   double &dreg) {
    using T = Tile<S, L, TV>;
    constexpr int NSTEP = T::CV;
    const int lane = threadIdx.x & 63, wv = uni(threadIdx.x >> 6);
    const int u = lane;
    const int cv0 = wv * T::CV;
    const int U = U0 + u;
    const int ur = min(u, T::TH - 1);
    const float e2 = eps * eps;
    const bool own_row = CHECK ? (u >= ru0 && u < ru1) : (u < T::TH);
    bool rok[3];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) rok[dy] = !CHECK || (U + dy < H);
    const int off = (T::EXT + ur) * T::WCP + T::EXT + cv0;
    float wx[3][3], wp[3][3];   // [dy][slot]: window column c in slot c % 3
#pragma unroll
    for (int dy = 0; dy < 3; ++dy)
#pragma unroll
        for (int dx = 0; dx < 2; ++dx) {
            wx[dy][dx] = xs[off + dy * T::WCP + dx];
            wp[dy][dx] = ps[off + dy * T::WCP + dx];
        }
    float gq[8];   // gamma_d eps^2
#pragma unroll
    for (int d = 0; d < 8; ++d) gq[d] = gam[d] * e2;
    constexpr float kCurvTau = 1e-4f;
    const float c15 = -1.5f * sk;
    const float umax_ok = kCurvTau / sk;   // sk |u| < tau  <=>  |u| < tau / sk
    double acc = 0.0;
    // step t handles column cv0 + t and loads window column t + 2 (slot (t+2) % 3)
    auto step = [&](auto slot_c, int t) {
        constexpr int Q = decltype(slot_c)::value;   // slot of column t
#pragma unroll
        for (int dy = 0; dy < 3; ++dy) {
            wx[dy][(Q + 2) % 3] = xs[off + dy * T::WCP + t + 2];
            wp[dy][(Q + 2) % 3] = ps[off + dy * T::WCP + t + 2];
        }
        const int v = cv0 + t, V = V0 + v;
        float a = 0.f;
        if (EPS0) {
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const int dx = kDX[d], dy = kDY[d];
                const float z = wx[0][Q] - wx[dy][(Q + dx) % 3];
                const float qd = wp[0][Q] - wp[dy][(Q + dx) % 3];
                const float tq = gam[d] * qd * qd * psi_quot(z, sk * qd, eps, e2);
                if (CHECK)
                    a += (rok[dy] && V + dx < W) ? tq : 0.f;
                else
                    a += tq;
            }
        } else {
            float umax = 0.f;
#pragma unroll
            for (int d = 0; d < 8; ++d) {
                const int dx = kDX[d], dy = kDY[d];
                const float z = wx[0][Q] - wx[dy][(Q + dx) % 3];
                const float qd = wp[0][Q] - wp[dy][(Q + dx) % 3];
                const float rB = rsq(fmaf(z, z, e2));
                const float u = qd * rB;
                const float poly = fmaf(c15, u * (z * rB), 1.f);
                const float tq = (u * u) * rB * poly;
                umax = fmaxf(umax, fabsf(u));
                if (CHECK)
                    a = fmaf((rok[dy] && V + dx < W) ? gq[d] : 0.f, tq, a);
                else
                    a = fmaf(gq[d], tq, a);
            }
            if (!(umax < umax_ok)) {
                // some pair is beyond the series' range: the column again,
                // each such pair with the closed form
                a = 0.f;
#pragma unroll
                for (int d = 0; d < 8; ++d) {
                    const int dx = kDX[d], dy = kDY[d];
                    const float z = wx[0][Q] - wx[dy][(Q + dx) % 3];
                    const float qd = wp[0][Q] - wp[dy][(Q + dx) % 3];
                    const float rB = rsq(fmaf(z, z, e2));
                    const float u = qd * rB;
                    float tq;
                    if (fabsf(u) < umax_ok)
                        tq = gq[d] * ((u * u) * rB * fmaf(c15, u * (z * rB), 1.f));
                    else
                        tq = gam[d] * qd * qd * psi_quot(z, sk * qd, eps, e2);
                    if (CHECK)
                        a += (rok[dy] && V + dx < W) ? tq : 0.f;
                    else
                        a += tq;
                }
            }
        }
        const bool own = own_row && (!CHECK || (v >= rv0 && v < rv1));
        acc += own ? (double)a : 0.0;
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
#pragma unroll 1
    for (int t = 0; t + 2 < NSTEP; t += 3) {
        step(I0{}, t);
        step(I1{}, t + 1);
        step(I2{}, t + 2);
    }
    constexpr int REM = NSTEP % 3;
    if constexpr (REM >= 1) step(I0{}, NSTEP - REM);
    if constexpr (REM >= 2) step(I1{}, NSTEP - REM + 1);
    dreg += acc;
}

// --------------------------------------------------------------- the tiles
// Window staging by rows: wave wv takes window rows wv, wv + kNWI, ... (so
// every row quantity is wave-uniform and sits in scalar registers) and lane
// takes columns lane + 64 c.  Loads are issued unconditionally from clamped
// coordinates; elements outside the view are stored as zero.
template <class T>
struct WinMap {
    static constexpr int NR = (T::WR + kNWI - 1) / kNWI;   // rows per wave
    static constexpr int NC = (T::WC + 63) / 64;           // columns per lane
};
struct WinCol {
    int vb, vc;   // view column, clamped into the view
    bool in;      // inside the window and the view
};
template <class T>
FI WinCol win_col(int lane, int c, int v0, int Wb) {
    WinCol w;
    const int col = lane + 64 * c;
    w.vb = v0 - T::EXT + col;
    w.vc = min(max(w.vb, 0), Wb - 1);
    w.in = col < T::WC && w.vb >= 0 && w.vb < Wb;
    return w;
}

struct TileOrigin {
    int u0, v0, u1, v1, U0, V0;
};

template <int S, int L, int TV>
FI TileOrigin tile_origin(const AS4 Proj &P, int ty, int tx) {
    using T = Tile<S, L, TV>;
    TileOrigin o;
    o.u0 = P.oy0 + ty * T::TH;
    o.v0 = P.ox0 + tx * T::TW;
    o.u1 = min(o.u0 + T::TH, P.oy1);
    o.v1 = min(o.v0 + T::TW, P.ox1);
    o.U0 = P.gy0 + o.u0;
    o.V0 = P.gx0 + o.v0;
    return o;
}

// Fused cost + gradient at x_t = x + alpha p (mode 1) or at x (mode 0):
// every frame's forward, residual, data cost and adjoint, then the BTV cost
// and gradient; writes g_t = grad J(x_t) to g[cur^1] for the owned pixels and
// the partial sums {E_data, E_reg, |g_t|^2, g_t.g_k, g_t.p}.
template <int S, int L, int TV, class ST, class SY>
FI void tile_trial(const AS4 Proj &P, const AS4 ScgState &st, int ty, int tx, int mode,
                   float *sm, double *red, double *part) {
    using T = Tile<S, L, TV>;
    using raw = typename ST::raw;
    using rawy = typename SY::raw;
    const AS4 OpDev &op = *cst(P.op);
    int tid = threadIdx.x;
    // per-tile index arithmetic is recomputed rather than kept live across the
    // work-list loop (where it would be spilled)
    asm volatile("" : "+v"(tid));
    const TileOrigin o = tile_origin<S, L, TV>(P, ty, tx);
    const int H = op.H, W = op.W, h = H / S, w = W / S, K = op.K;
    float *xs = sm;
    float *hx = xs + T::XS;
    float *rs = hx + T::HXS;
    float *po = sm + T::PO;     // p at the owned pixels, for g_t . p

    const int xc = st.xc;
    const AS1 raw *xb = glb((const raw *)P.x[xc]);
    const AS1 float *pb = glb(P.p[xc]);
    const float af = (mode == 1) ? st.alpha_f : 0.f;
    const int Hb = P.Hb, Wb = P.Wb, ld = P.ld;
    const bool sr = st.wt.x_rounding == 1;
    const unsigned seed = st.rseed;
    const AS4 OpDev &opg = op;
    const i64 Wg = opg.W;
    // window of x_t into LDS: every load first (clamped, unconditional), then
    // the arithmetic, so that the loads are in flight together.  Global loads
    // are issued at raised wave priority (here, for g_k and for the frames):
    // the other workgroup on the CU is usually in a compute phase, and its
    // waves would otherwise delay the issue of the loads (measured: k_trial
    // 65.4 -> 64.0 us at 2048^2)
    using WM = WinMap<T>;
    const int lane0 = tid & 63, wv0 = uni(tid >> 6);
    WinCol wc[WM::NC];
#pragma unroll
    for (int c = 0; c < WM::NC; ++c) wc[c] = win_col<T>(lane0, c, o.v0, Wb);
    if (mode == 1) {
        float xr[WM::NR][WM::NC], pr[WM::NR][WM::NC];
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int r = 0; r < WM::NR; ++r) {
            const int ub = o.u0 - T::EXT + wv0 + kNWI * r;
            const i64 rb = (i64)min(max(ub, 0), Hb - 1) * ld;
#pragma unroll
            for (int c = 0; c < WM::NC; ++c) {
                xr[r][c] = ST::ld(xb + rb, wc[c].vc);
                pr[r][c] = pb[rb + wc[c].vc];
            }
        }
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int r = 0; r < WM::NR; ++r) {
            const int row = wv0 + kNWI * r, ub = o.u0 - T::EXT + row;
            if (row < T::WR) {
                const bool rin = ub >= 0 && ub < Hb;
                const int ou = row - T::EXT;
#pragma unroll
                for (int c = 0; c < WM::NC; ++c) {
                    const int col = lane0 + 64 * c, ov = col - T::EXT;
                    const float v = fmaf(af, pr[r][c], xr[r][c]);
                    const float vr =
                        sr ? ST::rnd_sr(v, pixel_hash((i64)(P.gy0 + ub) * Wg + P.gx0 + wc[c].vb,
                                                      seed))
                           : ST::rnd(v);
                    if (col < T::WC) xs[row * T::WCP + col] = (rin && wc[c].in) ? vr : 0.f;
                    if (ou >= 0 && ou < T::TH && ov >= 0 && ov < T::TW)
                        po[ou * T::TW + ov] = pr[r][c];
                }
            }
        }
    } else {
        float xr[WM::NR][WM::NC];
#pragma unroll
        for (int r = 0; r < WM::NR; ++r) {
            const int ub = o.u0 - T::EXT + wv0 + kNWI * r;
            const i64 rb = (i64)min(max(ub, 0), Hb - 1) * ld;
#pragma unroll
            for (int c = 0; c < WM::NC; ++c) xr[r][c] = ST::ld(xb + rb, wc[c].vc);
        }
#pragma unroll
        for (int r = 0; r < WM::NR; ++r) {
            const int row = wv0 + kNWI * r, ub = o.u0 - T::EXT + row;
            if (row < T::WR) {
                const bool rin = ub >= 0 && ub < Hb;
#pragma unroll
                for (int c = 0; c < WM::NC; ++c) {
                    const int col = lane0 + 64 * c;
                    if (col < T::WC) xs[row * T::WCP + col] = (rin && wc[c].in) ? xr[r][c] : 0.f;
                }
            }
        }
    }
    float gacc[T::CV];
#pragma unroll
    for (int c = 0; c < T::CV; ++c) gacc[c] = 0.f;
    double e_data = 0.0;
    const int data_p = st.wt.data_p;
    const float epsd = st.wt.eps_data, e2d = epsd * epsd;
    const AS1 rawy *yb = glb((const rawy *)P.y);
    const float yscale = st.wt.y_scale;
    __syncthreads();

    for (int k = 0; k < K; ++k) {
        const int offy = op.offy[k], offx = op.offx[k];
        const int iA = max(0, cdiv(o.U0 - L + 1 - offy, S));
        const int iB = min(h - 1, fdiv(o.U0 + T::TH - 1 - offy, S));
        const int jA = max(0, cdiv(o.V0 - L + 1 - offx, S));
        const int jB = min(w - 1, fdiv(o.V0 + T::TW - 1 - offx, S));
        const int NI = iB - iA + 1, NJ = jB - jA + 1;
        if (NI <= 0 || NJ <= 0) continue;
        const AS4 float *wyk = cst(op.wy) + (i64)k * op.fsy * L;
        const AS4 float *wxk = cst(op.wx) + (i64)k * op.fsx * L;
        pass1<S, L, TV>(xs, S * iA + offy - o.U0 + T::EXT, S * jA + offx - o.V0 + T::EXT,
                    S * (NI - 1) + L, NJ, wxk, jA, w - 1, hx);
        __syncthreads();
        const AS1 rawy *yk = yb + (i64)k * h * w;
        pass2<S, L, TV>(hx, NI, NJ, wyk, iA, h - 1, [&](int i0, int j, const float (&av)[T::CI]) {
            const int gj = jA + j;
            float yv[T::CI];
            __builtin_amdgcn_s_setprio(2);
#pragma unroll
            for (int c = 0; c < T::CI; ++c)
                yv[c] = SY::ld(yk, (i64)min(iA + i0 + c, h - 1) * w + gj) * yscale;
            __builtin_amdgcn_s_setprio(0);
            const bool own_j = (S * gj >= o.V0) && (S * gj < P.gx0 + o.v1);
#pragma unroll
            for (int c = 0; c < T::CI; ++c) {
                if (i0 + c >= NI) break;
                const int gi = iA + i0 + c;
                const float r = av[c] - yv[c];
                const bool own = own_j && (S * gi >= o.U0) && (S * gi < P.gy0 + o.u1);
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
                rs[(i0 + c) * T::NJP + j] = rv;
            }
        });
        __syncthreads();
        pass3<S, L, TV>(pmod(o.U0 - offy, S), rs, hx, o.U0, offy, iA, iB, NJ, wyk);
        __syncthreads();
        pass4<S, L, TV>(pmod(o.V0 - offx, S), hx, gacc, o.V0, offx, jA, jB, wxk);
        __syncthreads();
    }

    // data-term gradient to LDS (lanes hold rows), then the prior adds in place
    float *gs = hx;
    {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int u = lane - 2;
        if (u >= 0 && u < T::TH)
#pragma unroll
            for (int c = 0; c < T::CV; ++c) gs[u * T::GP + wv * T::CV + c] = gacc[c];
    }
    // the output pass's loads of g_k are issued here, so that they are in
    // flight during the prior's sweep (p at the owned pixels is in LDS)
    const int cur = st.cur;
    AS1 float *gout = glbw(P.g[cur ^ 1]);
    const AS1 float *gk = glb(P.g[cur]);
    AS1 float *pz = glbw(P.p[xc]);
    // owned pixels by rows as in the staging: wave wv0 takes tile rows
    // wv0 + kNWI r, lane takes columns lane0 + 64 c
    constexpr int ONR = (T::TH + kNWI - 1) / kNWI, ONC = (T::TW + 63) / 64;
    int ocol[ONC];     // clamped view column
    bool cown[ONC];    // column owned
#pragma unroll
    for (int c = 0; c < ONC; ++c) {
        const int col = lane0 + 64 * c;
        cown[c] = col < T::TW && o.v0 + col < o.v1;
        ocol[c] = min(o.v0 + col, o.v1 - 1);
    }
    // g_k at the owned pixels; the wide tile issues these loads before the
    // prior's sweep so that they are in flight during it, the narrow tile
    // (whose sweep leaves no registers to carry them) after it
    constexpr bool PRE = TV == 0;
    float gkv[ONR][ONC];
    auto load_gk = [&]() {
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int r = 0; r < ONR; ++r) {
            const i64 rb = (i64)min(o.u0 + wv0 + kNWI * r, o.u1 - 1) * ld;
#pragma unroll
            for (int c = 0; c < ONC; ++c) gkv[r][c] = gk[rb + ocol[c]];
        }
        __builtin_amdgcn_s_setprio(0);
    };
    if (PRE && mode == 1) load_gk();
    float gam[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) gam[d] = st.wt.gam[kDY[d] * 3 + kDX[d]];
    const float eps = st.wt.eps;
    double e_reg = 0.0;
    // interior tiles: every pair of the sweep lies inside the image, tile owned whole
    const bool inner = o.U0 >= 2 && o.V0 >= 2 && o.U0 + T::TH + 2 <= H &&
                       o.V0 + T::TW + 2 <= W && o.u1 - o.u0 == T::TH && o.v1 - o.v0 == T::TW;
    const int tho = o.u1 - o.u0, two = o.v1 - o.v0;
    if (eps == 0.f)
        btv_sweep<S, L, TV, true, true>(xs, gs, gam, eps, o.U0, o.V0, H, W, tho, two, e_reg);
    else if (inner)
        btv_sweep<S, L, TV, false, false>(xs, gs, gam, eps, o.U0, o.V0, H, W, tho, two, e_reg);
    else
        btv_sweep<S, L, TV, false, true>(xs, gs, gam, eps, o.U0, o.V0, H, W, tho, two, e_reg);
    __syncthreads();
    // owned gradient out, with its inner products (g_k is widened to double
    // only here: widened at its load, it would be carried across the sweep
    // in twice the registers)
    double gg = 0.0, ggk = 0.0, gp = 0.0;
    if (!PRE && mode == 1) load_gk();
    if (mode == 1)
#pragma unroll
        for (int r = 0; r < ONR; ++r)
#pragma unroll
            for (int c = 0; c < ONC; ++c) asm volatile("" : "+v"(gkv[r][c]));
#pragma unroll
    for (int r = 0; r < ONR; ++r) {
        const int row = wv0 + kNWI * r;
        if (row >= T::TH || o.u0 + row >= o.u1) continue;   // wave-uniform
        const i64 rb = (i64)(o.u0 + row) * ld;
#pragma unroll
        for (int c = 0; c < ONC; ++c) {
            if (!cown[c]) continue;
            const int col = lane0 + 64 * c;
            const float gv = gs[row * T::GP + col];
            gout[rb + ocol[c]] = gv;
            gg += (double)gv * (double)gv;
            // start direction buffer for the init pass (none when the caller
            // evaluates the cost and gradient alone without one)
            if (mode == 0 && pz) pz[rb + ocol[c]] = 0.f;
            if (mode == 1) {
                ggk += (double)gv * (double)gkv[r][c];
                gp += (double)gv * (double)po[row * T::TW + col];
            }
        }
    }
    double v[5] = {e_data, e_reg, gg, ggk, gp};
    block_sum_store<5, kNTI>(v, part, red);
}

// Data part of the curvature over the owned LR pixels (all edges are
// multiples of S): L2 (DP = 2), 2 |A_k p|^2, exact since the term is
// quadratic; L1 (DP = 1, Charbonnier), the sum of (A_k p)^2 Q(r, sk A_k p) with
// r = A_k x - y_k and Q the quotient the prior's pairs use.
template <int S, int L, int TV, class SY, int DP>
FI double upd_data_part(const AS4 Proj &P, const AS4 ScgState &st, const TileOrigin &o,
                        const float *xs, const float *ps, float *hx, float *ax, int NIo,
                        int NJo, int iA, int jA) {
    using T = Tile<S, L, TV>;
    using rawy = typename SY::raw;
    const AS4 OpDev &op = *cst(P.op);
    const int h = op.H / S, w = op.W / S, K = op.K;
    const float skd = st.sigk_f, epsd = st.wt.eps_data, e2d = epsd * epsd;
    const AS1 rawy *yb = glb((const rawy *)P.y);
    double ap2 = 0.0;
    for (int k = 0; k < K; ++k) {
        const int offy = op.offy[k], offx = op.offx[k];
        const AS4 float *wyk = cst(op.wy) + (i64)k * op.fsy * L;
        const AS4 float *wxk = cst(op.wx) + (i64)k * op.fsx * L;
        if (DP == 1) {
            pass1<S, L, TV>(xs, S * iA + offy - o.U0 + T::EXT, S * jA + offx - o.V0 + T::EXT,
                        S * (NIo - 1) + L, NJo, wxk, jA, w - 1, hx);
            __syncthreads();
            pass2<S, L, TV>(hx, NIo, NJo, wyk, iA, h - 1, [&](int i0, int j, const float (&av)[T::CI]) {
#pragma unroll
                for (int c = 0; c < T::CI; ++c)
                    if (i0 + c < NIo) ax[(i0 + c) * T::NJP + j] = av[c];
            });
            __syncthreads();
        }
        pass1<S, L, TV>(ps, S * iA + offy - o.U0 + T::EXT, S * jA + offx - o.V0 + T::EXT,
                    S * (NIo - 1) + L, NJo, wxk, jA, w - 1, hx);
        __syncthreads();
        const AS1 rawy *yk = yb + (i64)k * h * w;
        pass2<S, L, TV>(hx, NIo, NJo, wyk, iA, h - 1, [&](int i0, int j, const float (&av)[T::CI]) {
#pragma unroll
            for (int c = 0; c < T::CI; ++c) {
                if (i0 + c >= NIo) break;
                if (DP == 2) {
                    ap2 += (double)av[c] * (double)av[c];
                } else {
                    const float r = ax[(i0 + c) * T::NJP + j] -
                                    SY::ld(yk, (i64)(iA + i0 + c) * w + jA + j) *
                                        st.wt.y_scale;
                    ap2 += (double)(av[c] * av[c] * psi_quot(r, skd * av[c], epsd, e2d));
                }
            }
        });
        __syncthreads();
    }
    return DP == 2 ? 2.0 * ap2 : ap2;
}

// Accepted step: x <- x + alpha p, p <- -g_t + beta p (into the other buffer
// of each pair), then Moller's curvature at the new (x, p) without forming
// x + sigma_k p: data part 2 sum_k |A_k p|^2 for the L2 term (exact: it is
// quadratic) or sum_k (A_k p)^2 Q(A_k x - y_k, sigma_k A_k p) for the L1
// (Charbonnier) term, prior part lambda sum gamma q^2 Q(z, sigma_k q).
// Partial sums {data part, prior part, |p|^2, p.r}.
template <int S, int L, int TV, class ST, class SY>
FI void tile_upcurv(const AS4 Proj &P, const AS4 ScgState &st, int ty, int tx, float *sm,
                    double *red, double *part) {
    static_assert(TV != 2, "the trial kernel's own tile shape");
    using T = Tile<S, L, TV>;
    using raw = typename ST::raw;
    const AS4 OpDev &op = *cst(P.op);
    int tid = threadIdx.x;
    // per-tile index arithmetic is recomputed rather than kept live across the
    // work-list loop (where it would be spilled)
    asm volatile("" : "+v"(tid));
    // update tiles cover the update rectangle (owned plus halo); reductions
    // count only their intersection with the owned rectangle [ou0,ou1) x [ov0,ov1)
    TileOrigin o;
    o.u0 = P.uy0 + ty * T::TH;
    o.v0 = P.ux0 + tx * T::TW;
    o.u1 = min(o.u0 + T::TH, P.uy1);
    o.v1 = min(o.v0 + T::TW, P.ux1);
    o.U0 = P.gy0 + o.u0;
    o.V0 = P.gx0 + o.v0;
    const int ou0 = max(o.u0, P.oy0), ou1 = min(o.u1, P.oy1);
    const int ov0 = max(o.v0, P.ox0), ov1 = min(o.v1, P.ox1);
    const int H = op.H, W = op.W, h = H / S, w = W / S, K = op.K;
    float *xs = sm;
    float *ps = xs + T::XS;
    float *hx = ps + T::XS;
    float *ax = hx + T::HXS;    // A_k x at the owned LR pixels (L1 data term)

    const int src = st.upd_src, dst = src ^ 1;
    const AS1 raw *xb = glb((const raw *)P.x[src]);
    const AS1 float *pb = glb(P.p[src]);
    const AS1 float *gt = glb(P.g[st.cur]);
    AS1 raw *xo = glbw((raw *)P.x[dst]);
    AS1 float *po = glbw(P.p[dst]);
    const float af = st.alpha_f, bf = st.beta_f;
    const int Hb = P.Hb, Wb = P.Wb, ld = P.ld;
    const bool sr = st.wt.x_rounding == 1;
    const unsigned seed = st.rseed;
    const i64 Wg = W;
    double pp = 0.0, pr = 0.0;
    {
        // every load first (clamped, unconditional, at raised wave priority
        // as in the trial pass), then the update
        using WM = WinMap<T>;
        const int lane0 = tid & 63, wv0 = uni(tid >> 6);
        WinCol wc[WM::NC];
#pragma unroll
        for (int c = 0; c < WM::NC; ++c) wc[c] = win_col<T>(lane0, c, o.v0, Wb);
        float xr[WM::NR][WM::NC], pr0[WM::NR][WM::NC], gr[WM::NR][WM::NC];
        __builtin_amdgcn_s_setprio(2);
#pragma unroll
        for (int r = 0; r < WM::NR; ++r) {
            const int ub = o.u0 - T::EXT + wv0 + kNWI * r;
            const i64 rb = (i64)min(max(ub, 0), Hb - 1) * ld;
#pragma unroll
            for (int c = 0; c < WM::NC; ++c) {
                xr[r][c] = ST::ld(xb + rb, wc[c].vc);
                pr0[r][c] = pb[rb + wc[c].vc];
                gr[r][c] = gt[rb + wc[c].vc];
            }
        }
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int r = 0; r < WM::NR; ++r) {
            const int row = wv0 + kNWI * r, ub = o.u0 - T::EXT + row;
            if (row < T::WR) {
                const bool rin = ub >= 0 && ub < Hb;
                const bool urow = rin && ub >= o.u0 && ub < o.u1;   // updated rows
                const bool orow = ub >= ou0 && ub < ou1;            // owned rows
                const i64 rb = (i64)ub * ld;                        // in the view when urow
#pragma unroll
                for (int c = 0; c < WM::NC; ++c) {
                    const int col = lane0 + 64 * c, vb = wc[c].vb;
                    const bool in = rin && wc[c].in;
                    const float v = fmaf(af, pr0[r][c], xr[r][c]);
                    float xv = sr ? ST::rnd_sr(v, pixel_hash((i64)(P.gy0 + ub) * Wg + P.gx0 + vb,
                                                             seed))
                                  : ST::rnd(v);
                    float pv = fmaf(bf, pr0[r][c], -gr[r][c]);
                    xv = in ? xv : 0.f;
                    pv = in ? pv : 0.f;
                    if (urow && wc[c].in && vb >= o.v0 && vb < o.v1) {
                        ST::st(xo, rb + vb, xv);
                        po[rb + vb] = pv;
                        if (orow && vb >= ov0 && vb < ov1) {
                            pp += (double)pv * (double)pv;
                            pr -= (double)pv * (double)gr[r][c];
                        }
                    }
                    if (col < T::WC) {
                        xs[row * T::WCP + col] = xv;
                        ps[row * T::WCP + col] = pv;
                    }
                }
            }
        }
    }
    __syncthreads();
    // data part over the owned LR pixels (all edges are multiples of S): L2,
    // 2 |A_k p|^2 (exact, the term is quadratic); L1 (Charbonnier), the sum of
    // (A_k p)^2 Q(r, sk A_k p) with r = A_k x - y_k, the same quotient as the
    // prior's pairs
    double ap2 = 0.0;
    const int NIo = (ou1 - ou0) / S, NJo = (ov1 - ov0) / S;
    const int iA = (P.gy0 + ou0) / S, jA = (P.gx0 + ov0) / S;
    const int data_p = st.wt.data_p;
    if (NIo > 0 && NJo > 0) {
        if (data_p == 2)
            ap2 = upd_data_part<S, L, TV, SY, 2>(P, st, o, xs, ps, hx, ax, NIo, NJo, iA, jA);
        else
            ap2 = upd_data_part<S, L, TV, SY, 1>(P, st, o, xs, ps, hx, ax, NIo, NJo, iA, jA);
    }
    // prior part over the owned pairs (i, i+d)
    const float eps = st.wt.eps, sk = st.sigk_f;
    float gam[8];
#pragma unroll
    for (int d = 0; d < 8; ++d) gam[d] = st.wt.gam[kDY[d] * 3 + kDX[d]];
    double dreg = 0.0;
    const int ru0 = ou0 - o.u0, ru1 = ou1 - o.u0, rv0 = ov0 - o.v0, rv1 = ov1 - o.v0;
    const bool inner = o.U0 + T::TH + 2 <= H && o.V0 + T::TW + 2 <= W && ru0 == 0 &&
                       ru1 == T::TH && rv0 == 0 && rv1 == T::TW;
    if (eps == 0.f)
        curv_sweep<S, L, TV, true, true>(xs, ps, gam, eps, sk, o.U0, o.V0, H, W, ru0, ru1, rv0, rv1,
                                     dreg);
    else if (inner)
        curv_sweep<S, L, TV, false, false>(xs, ps, gam, eps, sk, o.U0, o.V0, H, W, ru0, ru1, rv0,
                                       rv1, dreg);
    else
        curv_sweep<S, L, TV, true, false>(xs, ps, gam, eps, sk, o.U0, o.V0, H, W, ru0, ru1, rv0,
                                      rv1, dreg);
    double v[4] = {ap2, dreg, pp, pr};
    block_sum_store<4, kNTI>(v, part, red);
}

// y[k] = A_k x on the owned LR pixels of one tile.
template <int S, int L, int TV, class ST>
FI void tile_forward(const AS4 Proj &P, int ty, int tx, void *yout, float *sm) {
    using T = Tile<S, L, TV>;
    using raw = typename ST::raw;
    const AS4 OpDev &op = *cst(P.op);
    int tid = threadIdx.x;
    // per-tile index arithmetic is recomputed rather than kept live across the
    // work-list loop (where it would be spilled)
    asm volatile("" : "+v"(tid));
    const TileOrigin o = tile_origin<S, L, TV>(P, ty, tx);
    const int h = op.H / S, w = op.W / S, K = op.K;
    float *xs = sm;
    float *hx = xs + T::XS;
    const AS1 raw *xb = glb((const raw *)P.x[0]);
    const int Hb = P.Hb, Wb = P.Wb, ld = P.ld;
    for (int q = tid; q < T::WR * T::WC; q += kNTI) {
        const int r = q / T::WC, c = q - r * T::WC;
        const int ub = o.u0 - T::EXT + r, vb = o.v0 - T::EXT + c;
        float val = 0.f;
        if (ub >= 0 && ub < Hb && vb >= 0 && vb < Wb) val = ST::ld(xb, (i64)ub * ld + vb);
        xs[r * T::WCP + c] = val;
    }
    __syncthreads();
    const int NIo = (o.u1 - o.u0) / S, NJo = (o.v1 - o.v0) / S;
    const int iA = o.U0 / S, jA = o.V0 / S;
    if (NIo <= 0 || NJo <= 0) return;
    AS1 raw *yo = glbw((raw *)yout);
    for (int k = 0; k < K; ++k) {
        const int offy = op.offy[k], offx = op.offx[k];
        const AS4 float *wyk = cst(op.wy) + (i64)k * op.fsy * L;
        const AS4 float *wxk = cst(op.wx) + (i64)k * op.fsx * L;
        pass1<S, L, TV>(xs, offy + T::EXT, offx + T::EXT, S * (NIo - 1) + L, NJo, wxk, jA, w - 1, hx);
        __syncthreads();
        const i64 yb = (i64)k * h * w;
        pass2<S, L, TV>(hx, NIo, NJo, wyk, iA, h - 1, [&](int i0, int j, const float (&av)[T::CI]) {
#pragma unroll
            for (int c = 0; c < T::CI; ++c)
                if (i0 + c < NIo) ST::st(yo, yb + (i64)(iA + i0 + c) * w + jA + j, av[c]);
        });
        __syncthreads();
    }
}

// x = sum_k A_k^T r_k on the owned HR pixels of one tile.
template <int S, int L, int TV, class ST>
FI void tile_adjoint(const AS4 Proj &P, int ty, int tx, const void *r, float *xout, float *sm) {
    using T = Tile<S, L, TV>;
    using raw = typename ST::raw;
    const AS4 OpDev &op = *cst(P.op);
    int tid = threadIdx.x;
    // per-tile index arithmetic is recomputed rather than kept live across the
    // work-list loop (where it would be spilled)
    asm volatile("" : "+v"(tid));
    const TileOrigin o = tile_origin<S, L, TV>(P, ty, tx);
    const int h = op.H / S, w = op.W / S, K = op.K;
    float *gs = sm;
    float *tt = gs + T::XS;
    float *rs = tt + T::HXS;
    const AS1 raw *rb = glb((const raw *)r);
    float gacc[T::CV];
#pragma unroll
    for (int c = 0; c < T::CV; ++c) gacc[c] = 0.f;
    for (int k = 0; k < K; ++k) {
        const int offy = op.offy[k], offx = op.offx[k];
        const int iA = max(0, cdiv(o.U0 - L + 1 - offy, S));
        const int iB = min(h - 1, fdiv(o.U0 + T::TH - 1 - offy, S));
        const int jA = max(0, cdiv(o.V0 - L + 1 - offx, S));
        const int jB = min(w - 1, fdiv(o.V0 + T::TW - 1 - offx, S));
        const int NI = iB - iA + 1, NJ = jB - jA + 1;
        if (NI <= 0 || NJ <= 0) continue;
        const AS4 float *wyk = cst(op.wy) + (i64)k * op.fsy * L;
        const AS4 float *wxk = cst(op.wx) + (i64)k * op.fsx * L;
        for (int q = tid; q < NI * T::NJP; q += kNTI) {
            const int ii = q / T::NJP, jj = q - ii * T::NJP;
            if (jj < NJ) rs[q] = ST::ld(rb, (i64)k * h * w + (i64)(iA + ii) * w + jA + jj);
        }
        __syncthreads();
        pass3<S, L, TV>(pmod(o.U0 - offy, S), rs, tt, o.U0, offy, iA, iB, NJ, wyk);
        __syncthreads();
        pass4<S, L, TV>(pmod(o.V0 - offx, S), tt, gacc, o.V0, offx, jA, jB, wxk);
        __syncthreads();
    }
    {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        const int u = lane - 2;
        if (u >= 0 && u < T::TH)
#pragma unroll
            for (int c = 0; c < T::CV; ++c) gs[u * T::GP + wv * T::CV + c] = gacc[c];
    }
    __syncthreads();
    AS1 float *xo = glbw(xout);
    const int ld = P.ld;
    for (int q = tid; q < T::TH * T::TW; q += kNTI) {
        const int uu = q / T::TW, vv = q - uu * T::TW;
        if (o.u0 + uu >= o.u1 || o.v0 + vv >= o.v1) continue;
        xo[(i64)(o.u0 + uu) * ld + o.v0 + vv] = gs[uu * T::GP + vv];
    }
}

// -------------------------------------------------------------- the kernels
// The item count is read from device memory so that one captured launch can
// serve a changing list; the trial and update kernels are launched with one
// workgroup per item, the standalone operators walk the list with a grid
// stride.
//
// Workgroups are dispatched to the 8 XCDs round-robin in blockIdx order, and
// each XCD has its own L2.  With one workgroup per item, workgroup b takes
// item xcd_item(b, n): XCD b % 8 gets one contiguous run of the list (a band
// of neighbouring tiles), so the halos neighbouring tiles share are re-read
// from that XCD's L2 rather than fetched again.
FI int xcd_item(int b, int n) {
    const int q = n >> 3, r = n & 7, x = b & 7, j = b >> 3;
    return x * q + min(x, r) + j;
}
template <int S, int L, int TV, class ST, class SY>
__global__ void __launch_bounds__(kNTI, 4) k_trial(const Proj *projs, const Item *items,
                                                const int *n_items, double *partials,
                                                int mode) {
    __shared__ float sm[Tile<S, L, TV>::SMEM];
    __shared__ double red[kNV * kNWI];
    // one workgroup per item (the launch grid is the item count): no loop, so
    // nothing is hoisted out of one and kept live through the tile
    const int n = *cst(n_items);
    const int b = blockIdx.x;
    if (b >= n) return;
    const int it = (int)gridDim.x == n ? xcd_item(b, n) : b;
    const AS4 Item &itm = cst(items)[it];
    const AS4 Proj &P = cst(projs)[itm.proj];
    const AS4 ScgState &st = *cst(P.st);
    if (mode == 1 && !st.active) return;
    tile_trial<S, L, TV, ST, SY>(P, st, itm.ty, itm.tx, mode, sm, red, partials + (i64)it * kNV);
}

template <int S, int L, int TV, class ST, class SY>
__global__ void __launch_bounds__(kNTI, 4) k_upcurv(const Proj *projs, const Item *items,
                                                 const int *n_items, double *partials) {
    __shared__ float sm[Tile<S, L, TV>::SMEM];
    __shared__ double red[kNV * kNWI];
    const int n = *cst(n_items);
    const int b = blockIdx.x;
    if (b >= n) return;
    const int it = (int)gridDim.x == n ? xcd_item(b, n) : b;
    const AS4 Item &itm = cst(items)[it];
    const AS4 Proj &P = cst(projs)[itm.proj];
    const AS4 ScgState &st = *cst(P.st);
    if (!st.do_update) return;
    tile_upcurv<S, L, TV, ST, SY>(P, st, itm.ty, itm.tx, sm, red, partials + (i64)it * kNV);
}

template <int S, int L, int TV, class ST>
__global__ void __launch_bounds__(kNTI) k_forward(const Proj *projs, const Item *items, int n,
                                                  void *yout) {
    __shared__ float sm[Tile<S, L, TV>::SMEM];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const AS4 Item &itm = cst(items)[it];
        tile_forward<S, L, TV, ST>(cst(projs)[itm.proj], itm.ty, itm.tx, yout, sm);
        __syncthreads();
    }
}

template <int S, int L, int TV, class ST>
__global__ void __launch_bounds__(kNTI) k_adjoint(const Proj *projs, const Item *items, int n,
                                                  const void *r, float *xout) {
    __shared__ float sm[Tile<S, L, TV>::SMEM];
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const AS4 Item &itm = cst(items)[it];
        tile_adjoint<S, L, TV, ST>(cst(projs)[itm.proj], itm.ty, itm.tx, r, xout, sm);
        __syncthreads();
    }
}

// --------------------------------------------------- launchers for this S
// Band lengths instantiated per scale (the operator's L is rounded up).
#if MISR_SCALE == 1
#define MISR_LIST(X) X(4) X(8) X(16)
#elif MISR_SCALE == 2
#define MISR_LIST(X) X(6) X(8) X(9) X(12) X(16)
#elif MISR_SCALE == 3
#define MISR_LIST(X) X(6) X(9) X(10) X(12) X(16)
#elif MISR_SCALE == 4
#define MISR_LIST(X) X(12) X(16)
#endif

#define MISR_CAT2(a, b) a##b
#define MISR_CAT(a, b) MISR_CAT2(a, b)
#define MISR_FN(name) MISR_CAT(name, MISR_SCALE)

// Kernel keys: key = Lp | (tile variant << 8); variant 0 is the widest tile
// that fits, variant 1 about half as wide (chosen per operator by the tile
// autotuner).
// the update pass and the operators: variant 2 runs variant 0's shape
#define MISR_VARIANT(key, BODY) \
    if (((key) >> 8) == 1) {    \
        constexpr int tv = 1;   \
        BODY                    \
    } else {                    \
        constexpr int tv = 0;   \
        BODY                    \
    }
// the trial pass: every variant is its own shape
#define MISR_VARIANT_TRIAL(key, BODY) \
    if (((key) >> 8) == 0) {          \
        constexpr int tv = 0;         \
        BODY                          \
    } else if (((key) >> 8) == 1) {   \
        constexpr int tv = 1;         \
        BODY                          \
    } else {                          \
        constexpr int tv = 2;         \
        BODY                          \
    }

// Tile shapes of a kernel key (band length | variant << 8): the update
// pass's (and the operators'), then the trial pass's.  Variant 2 pairs the
// trial kernel's own wider shape with variant 0's update shape; it exists
// only where that shape is wider.
template <int L>
constexpr bool wide_trial() {
    return Tile<MISR_SCALE, L, 2>::TW > Tile<MISR_SCALE, L, 0>::TW;
}

int MISR_FN(tile_dims_s)(int key, int *th, int *tw) {
    const int v = key >> 8, Lp = key & 255;
#define X(l)                                                        \
    if (Lp == l) {                                                  \
        if (v == 1) {                                               \
            *th = Tile<MISR_SCALE, l, 1>::TH;                       \
            *tw = Tile<MISR_SCALE, l, 1>::TW;                       \
            return 1;                                               \
        }                                                           \
        if (v == 0 || (v == 2 && wide_trial<l>())) {                \
            *th = Tile<MISR_SCALE, l, 0>::TH;                       \
            *tw = Tile<MISR_SCALE, l, 0>::TW;                       \
            return 1;                                               \
        }                                                           \
        return 0;                                                   \
    }
    MISR_LIST(X)
#undef X
    return 0;
}

int MISR_FN(tile_dims_trial_s)(int key, int *th, int *tw) {
    if (!MISR_FN(tile_dims_s)(key, th, tw)) return 0;
    const int Lp = key & 255;
#define X(l)                                         \
    if (Lp == l && (key >> 8) == 2) {                \
        *th = Tile<MISR_SCALE, l, 2>::TH;            \
        *tw = Tile<MISR_SCALE, l, 2>::TW;            \
    }
    MISR_LIST(X)
#undef X
    return 1;
}

// code = st_code(x storage, y storage): the frames share the iterate's
// storage, or the iterate is FP32 over 16-bit frames.
#define MISR_CODES(LAUNCH, l)                         \
    if (code == st_code(ST_F32, ST_F32))              \
        LAUNCH(l, StF32, StF32);                      \
    else if (code == st_code(ST_F16, ST_F16))         \
        LAUNCH(l, StF16, StF16);                      \
    else if (code == st_code(ST_BF16, ST_BF16))       \
        LAUNCH(l, StBF16, StBF16);                    \
    else if (code == st_code(ST_F32, ST_F16))         \
        LAUNCH(l, StF32, StF16);                      \
    else if (code == st_code(ST_F32, ST_BF16))        \
        LAUNCH(l, StF32, StBF16);                     \
    else if (code == st_code(ST_F32, ST_U16))         \
        LAUNCH(l, StF32, StU16);                      \
    else                                              \
        return hipErrorInvalidValue;

hipError_t MISR_FN(launch_trial_s)(int key, int code, int grid, hipStream_t s, const Proj *projs,
                                   const Item *items, const int *n_items, double *partials,
                                   int mode) {
    if ((key >> 8) > 2) return hipErrorInvalidValue;
    const int Lp = key & 255;
#define LAUNCH(l, SX, SY)                                                                    \
    hipLaunchKernelGGL((k_trial<MISR_SCALE, l, tv, SX, SY>), dim3(grid), dim3(kNTI), 0, s, \
                       projs, items, n_items, partials, mode)
#define X(l)                                        \
    if (Lp == l) {                                  \
        MISR_VARIANT_TRIAL(key, MISR_CODES(LAUNCH, l))    \
        return hipGetLastError();                   \
    }
    MISR_LIST(X)
#undef X
#undef LAUNCH
    return hipErrorInvalidValue;
}

hipError_t MISR_FN(launch_upcurv_s)(int key, int code, int grid, hipStream_t s, const Proj *projs,
                                    const Item *items, const int *n_items,
                                    double *partials) {
    if ((key >> 8) > 2) return hipErrorInvalidValue;
    const int Lp = key & 255;
#define LAUNCH(l, SX, SY)                                                                     \
    hipLaunchKernelGGL((k_upcurv<MISR_SCALE, l, tv, SX, SY>), dim3(grid), dim3(kNTI), 0, s, \
                       projs, items, n_items, partials)
#define X(l)                                        \
    if (Lp == l) {                                  \
        MISR_VARIANT(key, MISR_CODES(LAUNCH, l))    \
        return hipGetLastError();                   \
    }
    MISR_LIST(X)
#undef X
#undef LAUNCH
    return hipErrorInvalidValue;
}

#define MISR_STYPES(LAUNCH, l)          \
    if (stype == ST_F32)                \
        LAUNCH(l, StF32);               \
    else if (stype == ST_F16)           \
        LAUNCH(l, StF16);               \
    else                                \
        LAUNCH(l, StBF16);

hipError_t MISR_FN(launch_forward_s)(int key, int stype, int grid, hipStream_t s, const Proj *projs,
                                     const Item *items, int n, void *y) {
    if ((key >> 8) > 2) return hipErrorInvalidValue;
    const int Lp = key & 255;
#define LAUNCH(l, ST)                                                                            \
    hipLaunchKernelGGL((k_forward<MISR_SCALE, l, tv, ST>), dim3(grid), dim3(kNTI), 0, s, projs, \
                       items, n, y)
#define X(l)                                         \
    if (Lp == l) {                                   \
        MISR_VARIANT(key, MISR_STYPES(LAUNCH, l))    \
        return hipGetLastError();                    \
    }
    MISR_LIST(X)
#undef X
#undef LAUNCH
    return hipErrorInvalidValue;
}

hipError_t MISR_FN(launch_adjoint_s)(int key, int stype, int grid, hipStream_t s, const Proj *projs,
                                     const Item *items, int n, const void *r, float *x) {
    if ((key >> 8) > 2) return hipErrorInvalidValue;
    const int Lp = key & 255;
#define LAUNCH(l, ST)                                                                            \
    hipLaunchKernelGGL((k_adjoint<MISR_SCALE, l, tv, ST>), dim3(grid), dim3(kNTI), 0, s, projs, \
                       items, n, r, x)
#define X(l)                                         \
    if (Lp == l) {                                   \
        MISR_VARIANT(key, MISR_STYPES(LAUNCH, l))    \
        return hipGetLastError();                    \
    }
    MISR_LIST(X)
#undef X
#undef LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace misr
