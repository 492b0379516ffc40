/*
 * misr_oracle.c -- FP64 CPU checker for the MISR cost and gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or table with the GPU
 * path.
 *
 * Every operator is the plain 2-D definition written out, in double precision,
 * on an H x W high-resolution grid with zero outside the grid:
 *   - observation model y_k = D B M_k x                   (Sec. 3.1, Eq. sisr)
 *   - data term sum_k ||A_k x - y_k||_p^p, p in {1, 2}    (Eq. l2misr, Eq. misr)
 *   - BTV prior sum_d alpha^(dx+dy) ||x - S_d x||_1       (Eq. prior)
 *   - objective J = data + lambda * prior                 (Eq. objective)
 * The L1 norms are smoothed with the Charbonnier function
 *   phi(z) = sqrt(z^2 + eps^2) - eps   (eps = 0 gives |z|, derivative sign(z)
 *   with sign(0) = 0),
 * which the paper leaves open (it does not say how the L1 terms are
 * differentiated for SCG).
 *
 * Deliberately NOT factorised: the warp is 2-D bilinear, the blur a P x P
 * 2-D convolution and the decimation an s x s block mean, so that the GPU's
 * separable band factorisation is itself under test.
 *
 * Conventions (readings of points the paper leaves open):
 *   M_k : (M_k x)(u,v) = bilinear sample of x at (u + ty, v + tx), where
 *         (tx, ty) = s * (dx_k, dy_k) are HR-pixel shifts; zero off-grid.
 *         Defined on the H x W grid only (an n x n matrix).
 *   B   : (B z)(u,v) = sum_{a,b in [-R,R]} h(a,b) z(u-a, v-b), zero padding,
 *         h(a,b) = psf[a+R] * psf[b+R]   (P = 2R+1 taps).
 *   D   : (D w)(i,j) = s^-2 sum_{a,b<s} w(s i + a, s j + b)   (s x s binning).
 *   A_k = D B M_k, applied M first.
 *   General warps (the "_w" functions): M_k may instead be affine,
 *         (M_k x)(u,v) = bilinear sample of x at row m0 u + m1 v + m2,
 *         column m3 u + m4 v + m5 (m = frame k's six coefficients, HR
 *         pixels, zero off-grid); the translation above is
 *         m = (1, 0, ty, 0, 1, tx).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef long long i64;

static inline double at(const double *z, int H, int W, i64 u, i64 v) {
    return (u < 0 || v < 0 || u >= H || v >= W) ? 0.0 : z[u * (i64)W + v];
}

/* ---------------------------------------------------------------- warp M */
void orc_warp(int H, int W, double tx, double ty, const double *x, double *out) {
    const double fy0 = floor(ty), fx0 = floor(tx);
    const double fa = ty - fy0, fb = tx - fx0;
    const i64 oy = (i64)fy0, ox = (i64)fx0;
#pragma omp parallel for schedule(static)
    for (i64 u = 0; u < H; ++u)
        for (i64 v = 0; v < W; ++v) {
            const i64 a0 = u + oy, b0 = v + ox;
            out[u * W + v] = (1 - fa) * (1 - fb) * at(x, H, W, a0, b0)
                           + (1 - fa) * fb * at(x, H, W, a0, b0 + 1)
                           + fa * (1 - fb) * at(x, H, W, a0 + 1, b0)
                           + fa * fb * at(x, H, W, a0 + 1, b0 + 1);
        }
}

/* transpose of orc_warp: out(r,c) collects every sample that read x(r,c) */
void orc_warp_T(int H, int W, double tx, double ty, const double *z, double *out) {
    const double fy0 = floor(ty), fx0 = floor(tx);
    const double fa = ty - fy0, fb = tx - fx0;
    const i64 oy = (i64)fy0, ox = (i64)fx0;
#pragma omp parallel for schedule(static)
    for (i64 r = 0; r < H; ++r)
        for (i64 c = 0; c < W; ++c) {
            const i64 u = r - oy, v = c - ox;
            out[r * W + c] = (1 - fa) * (1 - fb) * at(z, H, W, u, v)
                           + (1 - fa) * fb * at(z, H, W, u, v - 1)
                           + fa * (1 - fb) * at(z, H, W, u - 1, v)
                           + fa * fb * at(z, H, W, u - 1, v - 1);
        }
}

/* affine M_k (general warps): the sample of out(u,v) sits at row
 * m[0] u + m[1] v + m[2], column m[3] u + m[4] v + m[5] */
void orc_warp_affine(int H, int W, const double *m, const double *x, double *out) {
#pragma omp parallel for schedule(static)
    for (i64 u = 0; u < H; ++u)
        for (i64 v = 0; v < W; ++v) {
            const double r = m[0] * u + m[1] * v + m[2], c = m[3] * u + m[4] * v + m[5];
            const double r0 = floor(r), c0 = floor(c);
            const double fa = r - r0, fb = c - c0;
            const i64 a0 = (i64)r0, b0 = (i64)c0;
            out[u * W + v] = (1 - fa) * (1 - fb) * at(x, H, W, a0, b0)
                           + (1 - fa) * fb * at(x, H, W, a0, b0 + 1)
                           + fa * (1 - fb) * at(x, H, W, a0 + 1, b0)
                           + fa * fb * at(x, H, W, a0 + 1, b0 + 1);
        }
}

/* transpose of orc_warp_affine: every sample adds its value, times its four
 * bilinear weights, to the pixels it read (serial scatter) */
void orc_warp_affine_T(int H, int W, const double *m, const double *z, double *out) {
    memset(out, 0, sizeof(double) * (i64)H * W);
    for (i64 u = 0; u < H; ++u)
        for (i64 v = 0; v < W; ++v) {
            const double r = m[0] * u + m[1] * v + m[2], c = m[3] * u + m[4] * v + m[5];
            const double r0 = floor(r), c0 = floor(c);
            const double fa = r - r0, fb = c - c0;
            const i64 a0 = (i64)r0, b0 = (i64)c0;
            const double zv = z[u * W + v];
            const double wgt[4] = {(1 - fa) * (1 - fb), (1 - fa) * fb, fa * (1 - fb), fa * fb};
            const i64 ra[4] = {a0, a0, a0 + 1, a0 + 1}, cb[4] = {b0, b0 + 1, b0, b0 + 1};
            for (int q = 0; q < 4; ++q)
                if (ra[q] >= 0 && ra[q] < H && cb[q] >= 0 && cb[q] < W)
                    out[ra[q] * W + cb[q]] += wgt[q] * zv;
        }
}

/* ---------------------------------------------------------------- blur B */
/* h: the P x P PSF (row-major, h[(a+R) P + (b+R)] weights the sample at
 * offset (-a, -b)); "same" convolution with zero padding. */
void orc_blur(int H, int W, int P, const double *h, const double *z, double *out) {
    const int R = (P - 1) / 2;
#pragma omp parallel for schedule(static)
    for (i64 u = 0; u < H; ++u)
        for (i64 v = 0; v < W; ++v) {
            double acc = 0.0;
            for (int a = -R; a <= R; ++a)
                for (int b = -R; b <= R; ++b)
                    acc += h[(a + R) * P + (b + R)] * at(z, H, W, u - a, v - b);
            out[u * W + v] = acc;
        }
}

void orc_blur_T(int H, int W, int P, const double *h, const double *w, double *out) {
    const int R = (P - 1) / 2;
#pragma omp parallel for schedule(static)
    for (i64 u = 0; u < H; ++u)
        for (i64 v = 0; v < W; ++v) {
            double acc = 0.0;
            for (int a = -R; a <= R; ++a)
                for (int b = -R; b <= R; ++b)
                    acc += h[(a + R) * P + (b + R)] * at(w, H, W, u + a, v + b);
            out[u * W + v] = acc;
        }
}

/* ---------------------------------------------------------------- bin D */
void orc_bin(int H, int W, int s, const double *z, double *out) {
    const int h = H / s, w = W / s;
    const double inv = 1.0 / ((double)s * s);
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < h; ++i)
        for (i64 j = 0; j < w; ++j) {
            double acc = 0.0;
            for (int a = 0; a < s; ++a)
                for (int b = 0; b < s; ++b) acc += z[(s * i + a) * (i64)W + s * j + b];
            out[i * w + j] = acc * inv;
        }
}

void orc_bin_T(int H, int W, int s, const double *r, double *out) {
    const int w = W / s;
    const double inv = 1.0 / ((double)s * s);
#pragma omp parallel for schedule(static)
    for (i64 u = 0; u < H; ++u)
        for (i64 v = 0; v < W; ++v) out[u * W + v] = r[(u / s) * w + v / s] * inv;
}

/* ------------------------------------------------------ A_k and sum A_k^T */
/* y has K frames of (H/s) x (W/s); shifts is K x 2 as (dx, dy) in LR px;
 * psf holds each frame's P x P PSF (K of them: B_k may differ per frame). */
/* warps: NULL (translations from shifts) or [K][6] affine coefficients */
void orc_forward_w(int H, int W, int s, int K, const double *shifts, const double *warps,
                   int P, const double *psf, const double *x, double *y) {
    const i64 n = (i64)H * W, m = (i64)(H / s) * (W / s);
    double *t1 = (double *)malloc(sizeof(double) * n);
    double *t2 = (double *)malloc(sizeof(double) * n);
    for (int k = 0; k < K; ++k) {
        if (warps)
            orc_warp_affine(H, W, warps + 6 * k, x, t1);
        else
            orc_warp(H, W, s * shifts[2 * k], s * shifts[2 * k + 1], x, t1);
        orc_blur(H, W, P, psf + (i64)k * P * P, t1, t2);
        orc_bin(H, W, s, t2, y + k * m);
    }
    free(t1);
    free(t2);
}

void orc_forward(int H, int W, int s, int K, const double *shifts, int P,
                 const double *psf, const double *x, double *y) {
    orc_forward_w(H, W, s, K, shifts, NULL, P, psf, x, y);
}

void orc_adjoint_w(int H, int W, int s, int K, const double *shifts, const double *warps,
                   int P, const double *psf, const double *r, double *x) {
    const i64 n = (i64)H * W, m = (i64)(H / s) * (W / s);
    double *t1 = (double *)malloc(sizeof(double) * n);
    double *t2 = (double *)malloc(sizeof(double) * n);
    memset(x, 0, sizeof(double) * n);
    for (int k = 0; k < K; ++k) {
        orc_bin_T(H, W, s, r + k * m, t1);
        orc_blur_T(H, W, P, psf + (i64)k * P * P, t1, t2);
        if (warps)
            orc_warp_affine_T(H, W, warps + 6 * k, t2, t1);
        else
            orc_warp_T(H, W, s * shifts[2 * k], s * shifts[2 * k + 1], t2, t1);
#pragma omp parallel for schedule(static)
        for (i64 i = 0; i < n; ++i) x[i] += t1[i];
    }
    free(t1);
    free(t2);
}

void orc_adjoint(int H, int W, int s, int K, const double *shifts, int P,
                 const double *psf, const double *r, double *x) {
    orc_adjoint_w(H, W, s, K, shifts, NULL, P, psf, r, x);
}

/* ------------------------------------------------ Charbonnier phi and psi */
static inline double phi_eps(double z, double eps) {
    if (eps == 0.0) return fabs(z);
    return z * z / (sqrt(z * z + eps * eps) + eps);
}
static inline double psi_eps(double z, double eps) {
    if (eps == 0.0) return (z > 0) - (z < 0);
    return z / sqrt(z * z + eps * eps);
}

/* ------------------------------------------------------------ BTV prior */
/* E_reg = lambda * sum_{d in [0,w-1]^2 \ {0}} alpha^(dx+dy)
 *                 * sum_{(u,v), (u+dy, v+dx) both in grid} phi(x(u,v) - x(u+dy, v+dx)).
 * g (if not NULL) receives += dE_reg/dx, written in gather form so that rows
 * can be processed in parallel. */
double orc_btv(int H, int W, double lambda, double alpha, double eps, int w,
               const double *x, double *g) {
    double E = 0.0;
    double *gtab = (double *)malloc(sizeof(double) * w * w);
    for (int dy = 0; dy < w; ++dy)
        for (int dx = 0; dx < w; ++dx) gtab[dy * w + dx] = lambda * pow(alpha, dx + dy);
#pragma omp parallel for schedule(static) reduction(+ : E)
    for (i64 u = 0; u < H; ++u)
        for (i64 v = 0; v < W; ++v) {
            const double xi = x[u * W + v];
            double gi = 0.0;
            for (int dy = 0; dy < w; ++dy)
                for (int dx = 0; dx < w; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    const double gam = gtab[dy * w + dx];
                    if (u + dy < H && v + dx < W) {        /* pair (i, i+d) */
                        const double z = xi - x[(u + dy) * W + v + dx];
                        E += gam * phi_eps(z, eps);
                        gi += gam * psi_eps(z, eps);
                    }
                    if (u - dy >= 0 && v - dx >= 0) {      /* pair (i-d, i) */
                        const double z = x[(u - dy) * W + v - dx] - xi;
                        gi -= gam * psi_eps(z, eps);
                    }
                }
            if (g) g[u * W + v] += gi;
        }
    free(gtab);
    return E;
}

/* The part of the BTV prior one subdomain owns (Sec. 3.1, Eq. subfunction):
 * the pairs (i, i+d) whose first pixel i lies in the rectangle
 * [u0,u1) x [v0,v1), both pixels inside the H x W grid.  g (nullable)
 * receives += the gradient of that part, which reaches up to w-1 pixels
 * below and to the right of the rectangle.  Summed over rectangles that
 * tile the grid, the parts give orc_btv exactly (up to summation order). */
double orc_btv_owned(int H, int W, double lambda, double alpha, double eps, int w,
                     const double *x, int u0, int u1, int v0, int v1, double *g) {
    double E = 0.0;
    double *gtab = (double *)malloc(sizeof(double) * w * w);
    for (int dy = 0; dy < w; ++dy)
        for (int dx = 0; dx < w; ++dx) gtab[dy * w + dx] = lambda * pow(alpha, dx + dy);
    const i64 ue = (u1 + w - 1 < H) ? u1 + w - 1 : H, ve = (v1 + w - 1 < W) ? v1 + w - 1 : W;
#pragma omp parallel for schedule(static) reduction(+ : E)
    for (i64 u = u0; u < ue; ++u)
        for (i64 v = v0; v < ve; ++v) {
            const double xi = x[u * W + v];
            const int own_i = u < u1 && v < v1;
            double gi = 0.0;
            for (int dy = 0; dy < w; ++dy)
                for (int dx = 0; dx < w; ++dx) {
                    if (dx == 0 && dy == 0) continue;
                    const double gam = gtab[dy * w + dx];
                    if (own_i && u + dy < H && v + dx < W) {   /* owned pair (i, i+d) */
                        const double z = xi - x[(u + dy) * W + v + dx];
                        E += gam * phi_eps(z, eps);
                        gi += gam * psi_eps(z, eps);
                    }
                    /* pair (i-d, i), owned when i-d is */
                    if (u - dy >= u0 && v - dx >= v0 && u - dy < u1 && v - dx < v1) {
                        const double z = x[(u - dy) * W + v - dx] - xi;
                        gi -= gam * psi_eps(z, eps);
                    }
                }
            if (g) g[u * W + v] += gi;
        }
    free(gtab);
    return E;
}

/* ------------------------------------------------------- cost + gradient */
/* J(x) = sum_k sum phi_p(A_k x - y_k) + E_reg(x), with phi_2(r) = r^2 and
 * phi_1 = Charbonnier with eps_data.  g (nullable) receives grad J.
 * parts (nullable) receives {E_data, E_reg}.  Returns J. */
double orc_cost_grad_w(int H, int W, int s, int K, const double *shifts,
                       const double *warps, int P, const double *psf, double lambda,
                       double alpha, double eps, int w, int data_p, double eps_data,
                       const double *x, const double *y, double *g, double *parts) {
    const i64 n = (i64)H * W, m = (i64)(H / s) * (W / s) * K;
    double *r = (double *)malloc(sizeof(double) * m);
    orc_forward_w(H, W, s, K, shifts, warps, P, psf, x, r);
    double Ed = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : Ed)
    for (i64 i = 0; i < m; ++i) {
        const double e = r[i] - y[i];
        if (data_p == 2) {
            Ed += e * e;
            r[i] = 2.0 * e;
        } else {
            Ed += phi_eps(e, eps_data);
            r[i] = psi_eps(e, eps_data);
        }
    }
    if (g) orc_adjoint_w(H, W, s, K, shifts, warps, P, psf, r, g);
    free(r);
    const double Er = orc_btv(H, W, lambda, alpha, eps, w, x, g);
    if (parts) {
        parts[0] = Ed;
        parts[1] = Er;
    }
    (void)n;
    return Ed + Er;
}

double orc_cost_grad(int H, int W, int s, int K, const double *shifts, int P,
                     const double *psf, double lambda, double alpha, double eps, int w,
                     int data_p, double eps_data, const double *x, const double *y,
                     double *g, double *parts) {
    return orc_cost_grad_w(H, W, s, K, shifts, NULL, P, psf, lambda, alpha, eps, w, data_p,
                           eps_data, x, y, g, parts);
}

/* --------------------------------------- curvature in closed form (check) */
/* Finite-difference quotient of psi between b and a = b + h, written without
 * cancellation:  (psi(a) - psi(b)) / h = (eps^2 + C) / (A B (A + B)),
 * A = sqrt(a^2+eps^2), B = sqrt(b^2+eps^2), C = A B - a b, where C is
 * evaluated as (eps^2 (a^2+b^2) + eps^4) / (A B + a b) when a b > 0. */
double orc_psi_quotient(double b, double h, double eps) {
    const double a = b + h;
    if (eps == 0.0) {
        if (h == 0.0) return 0.0;
        return (psi_eps(a, 0.0) - psi_eps(b, 0.0)) / h;
    }
    const double e2 = eps * eps;
    const double A = sqrt(a * a + e2), B = sqrt(b * b + e2);
    const double C = (a * b > 0) ? (e2 * (a * a + b * b) + e2 * e2) / (A * B + a * b)
                                 : A * B - a * b;
    return (e2 + C) / (A * B * (A + B));
}

/* delta = p^T (grad J(x + sk p) - grad J(x)) / sk, for p = 2, evaluated as
 *   2 sum_k ||A_k p||^2  +  lambda sum_d gamma_d sum_pairs q^2 Q(z, sk q),
 * z = x_i - x_{i+d}, q = p_i - p_{i+d}.  Equal in exact arithmetic to the
 * literal quotient.  parts (nullable) receives {data part, BTV part}. */
double orc_curv_exact(int H, int W, int s, int K, const double *shifts, int P,
                      const double *psf, double lambda, double alpha, double eps, int w,
                      double sk, const double *x, const double *p, double *parts) {
    const i64 m = (i64)(H / s) * (W / s) * K;
    double *ap = (double *)malloc(sizeof(double) * m);
    orc_forward(H, W, s, K, shifts, P, psf, p, ap);
    double dd = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : dd)
    for (i64 i = 0; i < m; ++i) dd += ap[i] * ap[i];
    free(ap);
    dd *= 2.0;
    double dr = 0.0;
    double *gtab = (double *)malloc(sizeof(double) * w * w);
    for (int dy = 0; dy < w; ++dy)
        for (int dx = 0; dx < w; ++dx) gtab[dy * w + dx] = lambda * pow(alpha, dx + dy);
#pragma omp parallel for schedule(static) reduction(+ : dr)
    for (i64 u = 0; u < H; ++u)
        for (i64 v = 0; v < W; ++v)
            for (int dy = 0; dy < w; ++dy)
                for (int dx = 0; dx < w; ++dx) {
                    if ((dx == 0 && dy == 0) || u + dy >= H || v + dx >= W) continue;
                    const double z = x[u * W + v] - x[(u + dy) * W + v + dx];
                    const double q = p[u * W + v] - p[(u + dy) * W + v + dx];
                    dr += gtab[dy * w + dx] * q * q * orc_psi_quotient(z, sk * q, eps);
                }
    free(gtab);
    if (parts) {
        parts[0] = dd;
        parts[1] = dr;
    }
    return dd + dr;
}

/* Data part of delta for the Charbonnier L1 data term (Eq. misr, p = 1):
 *   sum_k sum_i (A_k p)_i^2 Q(r_i, sk (A_k p)_i),  r = A_k x - y_k,
 * Q the psi quotient above with eps_data.  Equal in exact arithmetic to
 * p^T (grad E_data(x + sk p) - grad E_data(x)) / sk. */
double orc_curv_data_l1(int H, int W, int s, int K, const double *shifts, int P,
                        const double *psf, double eps_data, double sk, const double *x,
                        const double *p, const double *y) {
    const i64 m = (i64)(H / s) * (W / s) * K;
    double *ap = (double *)malloc(sizeof(double) * m);
    double *ax = (double *)malloc(sizeof(double) * m);
    orc_forward(H, W, s, K, shifts, P, psf, p, ap);
    orc_forward(H, W, s, K, shifts, P, psf, x, ax);
    double dd = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : dd)
    for (i64 i = 0; i < m; ++i)
        dd += ap[i] * ap[i] * orc_psi_quotient(ax[i] - y[i], sk * ap[i], eps_data);
    free(ap);
    free(ax);
    return dd;
}

/* Multi-image interpolation, the paper's non-iterative fusion baseline
 * (Sec. 4: LR pixel values inserted at their integer HR positions).  Frame
 * k's pixel (i, j) lands on HR (s i + ty_k, s j + tx_k), t_k = round(s d_k)
 * (halves away from zero); an HR pixel takes the mean of the samples landing
 * on it, in frame order; one that receives none takes frame 0's pixel
 * (floor(u / s), floor(v / s)). */
void orc_interpolate(int H, int W, int s, int K, const double *shifts, const double *y,
                     double *x) {
    const int h = H / s, w = W / s;
    int *ty = (int *)malloc(sizeof(int) * K), *tx = (int *)malloc(sizeof(int) * K);
    for (int k = 0; k < K; ++k) {
        tx[k] = (int)lround(s * shifts[2 * k + 0]);
        ty[k] = (int)lround(s * shifts[2 * k + 1]);
    }
#pragma omp parallel for schedule(static)
    for (int u = 0; u < H; ++u)
        for (int v = 0; v < W; ++v) {
            double acc = 0.0;
            int n = 0;
            for (int k = 0; k < K; ++k) {
                const int a = u - ty[k], b = v - tx[k];
                if (a < 0 || b < 0 || a % s != 0 || b % s != 0) continue;
                const int i = a / s, j = b / s;
                if (i >= h || j >= w) continue;
                acc += y[((i64)k * h + i) * w + j];
                ++n;
            }
            x[(i64)u * W + v] = n ? acc / n : y[(i64)(u / s) * w + v / s];
        }
    free(ty);
    free(tx);
}

/* Keys cubic convolution kernel with a = -1/2. */
static double keys(double t) {
    t = fabs(t);
    if (t <= 1.0) return (1.5 * t - 2.5) * t * t + 1.0;
    if (t < 2.0) return ((-0.5 * t + 2.5) * t - 4.0) * t + 2.0;
    return 0.0;
}

/* Bicubic upsampling of one LR frame by s (the solver's start point): HR
 * sample u sits at LR coordinate (u + 1/2) / s - 1/2; the 4 x 4 taps around
 * it take Keys weights, indices clamped to the frame.  Evaluated as the full
 * 2-D sum (no separable passes). */
void orc_upsample(int H, int W, int s, const double *lr, double *x) {
    const int h = H / s, w = W / s;
#pragma omp parallel for schedule(static)
    for (int u = 0; u < H; ++u)
        for (int v = 0; v < W; ++v) {
            const double cy = (u + 0.5) / s - 0.5, cx = (v + 0.5) / s - 0.5;
            const int iy = (int)floor(cy), ix = (int)floor(cx);
            double acc = 0.0;
            for (int a = -1; a <= 2; ++a)
                for (int b = -1; b <= 2; ++b) {
                    int i = iy + a, j = ix + b;
                    i = i < 0 ? 0 : (i >= h ? h - 1 : i);
                    j = j < 0 ? 0 : (j >= w ? w - 1 : j);
                    acc += keys(cy - (iy + a)) * keys(cx - (ix + b)) * lr[(i64)i * w + j];
                }
            x[(i64)u * W + v] = acc;
        }
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
