// internal.h -- device-side data structures shared by the kernels and the
// host runtime of libmisr.so (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace misr {

constexpr int kNT = 256;     // threads per workgroup of the image kernels
constexpr int kNV = 6;       // FP64 partial sums per work item
constexpr int kMaxK = 16;    // frames per projection
constexpr int kMaxL = 16;    // band length
constexpr int kPadRows = 16; // zero weight rows before each frame's table

enum StorageType : int { ST_F32 = 0, ST_F16 = 1, ST_BF16 = 2, ST_U16 = 3 };
// Launch code of the image kernels: storage of the views' iterate x (low
// nibble) and of the frames y (high nibble).
constexpr int st_code(int sx, int sy) { return sx | (sy << 4); }
constexpr int st_x(int code) { return code & 15; }
constexpr int st_y(int code) { return code >> 4; }

// Operator of one geometry: per frame the two 1-D factors of A_k.
// Row factor: LR row i reads HR rows s*i + offy[k] + l, l in [0, L), with
// weight wy[(k*fsy + i)*L + l]; columns likewise with wx / offx / fsx.
// wy/wx point at row 0 of frame 0; kPadRows zero rows sit before every
// frame's rows and fsy - h - kPadRows (fsx - w - kPadRows) after them, so
// that kernels may index outside [0, h): the adjoint passes compute whole
// tiles, and a last tile past the image edge reads rows up to about a tile
// extent / s beyond it (band_pad_after).
//
// General operators (affine warps or non-separable PSFs, where A_k does not
// factor; wy/wx are then NULL) are evaluated from their factors (mf = 1):
// per frame the warp (row gm[k][0] u + gm[k][1] v + gm[k][2], column
// gm[k][3] u + gm[k][4] v + gm[k][5] for HR pixel (u, v)), its inverse gi[k]
// (u = gi[k][0] r + gi[k][1] c + gi[k][2], v likewise), the half extents
// eu/ev of the preimage of a pixel's bilinear support (|u - u(r, c)| < eu),
// the candidates per axis ncu/ncv (floor(2 eu) + 1), the caps ru/rv on the
// back-projection window of an adjoint tile, and gker: the blur-and-bin
// kernel C_k[a][b] (Q x Q, Q = s + P - 1) that takes the warped image at
// (s i + a - R, s j + b - R) to LR pixel (i, j).  Warps whose windows exceed
// the kernels' LDS (mf = 0) instead carry A = [A_0; ...; A_{K-1}] as an ELL
// matrix over the K h w LR rows, a_w entries per row, entry q of row r at
// [q * rows + r] (padding: weight 0 on one of the row's own columns), and
// its transpose the same way over the H W HR rows.
struct OpDev {
    const float *wy;
    const float *wx;
    int offy[kMaxK];
    int offx[kMaxK];
    int H, W, s, K, L;
    int fsy, fsx;        // frame stride of wy / wx in rows (padding included)
    int a_w, t_w;
    const int *a_col;
    const float *a_val;
    const int *t_col;
    const float *t_val;
    int mf, P, Q, pad_;
    int ncu[kMaxK], ncv[kMaxK], ru[kMaxK], rv[kMaxK];
    double gm[kMaxK][6], gi[kMaxK][6];
    double eu[kMaxK], ev[kMaxK];
    const float *gker;
};

// Matrix-free general kernels: the forward takes LR tiles of mf_ti(s) x
// kMfTJ pixels (kMfCPT columns per thread), the adjoint and update HR tiles
// of kMfTU x kMfTV pixels (four per thread).  LDS: the forward's warped
// window holds (s (mf_ti(s) - 1) + Q) x (s (kMfTJ - 1) + Q) floats (at most
// kMfZ); the
// adjoint's residual and back-projection windows together at most kMfWin,
// its copy of the kernel padded to s ceil(Q / s) rows and columns at most
// kMfQP^2.
constexpr int kMfCPT = 2;               // forward: LR columns per thread, 32 apart
constexpr int kMfTJ = 32 * kMfCPT;
__host__ __device__ constexpr int mf_ti(int) { return 8; }
constexpr int kMfLRG = 1;   // LR tiles per forward work item
constexpr int kMfTU = 16, kMfTV = 64;
constexpr int kMfQmax = 4 + 15 - 1;
constexpr int kMfQP = 20;
__host__ __device__ constexpr int mf_zwin(int s) {
    return (s * (mf_ti(s) - 1) + s + 14) * (s * (kMfTJ - 1) + s + 14);
}
__host__ __device__ constexpr int mf_cmax(int a, int b) { return a > b ? a : b; }
constexpr int kMfZ = mf_cmax(mf_cmax(mf_zwin(1), mf_zwin(2)), mf_cmax(mf_zwin(3), mf_zwin(4)));
constexpr int kMfWin = 7424;

// Rows (LR or HR pixels) per work item of the general-operator kernels; an
// item's tx is its role: 0 LR rows (forward, residual), 1 HR rows (adjoint,
// prior, update).
constexpr int kGenRows = 256;
// LR vectors of a general solve: the residual term, A x and A p (two each).
constexpr int kGenVecs = 5;

// One image (or one tile of an image held separately in HBM) in a work list.
// Buffers are H-major with row stride ld; buffer pixel (u, v) is global
// pixel (gy0 + u, gx0 + v).  The owned rectangle [oy0,oy1) x [ox0,ox1)
// (buffer coordinates, multiples of s in global coordinates) is where this
// view computes the gradient and what it counts in its reductions; the update
// rectangle [uy0,uy1) x [ux0,ux1) (owned plus halo) is where it applies the
// pointwise x, p update, so that halo copies stay identical to their owners.
struct Proj {
    void *x[2];          // storage type
    float *p[2];
    float *g[2];
    const void *y;       // global frames K x h x w, storage type
    int ld, Hb, Wb;
    int gy0, gx0;
    int oy0, oy1, ox0, ox1;
    int uy0, uy1, ux0, ux1;
    int ntx;             // tiles per row of the owned rectangle
    struct ScgState *st; // the solve this view belongs to
    const OpDev *op;
    float *res;          // general operators: the residual term per LR row (K h w)
    // matrix-free general operators: A x[i] and A p[i] per LR row (K h w
    // each), kept with the iterate so that the trial's forward at x + alpha p
    // is A x + alpha A p
    float *ax[2], *ap[2];
};

// Halo exchange: rows x cols pixels at global (gy, gx) of view src's owned
// gradient copied into view dst's halo.
struct HaloCopy {
    int src, dst;
    int gy, gx, rows, cols;
};

// Work-list order of a view's tiles: row-major, or for a view more than
// kStripMin tiles wide, strips of kStripTiles tile columns, each listed
// row by row (down the strip, then the next strip).
constexpr int kStripTiles = 8, kStripMin = 32;
__host__ __device__ inline void strip_tile(int i, int nty, int ntx, int &ty, int &tx) {
    if (ntx <= kStripMin) {
        ty = i / ntx;
        tx = i - ty * ntx;
        return;
    }
    const int s = i / (kStripTiles * nty), loc = i - s * kStripTiles * nty;
    const int ws = ntx - kStripTiles * s < kStripTiles ? ntx - kStripTiles * s : kStripTiles;
    ty = loc / ws;
    tx = kStripTiles * s + loc - ty * ws;
}

struct Item {
    int proj;            // index into Proj array
    int ty, tx;          // tile coordinates in the owned rectangle
    int pad_;
};

// Objective weights for the kernels (float) plus solver constants.
struct Weights {
    float gam[9];        // lambda * alpha^(dx+dy) at [dy*3+dx]; 0 outside window
    float eps;           // prior Charbonnier eps
    float eps_data;      // data Charbonnier eps (p = 1)
    int data_p;
    int x_rounding;      // 16-bit x storage: 0 nearest even, 1 stochastic (hashed)
    float y_scale;       // frame value = y_scale * stored value (1 unless uint16 counts)
    int pad_;
};

// Device-resident SCG state of one solve (Moller's scalars, FP64).
struct ScgState {
    double E, E0, lam, lam_bar, delta, mu, pi, rr;
    double alpha, beta, sigma, sigk;
    double E_t, Delta;
    long long N;         // restart period: number of unknowns
    int k, it, n_iter, n_success;
    int success;         // last pass accepted (curvature to be recomputed)
    int cur;             // g[cur] is the current gradient
    int xc;              // x[xc], p[xc] hold the current iterate
    int upd_src;         // k_upcurv reads x/p[upd_src], writes x/p[upd_src ^ 1]
    int active;          // 0 once stopped
    int stop;            // 0 running/complete, 1 ||r|| = 0, 2 non-finite
    int do_update;       // k_upcurv runs this pass
    float alpha_f, beta_f, sigk_f;
    unsigned rseed;      // per-pass seed of the stochastic rounding hash
    void *xglob;         // tiled solves: the caller's whole-image x (row stride ldg)
    float *gglob;        // tiled cost_grad: the caller's whole-image gradient
    int ldg, pad2_;
    Weights wt;
};

// A solve as seen by the scalar kernel: its state, its per-pass record and
// the range of work items (and partial sums) its views occupy.
struct SolveRef {
    ScgState *st;
    struct IterRec *trace;
    int item0, nitems;     // trial-pass items (owned tiles)
    int item0u, nitemsu;   // update-pass items (owned plus halo)
};

// Start-point kernels (interpolation, bicubic): grid and per-frame integer
// HR offsets t = round(s d).
struct InitArgs {
    int H, W, s, K;
    int ty[kMaxK], tx[kMaxK];
};

struct IterRec {
    double E, E_t, delta, mu, alpha, Delta, lam;
    double pi, rr;       // |p|^2 of the pass's direction, |r|^2 at the pass's start
    int success, pad_;
};

}  // namespace misr
