// TV-regularised linearised inversion on one level (Sec. II-C, eq. tv_iteration):
//   z_{l+1} = (L^T L + alpha D^T Gamma_l D)^{-1} L^T r,   Gamma_0 = I,
//   Gamma_l = diag(1 / max(|D z_l|, tau)),  tau = 1e-8 max|D z_l|  (Gamma = I if D z_l = 0).
// The coarse-to-fine variant over two nested levels (Sec. II-D/E) runs the same solver on
// L R_c and L R_f, matrices formed on the device by sparse column combination.
// When the normal matrix G = L^T L (M x M, FP64) is smaller than two passes over L, its
// upper 64 x 64 blocks are formed once per call on the FP64 matrix cores and each system
// G + alpha D^T Gamma D is solved exactly: dense Cholesky U^T U in place on those blocks,
// then two block triangular solves.  Otherwise (or on request, or when the factorisation
// meets a pivot that is not positive to working precision) each system is solved by
// preconditioned conjugate gradients (warm-started from z_l; Jacobi preconditioner
// diag(L^T L) + alpha diag(D^T Gamma D), or for few rows the Woodbury inverse of
// alpha diag(D^T Gamma D) + L^T L) with FP64 vectors and reductions.  CG products with L
// stream the matrix row-major: y = L x with one workgroup per row block, x = L^T y with
// thread-per-column partial sums over row chunks reduced in a fixed order
// (deterministic); with G formed they read only its upper blocks (a symmetric product).
#include <algorithm>
#include <cmath>
#include <string>
#include <utility>
#include <vector>

#include "mgrt_internal.hpp"

namespace mgrt {

namespace {

constexpr int ROWS_PER_BLOCK = 4;   // rows of L per workgroup in L x (one wave each)
constexpr int TCHUNK = 256;         // rows of L per partial sum in L^T y

template <typename T>
__global__ __launch_bounds__(256) void k_gemv_n(const T *__restrict__ L, int64_t rows, int64_t M,
                                                const double *__restrict__ x,
                                                double *__restrict__ y) {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int64_t r = (int64_t)blockIdx.x * ROWS_PER_BLOCK + wave;
    if (r >= rows) return;
    const T *row = L + r * M;
    double s = 0.0;
    for (int64_t j = lane; j < M; j += 64) s += (double)row[j] * x[j];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) y[r] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gemv_t_part(const T *__restrict__ L, int64_t rows,
                                                     int64_t M, const double *__restrict__ y,
                                                     double *__restrict__ part) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t chunk = blockIdx.y;
    if (j >= M) return;
    const int64_t r0 = chunk * TCHUNK, r1 = std::min(rows, r0 + TCHUNK);
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) s += (double)L[r * M + j] * y[r];
    part[chunk * M + j] = s;
}

template <typename T>
__global__ __launch_bounds__(256) void k_colsq_part(const T *__restrict__ L, int64_t rows,
                                                    int64_t M, double *__restrict__ part) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t chunk = blockIdx.y;
    if (j >= M) return;
    const int64_t r0 = chunk * TCHUNK, r1 = std::min(rows, r0 + TCHUNK);
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) {
        const double v = (double)L[r * M + j];
        s += v * v;
    }
    part[chunk * M + j] = s;
}

// Normal matrix G = L^T L (FP64) on the matrix cores: v_mfma_f64_16x16x4f64.  One
// workgroup forms a 64 x 64 block (bi, bj >= bi); each of its 4 waves a 32 x 32 quarter as
// 2 x 2 MFMA tiles.  L streams through LDS in panels (converted to FP64).
// MFMA operand layout (wave64): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// of the 16x4 and 4x16 operands and receives D[4 v + l / 16][l % 16] in slot v.
// Only the upper blocks are formed (the Woodbury row Gram matrix, which needs all of
// them, is completed by k_mirror_lower).
constexpr int SYRK_PAD = 4;
typedef double d4v __attribute__((ext_vector_type(4)));

// Panels of SYRK_KT2 rows; the next panel's elements are loaded into registers while the
// matrix cores work on the current one (the loads are in flight during the MFMAs).
constexpr int SYRK_KT2 = 32;

template <typename T>
__global__ __launch_bounds__(256) void k_syrk(const T *__restrict__ L, int64_t rows, int64_t M,
                                              double *__restrict__ G) {
    const int64_t bi = blockIdx.y, bj = blockIdx.x;
    if (bj < bi) return;
    __shared__ double As[SYRK_KT2][64 + SYRK_PAD];
    __shared__ double Bs[SYRK_KT2][64 + SYRK_PAD];
    constexpr int PER = SYRK_KT2 * 64 / 256;            // elements per thread per panel
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wy = wave >> 1, wx = wave & 1;
    const int64_t i0 = bi * 64, j0 = bj * 64;
    const int cc = tid & 63, kr0 = tid >> 6;            // element e = kr0 + 4 u of column cc
    const bool ci = i0 + cc < M, cj = j0 + cc < M;
    d4v acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4v{0.0, 0.0, 0.0, 0.0};
    T ra[PER], rb[PER];
    auto fetch = [&](int64_t r0) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int64_t r = r0 + kr0 + 4 * u;
            ra[u] = (r < rows && ci) ? L[r * M + i0 + cc] : T(0);
            rb[u] = (r < rows && cj) ? L[r * M + j0 + cc] : T(0);
        }
    };
    fetch(0);
    for (int64_t r0 = 0; r0 < rows; r0 += SYRK_KT2) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            As[kr0 + 4 * u][cc] = (double)ra[u];
            Bs[kr0 + 4 * u][cc] = (double)rb[u];
        }
        __syncthreads();
        if (r0 + SYRK_KT2 < rows) fetch(r0 + SYRK_KT2);
#pragma unroll
        for (int kk = 0; kk < SYRK_KT2; kk += 4) {
            const int kr = kk + (lane >> 4), c16 = lane & 15;
            const double a0 = As[kr][32 * wy + c16], a1 = As[kr][32 * wy + 16 + c16];
            const double b0 = Bs[kr][32 * wx + c16], b1 = Bs[kr][32 * wx + 16 + c16];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t i = i0 + 32 * wy + 16 * a + 4 * v + (lane >> 4);
                const int64_t j = j0 + 32 * wx + 16 * b + (lane & 15);
                if (i < M && j < M) G[i * M + j] = acc[a][b][v];
            }
}

// G[j][i] = G[i][j] for the blocks below the diagonal, through an LDS transpose
__global__ __launch_bounds__(256) void k_mirror_lower(double *__restrict__ G, int64_t M) {
    const int64_t bi = blockIdx.y, bj = blockIdx.x;   // destination block (bi > bj)
    if (bi <= bj) return;
    __shared__ double t[64][65];
    const int tid = threadIdx.x;
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e >> 6, cc = e & 63;
        const int64_t gi = bj * 64 + r, gj = bi * 64 + cc;   // source block (bj, bi), upper
        t[r][cc] = (gi < M && gj < M) ? G[gi * M + gj] : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < 64 * 64; e += 256) {
        const int r = e >> 6, cc = e & 63;
        const int64_t gi = bi * 64 + r, gj = bj * 64 + cc;
        if (gi < M && gj < M) G[gi * M + gj] = t[cc][r];
    }
}

// ---- Dense Cholesky A = U^T U of the formed normal matrix, on its upper 64 x 64 blocks ----
// (the same row-major M x M array: block (i, j), j >= i, holds U_ij).  Right-looking over
// block steps k: factor the diagonal block (one workgroup, LDS), form the row panel
// U_kj = U_kk^-T A_kj, update the trailing upper blocks A_ij -= U_ki^T U_kj (FP64 MFMA).
// Entries past M act as the identity (the ragged last block).

// Diagonal block k: A_kk = U_kk^T U_kk right-looking over its 64 rows, then X = U_kk^-1 by
// back substitution on I (row oriented); X goes to Uinv[k] and its transpose to UinvT[k].
// A pivot that is not finite or not above CHOL_PIV_TOL times the matrix's original
// diagonal entry (the system is then singular to working precision) sets *flag and the
// block continues with pivot 1 (every later kernel stays finite); the caller then
// discards the factor.
constexpr double CHOL_PIV_TOL = 1e-13;

__global__ __launch_bounds__(256) void k_chol_diag(double *__restrict__ A, int64_t M, int64_t k,
                                                   const double *__restrict__ diag0,
                                                   double *__restrict__ Uinv,
                                                   double *__restrict__ UinvT, int *__restrict__ flag) {
    // thread (q, j) = (tid / 64, tid % 64) keeps entries (i, j), i = q + 4 m, of the block
    // (r: the factor, x: the inverse) in registers; only the pivot row, and in the inverse
    // phase one row of X and one column of U, go through LDS (broadcast reads).  One
    // reciprocal square root per pivot gives U_pp and 1 / U_pp (no division on the
    // serial chain); the inverse phase reuses the reciprocals.
    __shared__ double prow[64];
    __shared__ double pcol[64];
    __shared__ double d0s[64];                 // the original diagonal of this block
    __shared__ double rinv[64];                // 1 / U_pp
    const int tid = threadIdx.x, j = tid & 63, q = tid >> 6;
    const int64_t o = k * 64;
    if (tid < 64) d0s[tid] = o + tid < M ? diag0[o + tid] : 1.0;
    double r[16], x[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int i = q + 4 * m;
        r[m] = j >= i ? (o + j < M ? A[(o + i) * M + o + j] : (i == j ? 1.0 : 0.0)) : 0.0;
        x[m] = i == j ? 1.0 : 0.0;
    }
#pragma unroll
    for (int p = 0; p < 64; ++p) {
        if (q == (p & 3)) prow[j] = r[p >> 2];
        __syncthreads();
        const double d = prow[p];
        const bool ok = isfinite(d) && d > CHOL_PIV_TOL * d0s[p] && d > 0.0;
        const double inv = ok ? rsqrt(d) : 1.0;
        const double rp = ok ? d * inv : 1.0;
        if (tid == 0) {
            rinv[p] = inv;
            if (!ok) *flag = 1;
        }
        const double uj = j == p ? rp : prow[j] * inv;         // U[p][j], j >= p
        if (q == (p & 3) && j >= p) r[p >> 2] = uj;
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int i = q + 4 * m;
            if (i > p && i <= j) r[m] -= (prow[i] * inv) * uj;
        }
        __syncthreads();
    }
    // X = U^-1: back substitution on I, rows mm = 63 .. 0
#pragma unroll
    for (int mm = 63; mm >= 0; --mm) {
        if (j == mm) {
#pragma unroll
            for (int m = 0; m < 16; ++m) pcol[q + 4 * m] = q + 4 * m <= mm ? r[m] : 0.0;
        }
        if (q == (mm & 3)) {
            x[mm >> 2] *= rinv[mm];
            prow[j] = x[mm >> 2];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 16; ++m)
            if (q + 4 * m < mm) x[m] -= pcol[q + 4 * m] * prow[j];
        __syncthreads();
    }
#pragma unroll
    for (int m = 0; m < 16; ++m) {
        const int i = q + 4 * m;
        if (j >= i && o + j < M) A[(o + i) * M + o + j] = r[m];
        Uinv[k * 4096 + i * 64 + j] = x[m];
        UinvT[k * 4096 + j * 64 + i] = x[m];
    }
}

// C = X^T Y for 64 x 64 blocks on the matrix cores (the k_syrk operand layout), X and Y
// 64 rows deep, in two panels of 32 rows (the second loaded while the first is used).
// mode 0 (row panel): X = U_kk^-1, Y = A_kj, A_kj = C for j = k + 1 + x.
// mode 1 (trailing update): X = U_ki, Y = U_kj, A_ij -= C for k < i <= j.
__global__ __launch_bounds__(256) void k_chol_xty(double *__restrict__ A, int64_t M, int64_t k,
                                                  const double *__restrict__ Uinv, int mode) {
    const int64_t j = k + 1 + blockIdx.x;
    const int64_t i = mode == 0 ? k : k + 1 + blockIdx.y;
    if (j < i) return;
    __shared__ double As[SYRK_KT2][64 + SYRK_PAD];
    __shared__ double Bs[SYRK_KT2][64 + SYRK_PAD];
    constexpr int PER = SYRK_KT2 * 64 / 256;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wy = wave >> 1, wx = wave & 1;
    const int64_t o = k * 64, i0 = i * 64, j0 = j * 64;
    const int cc = tid & 63, kr0 = tid >> 6;
    d4v acc[2][2];
#pragma unroll
    for (int ta = 0; ta < 2; ++ta)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb) acc[ta][tb] = d4v{0.0, 0.0, 0.0, 0.0};
    double ra[PER], rb[PER];
    auto fetch = [&](int r0) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int m = r0 + kr0 + 4 * u;
            const int64_t r = o + m;
            if (mode == 0) ra[u] = Uinv[k * 4096 + m * 64 + cc];
            else ra[u] = (r < M && i0 + cc < M) ? A[r * M + i0 + cc] : 0.0;
            rb[u] = (r < M && j0 + cc < M) ? A[r * M + j0 + cc] : 0.0;
        }
    };
    fetch(0);
#pragma unroll
    for (int r0 = 0; r0 < 64; r0 += SYRK_KT2) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            As[kr0 + 4 * u][cc] = ra[u];
            Bs[kr0 + 4 * u][cc] = rb[u];
        }
        __syncthreads();
        if (r0 + SYRK_KT2 < 64) fetch(r0 + SYRK_KT2);
#pragma unroll
        for (int kk = 0; kk < SYRK_KT2; kk += 4) {
            const int kr = kk + (lane >> 4), c16 = lane & 15;
            const double a0 = As[kr][32 * wy + c16], a1 = As[kr][32 * wy + 16 + c16];
            const double b0 = Bs[kr][32 * wx + c16], b1 = Bs[kr][32 * wx + 16 + c16];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0][0], 0, 0, 0);
            acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[0][1], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[1][1], 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int ta = 0; ta < 2; ++ta)
#pragma unroll
        for (int tb = 0; tb < 2; ++tb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t gi = i0 + 32 * wy + 16 * ta + 4 * v + (lane >> 4);
                const int64_t gj = j0 + 32 * wx + 16 * tb + (lane & 15);
                if (gi < M && gj < M) {
                    if (mode == 0) A[gi * M + gj] = acc[ta][tb][v];
                    else A[gi * M + gj] -= acc[ta][tb][v];
                }
            }
}

// Forward substitution step k of U^T y = b (b's later blocks are updated in place): every
// workgroup forms y_k = U_kk^-T b_k, the first stores it, and workgroup w subtracts
// U_kj^T y_k from b_j, j = k + 1 + w.  Sums in a fixed order.
__global__ __launch_bounds__(256) void k_chol_fwd(const double *__restrict__ A, int64_t M, int64_t k,
                                                  const double *__restrict__ Uinv,
                                                  double *__restrict__ b, double *__restrict__ y) {
    __shared__ double ys[64];
    __shared__ double red[4][64];
    const int tid = threadIdx.x, cidx = tid & 63, part = tid >> 6;
    const int64_t o = k * 64;
    double s = 0.0;
    for (int m = part * 16; m < part * 16 + 16; ++m)
        s += Uinv[k * 4096 + m * 64 + cidx] * (o + m < M ? b[o + m] : 0.0);
    red[part][cidx] = s;
    __syncthreads();
    if (tid < 64) ys[cidx] = ((red[0][cidx] + red[1][cidx]) + red[2][cidx]) + red[3][cidx];
    __syncthreads();
    if (blockIdx.x == 0 && tid < 64 && o + cidx < M) y[o + cidx] = ys[cidx];
    const int64_t col = (k + 1 + blockIdx.x) * 64 + cidx;
    double t = 0.0;
    if (col < M)
        for (int m = part * 16; m < part * 16 + 16; ++m)
            if (o + m < M) t += A[(o + m) * M + col] * ys[m];
    red[part][cidx] = t;
    __syncthreads();
    if (tid < 64 && col < M) b[col] -= ((red[0][cidx] + red[1][cidx]) + red[2][cidx]) + red[3][cidx];
}

// Back substitution step k of U z = y (y's earlier blocks are updated in place): every
// workgroup forms z_k = U_kk^-1 y_k, the first stores it, and workgroup w subtracts
// U_wk z_k from y_w (w < k; the block staged through LDS so that a thread owns a row).
__global__ __launch_bounds__(256) void k_chol_bwd(const double *__restrict__ A, int64_t M, int64_t k,
                                                  const double *__restrict__ UinvT,
                                                  double *__restrict__ y, double *__restrict__ z) {
    __shared__ double zs[64];
    __shared__ double red[4][64];
    __shared__ double ub[64][65];
    const int tid = threadIdx.x, cidx = tid & 63, part = tid >> 6;
    const int64_t o = k * 64;
    double s = 0.0;
    for (int m = part * 16; m < part * 16 + 16; ++m)
        s += UinvT[k * 4096 + m * 64 + cidx] * (o + m < M ? y[o + m] : 0.0);
    red[part][cidx] = s;
    __syncthreads();
    if (tid < 64) zs[cidx] = ((red[0][cidx] + red[1][cidx]) + red[2][cidx]) + red[3][cidx];
    __syncthreads();
    if (blockIdx.x == 0 && tid < 64 && o + cidx < M) z[o + cidx] = zs[cidx];
    const int64_t i = blockIdx.x;
    if (i >= k) return;
    for (int e = tid; e < 64 * 64; e += 256) {
        const int ra = e >> 6, cb = e & 63;
        ub[ra][cb] = (o + cb < M) ? A[(i * 64 + ra) * M + o + cb] : 0.0;
    }
    __syncthreads();
    double t = 0.0;
    for (int m = part * 16; m < part * 16 + 16; ++m) t += ub[cidx][m] * zs[m];
    red[part][cidx] = t;
    __syncthreads();
    if (tid < 64) y[i * 64 + cidx] -= ((red[0][cidx] + red[1][cidx]) + red[2][cidx]) + red[3][cidx];
}

// d[i] = A[i][i]
__global__ void k_get_diag(const double *__restrict__ A, int64_t M, double *__restrict__ d) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < M) d[i] = A[i * M + i];
}

// A[idx[e]] += alpha * val[e] (distinct indices)
__global__ void k_add_entries(double *__restrict__ A, const int64_t *__restrict__ idx,
                              const double *__restrict__ val, int64_t n, double alpha) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < n) A[idx[e]] += alpha * val[e];
}

// y = G x for symmetric G (M x M, FP64) reading only its upper 64 x 64 blocks: the block
// (bi, bj), bj >= bi, adds G_blk x_bj to row block bi and, off the diagonal, G_blk^T x_bi
// to row block bj.  Contributions go to part[b][k][0..63] (k = the other block index) and
// k_apply_sum adds them for each b in the fixed order k = 0 .. nb-1 (deterministic).
// Wave w loads rows 16 w .. 16 w + 15 of the block, all sixteen loads in flight (one row
// per wave instruction: 64 lanes x 8 B contiguous).  Column sums stay in the lane; the row
// sums go through LDS, where thread (w, r) adds columns 16 w .. 16 w + 15 of row r.
__global__ __launch_bounds__(256) void k_symv_blocks(const double *__restrict__ G, int64_t M,
                                                     const int2 *__restrict__ pairs,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ part) {
    __shared__ double prod[64][65];
    __shared__ double red[2][4][64];
    const int2 pr = pairs[blockIdx.x];
    const int64_t bi = pr.x, bj = pr.y, nb = (M + 63) / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t j = bj * 64 + lane, i0 = bi * 64 + wave * 16;
    const bool jin = j < M;
    double g[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) g[k] = (i0 + k < M && jin) ? G[(i0 + k) * M + j] : 0.0;
    const double xj = jin ? x[j] : 0.0;
    double cs = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        cs += g[k] * (i0 + k < M ? x[i0 + k] : 0.0);
        prod[wave * 16 + k][lane] = g[k] * xj;
    }
    red[1][wave][lane] = cs;
    __syncthreads();
    double rs = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) rs += prod[lane][wave * 16 + k];
    red[0][wave][lane] = rs;
    __syncthreads();
    if (wave == 0)
        part[(bi * nb + bj) * 64 + lane] =
            ((red[0][0][lane] + red[0][1][lane]) + red[0][2][lane]) + red[0][3][lane];
    else if (wave == 1 && bi != bj)
        part[(bj * nb + bi) * 64 + lane] =
            ((red[1][0][lane] + red[1][1][lane]) + red[1][2][lane]) + red[1][3][lane];
}

// Sum of n values by a 256-thread workgroup in a fixed order (the same in every workgroup);
// sh: 256 doubles of LDS.
__device__ double block_sum256(const double *__restrict__ v, int n, double *sh) {
    double a = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) a += v[k];
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double s = sh[0];
    __syncthreads();
    return s;
}

// Tree reduction of one value per thread of a 256-thread workgroup (result in thread 0).
__device__ double block_reduce256(double a, double *sh) {
    sh[threadIdx.x] = a;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    const double s = sh[0];
    __syncthreads();
    return s;
}

// Row block b (64 rows) of out = A x with A = L^T L + alpha D^T diag(gamma) D:
//   out = (sum_k part[b][k], or base) + alpha * Dt tD   (tD = diag(gamma) D x)
// and the partial <x, out> of the block in xpart[b].  1024 threads: with part, wave w adds
// k = w, w + 16, ... for every row and wave 0 then adds the sixteen sums in order.
__global__ __launch_bounds__(1024) void k_apply_sum(const double *__restrict__ part,
                                                    const double *__restrict__ base, int64_t M,
                                                    const int64_t *__restrict__ dtrp,
                                                    const int32_t *__restrict__ dtcol,
                                                    const double *__restrict__ dtval,
                                                    const double *__restrict__ tD, double alpha,
                                                    const double *__restrict__ x,
                                                    double *__restrict__ out,
                                                    double *__restrict__ xpart) {
    __shared__ double acc[16][64];
    const int64_t b = blockIdx.x, nb = (M + 63) / 64;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (part) {
        const double *pb = part + b * nb * 64 + lane;
        double s = 0.0;
        for (int64_t k = wave; k < nb; k += 16) s += pb[k * 64];
        acc[wave][lane] = s;
        __syncthreads();
    }
    if (wave) return;
    const int64_t i = b * 64 + lane;
    double v = 0.0;
    if (i < M) {
        if (part) {
            v = acc[0][lane];
#pragma unroll
            for (int w = 1; w < 16; ++w) v += acc[w][lane];
        } else {
            v = base[i];
        }
        if (dtrp) {
            double t = 0.0;
            for (int64_t k = dtrp[i]; k < dtrp[i + 1]; ++k) t += dtval[k] * tD[dtcol[k]];
            v = v + alpha * t;
        }
        out[i] = v;
    }
    double d = i < M ? x[i] * v : 0.0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) d += __shfl_xor(d, o);
    if (lane == 0) xpart[b] = d;
}

// out = a (.) b
__global__ void k_mul(const double *__restrict__ a, const double *__restrict__ b, int64_t M,
                      double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < M) out[i] = a[i] * b[i];
}

__global__ void k_sum_parts(const double *__restrict__ part, int64_t nchunk, int64_t M,
                            double *__restrict__ out) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= M) return;
    double s = 0.0;
    for (int64_t c = 0; c < nchunk; ++c) s += part[c * M + j];
    out[j] = s;
}

// y = diag(w) (A x) for CSR A (w may be null)
__global__ void k_spmv(const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                       const double *__restrict__ val, int64_t M, const double *__restrict__ x,
                       const double *__restrict__ w, double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= M) return;
    double s = 0.0;
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s += val[k] * x[col[k]];
    y[i] = w ? w[i] * s : s;
}

// out = a + alpha * b
__global__ void k_axpy(const double *__restrict__ a, double alpha, const double *__restrict__ b,
                       int64_t M, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < M) out[i] = a[i] + alpha * b[i];
}

// per-block partial dot products (fixed order); the host adds the partials
__global__ __launch_bounds__(256) void k_dot(const double *__restrict__ a,
                                             const double *__restrict__ b, int64_t M,
                                             double *__restrict__ part) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < M; i += (int64_t)gridDim.x * 256)
        s += a[i] * b[i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// the two partial dot products <a, b> and <a, a> of one CG step in one pass
__global__ __launch_bounds__(256) void k_dot2(const double *__restrict__ a,
                                              const double *__restrict__ b, int64_t M,
                                              double *__restrict__ part) {
    __shared__ double sh[2][256];
    double s = 0.0, t = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < M; i += (int64_t)gridDim.x * 256) {
        s += a[i] * b[i];
        t += a[i] * a[i];
    }
    sh[0][threadIdx.x] = s;
    sh[1][threadIdx.x] = t;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = sh[0][0];
        part[gridDim.x + blockIdx.x] = sh[1][0];
    }
}

// out[r][k] = sum_e w_e L[r][idx_e] over column k of a sparse combination matrix R
// (CSC: cptr, cidx, cw): L R for the coarse basis R_c and the pair basis R_f.
template <typename T>
__global__ __launch_bounds__(256) void k_colcomb(const T *__restrict__ L, int64_t rows, int64_t M,
                                                 const int64_t *__restrict__ cptr,
                                                 const int32_t *__restrict__ cidx,
                                                 const double *__restrict__ cw, int64_t K,
                                                 double *__restrict__ out) {
    const int64_t kb = (K + 255) / 256;
    const int64_t r = (int64_t)blockIdx.x / kb;
    const int64_t k = ((int64_t)blockIdx.x % kb) * 256 + threadIdx.x;
    if (r >= rows || k >= K) return;
    const T *row = L + r * M;
    double s = 0.0;
    for (int64_t e = cptr[k]; e < cptr[k + 1]; ++e) s += cw[e] * (double)row[cidx[e]];
    out[r * K + k] = s;
}

// Lt[c][a] = L[a][c] * sc[c]  (M x rows, FP64): the scaled transpose that the row Gram
// matrix L diag(sc^2) L^T is formed from
template <typename T>
__global__ __launch_bounds__(256) void k_scaled_transpose(const T *__restrict__ L, int64_t rows,
                                                          int64_t M, const double *__restrict__ sc,
                                                          double *__restrict__ Lt) {
    __shared__ double t[32][33];
    const int64_t c0 = (int64_t)blockIdx.x * 32, a0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    for (int k = ty; k < 32; k += 8) {
        const int64_t a = a0 + k, c = c0 + tx;
        t[k][tx] = (a < rows && c < M) ? (double)L[a * M + c] * sc[c] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int64_t c = c0 + k, a = a0 + tx;
        if (c < M && a < rows) Lt[c * rows + a] = t[tx][k];
    }
}

// In-place Cholesky factor (lower) and inverse of a small dense SPD matrix (host, n <= a
// few hundred): A^{-1} = L^{-T} L^{-1}.  Returns false if A is not positive definite.
bool spd_inverse(std::vector<double> &A, int64_t n) {
    for (int64_t j = 0; j < n; ++j) {
        double d = A[j * n + j];
        for (int64_t k = 0; k < j; ++k) d -= A[j * n + k] * A[j * n + k];
        if (!(d > 0)) return false;
        d = std::sqrt(d);
        A[j * n + j] = d;
        for (int64_t i = j + 1; i < n; ++i) {
            double v = A[i * n + j];
            for (int64_t k = 0; k < j; ++k) v -= A[i * n + k] * A[j * n + k];
            A[i * n + j] = v / d;
        }
    }
    // W = L^{-1} (lower), then A^{-1} = W^T W
    std::vector<double> W(n * n, 0.0);
    for (int64_t c = 0; c < n; ++c) {
        for (int64_t i = c; i < n; ++i) {
            double v = i == c ? 1.0 : 0.0;
            for (int64_t k = c; k < i; ++k) v -= A[i * n + k] * W[k * n + c];
            W[i * n + c] = v / A[i * n + i];
        }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            double v = 0.0;
            for (int64_t k = i; k < n; ++k) v += W[k * n + i] * W[k * n + j];
            A[i * n + j] = v;
            A[j * n + i] = v;
        }
    return true;
}

// CSR matrix (host)
struct Csr {
    int64_t nrows = 0, ncols = 0;
    std::vector<int64_t> rp{0};
    std::vector<int32_t> col;
    std::vector<double> val;

    std::vector<double> mul(const std::vector<double> &x) const {
        std::vector<double> y(nrows, 0.0);
        for (int64_t i = 0; i < nrows; ++i) {
            double s = 0.0;
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) s += val[k] * x[col[k]];
            y[i] = s;
        }
        return y;
    }

    Csr transpose() const {
        Csr t;
        t.nrows = ncols;
        t.ncols = nrows;
        t.rp.assign(ncols + 1, 0);
        t.col.resize(col.size());
        t.val.resize(val.size());
        for (size_t k = 0; k < col.size(); ++k) t.rp[col[k] + 1]++;
        for (int64_t i = 0; i < ncols; ++i) t.rp[i + 1] += t.rp[i];
        std::vector<int64_t> fill(t.rp.begin(), t.rp.end() - 1);
        for (int64_t i = 0; i < nrows; ++i)
            for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
                const int64_t p = fill[col[k]]++;
                t.col[p] = (int32_t)i;
                t.val[p] = val[k];
            }
        return t;
    }
};

Csr checked_csr(int64_t nrows, int64_t ncols, const int64_t *rp, const int32_t *col,
                const double *val, const char *what) {
    MGRT_REQUIRE(rp && col && val, MGRT_E_ARG, std::string("null CSR arrays for ") + what);
    MGRT_REQUIRE(rp[0] == 0, MGRT_E_ARG, std::string("bad CSR row pointer for ") + what);
    for (int64_t i = 0; i < nrows; ++i)
        MGRT_REQUIRE(rp[i + 1] >= rp[i], MGRT_E_ARG, std::string("CSR row pointer not monotone for ") + what);
    Csr a;
    a.nrows = nrows;
    a.ncols = ncols;
    a.rp.assign(rp, rp + nrows + 1);
    const int64_t nnz = rp[nrows];
    a.col.assign(col, col + nnz);
    a.val.assign(val, val + nnz);
    for (int64_t k = 0; k < nnz; ++k) {
        MGRT_REQUIRE(col[k] >= 0 && col[k] < ncols, MGRT_E_ARG, std::string("CSR column out of range for ") + what);
        MGRT_REQUIRE(std::isfinite(val[k]), MGRT_E_NONFINITE, std::string("non-finite entry in ") + what);
    }
    return a;
}

// Gamma = diag(1 / max(|v|, tau)), tau = 1e-8 max|v|; the identity when v vanishes
std::vector<double> tv_weights(const std::vector<double> &v) {
    double amax = 0.0;
    for (double x : v) amax = std::max(amax, std::fabs(x));
    std::vector<double> g(v.size(), 1.0);
    if (amax == 0.0) return g;
    const double tau = 1e-8 * amax;
    for (size_t i = 0; i < v.size(); ++i) g[i] = 1.0 / std::max(std::fabs(v[i]), tau);
    return g;
}

// One level of the TV iteration: L (rows x M, FP32/FP64 on the device) and D (CSR,
// Drows x M).  solve() runs preconditioned CG on
//   (L^T L + alpha D^T diag(gamma) D) z = b
// with FP64 vectors.  Products with L^T L use the normal matrix G when it is the smaller
// read (formed once on the matrix cores), else one pass over L each way.  Preconditioner:
// Jacobi, or for short L (rows <= LOWRANK_MAX_ROWS < M) the exact inverse of
// Lam + L^T L with Lam = alpha diag(D^T Gamma D), by the Woodbury identity
//   (Lam + L^T L)^{-1} v = Lam^{-1} v - Lam^{-1} L^T S^{-1} L Lam^{-1} v,
//   S = I + L Lam^{-1} L^T  (rows x rows, formed on the matrix cores, inverted on the host),
// Device-side CG scalars (so that an iteration needs no host synchronisation):
// sc[0], sc[1] rz (two slots, old and new alternate), sc[2] <p, A p>, sc[3] <r, r>,
// sc[4] a sticky flag set when <p, A p> was not positive (breakdown).
// Sum of per-block partials in a fixed order (one workgroup).
__global__ __launch_bounds__(256) void k_sum_to(const double *__restrict__ part, int n,
                                                double *__restrict__ out0, const double *__restrict__ part2,
                                                double *__restrict__ out1) {
    __shared__ double sh[2][256];
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) {
        a += part[k];
        if (part2) b += part2[k];
    }
    sh[0][threadIdx.x] = a;
    sh[1][threadIdx.x] = b;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + o];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *out0 = sh[0][0];
        if (out1) *out1 = sh[1][0];
    }
}

// One CG update with the step size a = rz / <p, A p> formed on the device: the partials of
// <p, A p> (qpart, nq of them) are added in a fixed order by every workgroup; rz = sc[slot].
// z += a p, r -= a q.  With pinv (Jacobi preconditioner) also zp = pinv r and the per-block
// partials of <r, zp> and <r, r> in part2[blockIdx], part2[gridDim + blockIdx].  A step with
// <p, A p> not positive (or not finite) is skipped and sets the breakdown flag sc[4].
__global__ __launch_bounds__(256) void k_cg_xr(double *__restrict__ z, const double *__restrict__ p,
                                               double *__restrict__ r, const double *__restrict__ q,
                                               int64_t M, const double *__restrict__ qpart, int nq,
                                               double *__restrict__ sc, int slot,
                                               const double *__restrict__ pinv,
                                               double *__restrict__ zp, double *__restrict__ part2) {
    __shared__ double sh[256];
    const double pq = block_sum256(qpart, nq, sh), rz = sc[slot];
    const bool ok = pq > 0.0 && isfinite(pq) && isfinite(rz);
    const double a = ok ? rz / pq : 0.0;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i == 0 && !ok) sc[4] = 1.0;
    double ri = 0.0, zi = 0.0;
    if (i < M) {
        z[i] += a * p[i];
        ri = r[i] - a * q[i];
        r[i] = ri;
        if (pinv) {
            zi = pinv[i] * ri;
            zp[i] = zi;
        }
    }
    if (!pinv) return;
    const double s = block_reduce256(ri * zi, sh);
    const double t = block_reduce256(ri * ri, sh);
    if (threadIdx.x == 0) {
        part2[blockIdx.x] = s;
        part2[gridDim.x + blockIdx.x] = t;
    }
}

// p = zp + (rz_new / rz_old) p with rz_new = <r, zp>, rr = <r, r> added from the n2 partials
// in part2 (fixed order); workgroup 0 stores rz_new in sc[slot_new] and rr in sc[3].
__global__ __launch_bounds__(256) void k_cg_p(const double *__restrict__ zp, double *__restrict__ p,
                                              int64_t M, const double *__restrict__ part2, int n2,
                                              double *__restrict__ sc, int slot_new, int slot_old) {
    __shared__ double sh[256];
    const double rn = block_sum256(part2, n2, sh);
    const double rr = block_sum256(part2 + n2, n2, sh);
    const double ro = sc[slot_old];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[slot_new] = rn;
        sc[3] = rr;
    }
    const double be = (ro > 0.0 && isfinite(rn / ro)) ? rn / ro : 0.0;
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < M) p[i] = zp[i] + be * p[i];
}

// which removes the spread of the data block from the spectrum CG sees.
struct TvSystem {
    Ctx &c;
    int64_t rows = 0, M = 0;
    int prec = 64;
    const void *L = nullptr;
    double alpha = 0.0;
    Csr D, Dt;
    DevBuf drp, dcol, dval, dtrp, dtcol, dtval, gam;
    DevBuf t_rows, t_D, t_M, part, dpart, Gm, pinv, res, p, q, zp, cgs, xpart, part2;
    std::vector<double> hltl;
    int64_t nchunk = 0;
    bool use_G = false;
    static constexpr int DOT_BLOCKS = 256;
    static constexpr int64_t LOWRANK_MAX_ROWS = 512;
    bool lowrank = false;
    DevBuf lam_inv, Sinv, pre_y, pre_t, pre_w, pre_u;
    DevBuf Am, Uinv, UinvT, cflag, wv, yv, dg0;    // direct solve: A = U^T U and its pieces
    bool no_room_direct = false;                    // the factor did not fit next to G

    explicit TvSystem(Ctx &cc) : c(cc) {}

    int64_t g(int64_t n) const { return (n + 255) / 256; }

    void init(int64_t rows_, int64_t M_, const void *L_, int prec_, Csr D_, double alpha_) {
        rows = rows_;
        M = M_;
        L = L_;
        prec = prec_;
        alpha = alpha_;
        D = std::move(D_);
        Dt = D.transpose();
        drp = upload(D.rp, c.stream); dcol = upload(D.col, c.stream); dval = upload(D.val, c.stream);
        dtrp = upload(Dt.rp, c.stream); dtcol = upload(Dt.col, c.stream); dtval = upload(Dt.val, c.stream);
        nchunk = (rows + TCHUNK - 1) / TCHUNK;
        part.alloc((size_t)nchunk * M * 8);
        dpart.alloc(2 * DOT_BLOCKS * 8);
        t_rows.alloc((size_t)rows * 8);
        t_D.alloc((size_t)std::max<int64_t>(D.nrows, 1) * 8);
        t_M.alloc((size_t)M * 8);
        cgs.alloc(8 * 8);
        xpart.alloc((size_t)((M + 63) / 64) * 8);
        part2.alloc((size_t)2 * std::max<int64_t>(g(M), DOT_BLOCKS) * 8);
        gam.alloc((size_t)std::max<int64_t>(D.nrows, 1) * 8);
        for (DevBuf *b : {&pinv, &res, &p, &q, &zp}) b->alloc((size_t)M * 8);
        // diag(L^T L) for the preconditioner
        DevBuf ltl(M * 8);
        colsq(ltl.as<double>());
        hltl.resize(M);
        MGRT_HIP(hipMemcpyAsync(hltl.data(), ltl.p, M * 8, hipMemcpyDeviceToHost, c.stream));
        MGRT_HIP(hipStreamSynchronize(c.stream));
        // normal matrix when one product with it moves fewer bytes than two passes over L
        // and it fits the free memory
        size_t fr = 0, tot = 0;
        MGRT_HIP(hipMemGetInfo(&fr, &tot));
        const double esz = prec == 32 ? 4.0 : 8.0;
        const double gbytes = (double)M * M * 8;
        if (gbytes < 2.0 * rows * M * esz && gbytes + (2ull << 30) < (double)fr) form_normal_matrix();
    }

    double dot(const double *a, const double *b) {
        hipLaunchKernelGGL(k_dot, dim3(DOT_BLOCKS), dim3(256), 0, c.stream, a, b, M, dpart.as<double>());
        double h[DOT_BLOCKS];
        MGRT_HIP(hipMemcpyAsync(h, dpart.p, sizeof(h), hipMemcpyDeviceToHost, c.stream));
        MGRT_HIP(hipStreamSynchronize(c.stream));
        double s = 0.0;
        for (int k = 0; k < DOT_BLOCKS; ++k) s += h[k];
        return s;
    }

    // {<a, b>, <a, a>} with one launch and one synchronisation
    void dot2(const double *a, const double *b, double &ab, double &aa) {
        hipLaunchKernelGGL(k_dot2, dim3(DOT_BLOCKS), dim3(256), 0, c.stream, a, b, M, dpart.as<double>());
        double h[2 * DOT_BLOCKS];
        MGRT_HIP(hipMemcpyAsync(h, dpart.p, sizeof(h), hipMemcpyDeviceToHost, c.stream));
        MGRT_HIP(hipStreamSynchronize(c.stream));
        ab = 0.0;
        aa = 0.0;
        for (int k = 0; k < DOT_BLOCKS; ++k) {
            ab += h[k];
            aa += h[DOT_BLOCKS + k];
        }
    }

    void Lx(const double *x, double *y) {
        const int64_t gr = (rows + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK;
        if (prec == 32)
            hipLaunchKernelGGL(k_gemv_n<float>, dim3(gr), dim3(256), 0, c.stream,
                               static_cast<const float *>(L), rows, M, x, y);
        else
            hipLaunchKernelGGL(k_gemv_n<double>, dim3(gr), dim3(256), 0, c.stream,
                               static_cast<const double *>(L), rows, M, x, y);
    }

    void Ltx(const double *y, double *x) {
        if (prec == 32)
            hipLaunchKernelGGL(k_gemv_t_part<float>, dim3(g(M), nchunk), dim3(256), 0, c.stream,
                               static_cast<const float *>(L), rows, M, y, part.as<double>());
        else
            hipLaunchKernelGGL(k_gemv_t_part<double>, dim3(g(M), nchunk), dim3(256), 0, c.stream,
                               static_cast<const double *>(L), rows, M, y, part.as<double>());
        hipLaunchKernelGGL(k_sum_parts, dim3(g(M)), dim3(256), 0, c.stream, part.as<double>(), nchunk, M, x);
    }

    void colsq(double *out) {
        if (prec == 32)
            hipLaunchKernelGGL(k_colsq_part<float>, dim3(g(M), nchunk), dim3(256), 0, c.stream,
                               static_cast<const float *>(L), rows, M, part.as<double>());
        else
            hipLaunchKernelGGL(k_colsq_part<double>, dim3(g(M), nchunk), dim3(256), 0, c.stream,
                               static_cast<const double *>(L), rows, M, part.as<double>());
        hipLaunchKernelGGL(k_sum_parts, dim3(g(M)), dim3(256), 0, c.stream, part.as<double>(), nchunk, M, out);
    }

    // G's upper blocks (the symmetric product reads nothing else) and their list
    DevBuf sym_pairs, sym_part;
    int64_t n_pairs = 0;

    void form_normal_matrix() {
        Gm.alloc((size_t)M * M * 8);
        const int64_t nb = (M + 63) / 64;
        if (prec == 32)
            hipLaunchKernelGGL(k_syrk<float>, dim3(nb, nb), dim3(256), 0, c.stream,
                               static_cast<const float *>(L), rows, M, Gm.as<double>());
        else
            hipLaunchKernelGGL(k_syrk<double>, dim3(nb, nb), dim3(256), 0, c.stream,
                               static_cast<const double *>(L), rows, M, Gm.as<double>());
        MGRT_HIP(hipGetLastError());
        std::vector<int2> pr;
        for (int64_t bi = 0; bi < nb; ++bi)
            for (int64_t bj = bi; bj < nb; ++bj) pr.push_back(make_int2((int)bi, (int)bj));
        n_pairs = (int64_t)pr.size();
        sym_pairs = upload(pr, c.stream);
        sym_part.alloc((size_t)nb * nb * 64 * 8);
        use_G = true;
    }

    // out = L^T L x + alpha D^T (gamma (.) D x), and the (M + 63) / 64 partials of <x, out>
    // in xpart
    void apply(const double *x, double *out) {
        const double *base = nullptr;
        if (use_G) {
            hipLaunchKernelGGL(k_symv_blocks, dim3(n_pairs), dim3(256), 0, c.stream,
                               static_cast<const double *>(Gm.as<double>()), M, sym_pairs.as<int2>(),
                               x, sym_part.as<double>());
        } else {
            Lx(x, t_rows.as<double>());
            Ltx(t_rows.as<double>(), t_M.as<double>());
            base = t_M.as<double>();
        }
        if (D.nrows)
            hipLaunchKernelGGL(k_spmv, dim3(g(D.nrows)), dim3(256), 0, c.stream, drp.as<int64_t>(),
                               dcol.as<int32_t>(), dval.as<double>(), D.nrows, x, gam.as<double>(),
                               t_D.as<double>());
        hipLaunchKernelGGL(k_apply_sum, dim3((M + 63) / 64), dim3(1024), 0, c.stream,
                           use_G ? static_cast<const double *>(sym_part.as<double>()) : nullptr, base, M,
                           D.nrows ? static_cast<const int64_t *>(dtrp.as<int64_t>()) : nullptr,
                           static_cast<const int32_t *>(dtcol.as<int32_t>()),
                           static_cast<const double *>(dtval.as<double>()),
                           static_cast<const double *>(t_D.as<double>()), alpha, x, out, xpart.as<double>());
    }

    // Woodbury preconditioner for Lam = diag(lam): S^{-1} = (I + L Lam^{-1} L^T)^{-1}
    bool build_lowrank(const std::vector<double> &lam) {
        std::vector<double> li(M), sc(M);
        for (int64_t j = 0; j < M; ++j) {
            li[j] = 1.0 / lam[j];
            sc[j] = std::sqrt(li[j]);
        }
        DevBuf dsc = upload(sc, c.stream);
        DevBuf Lt((size_t)M * rows * 8), Sg((size_t)rows * rows * 8);
        const dim3 tg((M + 31) / 32, (rows + 31) / 32);
        if (prec == 32)
            hipLaunchKernelGGL(k_scaled_transpose<float>, tg, dim3(256), 0, c.stream,
                               static_cast<const float *>(L), rows, M, dsc.as<double>(), Lt.as<double>());
        else
            hipLaunchKernelGGL(k_scaled_transpose<double>, tg, dim3(256), 0, c.stream,
                               static_cast<const double *>(L), rows, M, dsc.as<double>(), Lt.as<double>());
        const int64_t nb = (rows + 63) / 64;
        hipLaunchKernelGGL(k_syrk<double>, dim3(nb, nb), dim3(256), 0, c.stream,
                           static_cast<const double *>(Lt.as<double>()), M, rows, Sg.as<double>());
        hipLaunchKernelGGL(k_mirror_lower, dim3(nb, nb), dim3(256), 0, c.stream, Sg.as<double>(), rows);
        MGRT_HIP(hipGetLastError());
        std::vector<double> S((size_t)rows * rows);
        MGRT_HIP(hipMemcpyAsync(S.data(), Sg.p, S.size() * 8, hipMemcpyDeviceToHost, c.stream));
        MGRT_HIP(hipStreamSynchronize(c.stream));
        for (int64_t a = 0; a < rows; ++a) S[a * rows + a] += 1.0;
        if (!spd_inverse(S, rows)) return false;
        Sinv = upload(S, c.stream);
        lam_inv = upload(li, c.stream);
        for (DevBuf *b : {&pre_y, &pre_u}) b->alloc((size_t)M * 8);
        for (DevBuf *b : {&pre_t, &pre_w}) b->alloc((size_t)rows * 8);
        return true;
    }

    // zp = P^{-1} res
    void precondition(const double *res_, double *zp_) {
        if (!lowrank) {
            hipLaunchKernelGGL(k_mul, dim3(g(M)), dim3(256), 0, c.stream, pinv.as<double>(), res_, M, zp_);
            return;
        }
        double *y = pre_y.as<double>(), *u = pre_u.as<double>();
        hipLaunchKernelGGL(k_mul, dim3(g(M)), dim3(256), 0, c.stream, lam_inv.as<double>(), res_, M, y);
        Lx(y, pre_t.as<double>());
        const int64_t gr = (rows + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK;
        hipLaunchKernelGGL(k_gemv_n<double>, dim3(gr), dim3(256), 0, c.stream,
                           static_cast<const double *>(Sinv.as<double>()), rows, rows,
                           pre_t.as<double>(), pre_w.as<double>());
        Ltx(pre_w.as<double>(), u);
        hipLaunchKernelGGL(k_mul, dim3(g(M)), dim3(256), 0, c.stream, lam_inv.as<double>(), u, M, u);
        hipLaunchKernelGGL(k_axpy, dim3(g(M)), dim3(256), 0, c.stream, y, -1.0, u, M, zp_);
    }

    // The upper entries (a <= b) of D^T diag(gamma) D, row by row in a fixed order, as
    // (a * M + b, value) pairs.
    void dtgd_upper(const std::vector<double> &gamma, std::vector<int64_t> &idx,
                    std::vector<double> &val) const {
        idx.clear();
        val.clear();
        std::vector<double> acc(M, 0.0);
        std::vector<int64_t> mark(M, -1);
        std::vector<int32_t> cols;
        for (int64_t a = 0; a < M; ++a) {
            cols.clear();
            for (int64_t kr = Dt.rp[a]; kr < Dt.rp[a + 1]; ++kr) {
                const int32_t r = Dt.col[kr];
                const double gv = gamma[r] * Dt.val[kr];
                for (int64_t kk = D.rp[r]; kk < D.rp[r + 1]; ++kk) {
                    const int32_t bcol = D.col[kk];
                    if (bcol < a) continue;
                    if (mark[bcol] != a) {
                        mark[bcol] = a;
                        acc[bcol] = 0.0;
                        cols.push_back(bcol);
                    }
                    acc[bcol] += gv * D.val[kk];
                }
            }
            std::sort(cols.begin(), cols.end());
            for (int32_t bcol : cols) {
                idx.push_back(a * M + bcol);
                val.push_back(acc[bcol]);
            }
        }
    }

    // Direct solve of (G + alpha D^T Gamma D) z = b on the formed normal matrix: dense
    // Cholesky A = U^T U, then U^T y = b and U z = y.  Returns false (z untouched) when a
    // pivot is not positive, i.e. A is not numerically positive definite.
    bool solve_direct(const double *b, double *z, const std::vector<double> &gamma) {
        const int64_t nb = (M + 63) / 64;
        if (!Am.p) {
            Am.alloc((size_t)M * M * 8);
            Uinv.alloc((size_t)nb * 4096 * 8);
            UinvT.alloc((size_t)nb * 4096 * 8);
            cflag.alloc(sizeof(int));
            wv.alloc((size_t)M * 8);
            yv.alloc((size_t)M * 8);
            dg0.alloc((size_t)M * 8);
        }
        MGRT_HIP(hipMemcpyAsync(Am.p, Gm.p, (size_t)M * M * 8, hipMemcpyDeviceToDevice, c.stream));
        if (alpha > 0 && D.nrows > 0) {
            std::vector<int64_t> idx;
            std::vector<double> val;
            dtgd_upper(gamma, idx, val);
            if (!idx.empty()) {
                DevBuf di = upload(idx, c.stream), dv = upload(val, c.stream);
                hipLaunchKernelGGL(k_add_entries, dim3(g((int64_t)idx.size())), dim3(256), 0, c.stream,
                                   Am.as<double>(), di.as<int64_t>(), dv.as<double>(), (int64_t)idx.size(), alpha);
                MGRT_HIP(hipStreamSynchronize(c.stream));   // di, dv are freed on return
            }
        }
        MGRT_HIP(hipMemsetAsync(cflag.p, 0, sizeof(int), c.stream));
        double *A = Am.as<double>();
        hipLaunchKernelGGL(k_get_diag, dim3(g(M)), dim3(256), 0, c.stream, static_cast<const double *>(A), M,
                           dg0.as<double>());
        for (int64_t k = 0; k < nb; ++k) {
            hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, c.stream, A, M, k,
                               static_cast<const double *>(dg0.as<double>()), Uinv.as<double>(),
                               UinvT.as<double>(), cflag.as<int>());
            const int64_t rest = nb - k - 1;
            if (rest > 0) {
                hipLaunchKernelGGL(k_chol_xty, dim3(rest), dim3(256), 0, c.stream, A, M, k,
                                   static_cast<const double *>(Uinv.as<double>()), 0);
                hipLaunchKernelGGL(k_chol_xty, dim3(rest, rest), dim3(256), 0, c.stream, A, M, k,
                                   static_cast<const double *>(Uinv.as<double>()), 1);
            }
        }
        MGRT_HIP(hipGetLastError());
        int bad = 0;
        MGRT_HIP(hipMemcpyAsync(&bad, cflag.p, sizeof(int), hipMemcpyDeviceToHost, c.stream));
        MGRT_HIP(hipStreamSynchronize(c.stream));
        if (bad) return false;
        MGRT_HIP(hipMemcpyAsync(wv.p, b, (size_t)M * 8, hipMemcpyDeviceToDevice, c.stream));
        for (int64_t k = 0; k < nb; ++k)
            hipLaunchKernelGGL(k_chol_fwd, dim3(std::max<int64_t>(1, nb - k - 1)), dim3(256), 0, c.stream,
                               static_cast<const double *>(A), M, k,
                               static_cast<const double *>(Uinv.as<double>()), wv.as<double>(), yv.as<double>());
        for (int64_t k = nb - 1; k >= 0; --k)
            hipLaunchKernelGGL(k_chol_bwd, dim3(std::max<int64_t>(1, k)), dim3(256), 0, c.stream,
                               static_cast<const double *>(A), M, k,
                               static_cast<const double *>(UinvT.as<double>()), yv.as<double>(), z);
        MGRT_HIP(hipGetLastError());
        return true;
    }

    // One TV step's linear solve.  direct: Cholesky when the normal matrix is formed (0
    // iterations returned), PCG otherwise or when the factorisation meets a non-positive
    // pivot.
    int solve_step(const double *b, double *z, const std::vector<double> &gamma, double rtol, int maxit,
                   bool direct) {
        MGRT_REQUIRE((int64_t)gamma.size() == D.nrows, MGRT_E_ARG, "weights size mismatch");
        if (direct && use_G && !no_room_direct) {
            bool done = false;
            try {
                done = solve_direct(b, z, gamma);
            } catch (const Error &e) {
                if (e.code != MGRT_E_OOM_PLAN) throw;
                // no device memory for the factor next to G: solve by PCG from now on
                for (DevBuf *d : {&Am, &Uinv, &UinvT, &cflag, &wv, &yv, &dg0}) d->release();
                (void)hipGetLastError();
                no_room_direct = true;
            }
            if (done) return 0;
        }
        return solve(b, z, gamma, rtol, maxit);
    }

    // Preconditioned CG on A z = b from the z it is given (device vectors of length M);
    // gamma: D.nrows weights.  Returns the iterations taken.
    int solve(const double *b, double *z, const std::vector<double> &gamma, double rtol, int maxit) {
        MGRT_REQUIRE((int64_t)gamma.size() == D.nrows, MGRT_E_ARG, "weights size mismatch");
        if (D.nrows)
            MGRT_HIP(hipMemcpy(gam.p, gamma.data(), D.nrows * 8, hipMemcpyHostToDevice));
        std::vector<double> hp(M), lam(M);
        bool lam_pos = alpha > 0;
        for (int64_t j = 0; j < M; ++j) {
            double dd = 0;
            for (int64_t k = Dt.rp[j]; k < Dt.rp[j + 1]; ++k) dd += gamma[Dt.col[k]] * Dt.val[k] * Dt.val[k];
            const double dj = hltl[j] + alpha * dd;
            hp[j] = dj > 0 ? 1.0 / dj : 1.0;
            lam[j] = alpha * dd;
            lam_pos = lam_pos && lam[j] > 0 && std::isfinite(lam[j]);
        }
        MGRT_HIP(hipMemcpy(pinv.p, hp.data(), M * 8, hipMemcpyHostToDevice));
        lowrank = rows <= LOWRANK_MAX_ROWS && rows < M && lam_pos && build_lowrank(lam);
        const double bnorm = std::sqrt(dot(b, b));
        apply(z, q.as<double>());
        hipLaunchKernelGGL(k_axpy, dim3(g(M)), dim3(256), 0, c.stream, b, -1.0, q.as<double>(), M,
                           res.as<double>());
        precondition(res.as<double>(), zp.as<double>());
        MGRT_HIP(hipMemcpyAsync(p.p, zp.p, M * 8, hipMemcpyDeviceToDevice, c.stream));
        // scalars stay on the device; the host reads them every CHECK iterations
        constexpr int CHECK = 8;
        MGRT_HIP(hipMemsetAsync(cgs.p, 0, 8 * 8, c.stream));
        double *sc = cgs.as<double>(), *dp = dpart.as<double>(), *p2 = part2.as<double>();
        hipLaunchKernelGGL(k_dot2, dim3(DOT_BLOCKS), dim3(256), 0, c.stream, res.as<double>(), zp.as<double>(), M, dp);
        hipLaunchKernelGGL(k_sum_to, dim3(1), dim3(256), 0, c.stream, dp, DOT_BLOCKS, sc + 0,
                           (const double *)(dp + DOT_BLOCKS), sc + 3);
        double hs[5];
        MGRT_HIP(hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, c.stream));
        MGRT_HIP(hipStreamSynchronize(c.stream));
        MGRT_REQUIRE(std::isfinite(hs[3]), MGRT_E_NONFINITE, "non-finite CG residual");
        const int nq = (int)((M + 63) / 64);
        const int gM = (int)g(M);
        int k = 0, slot = 0;
        bool done = std::sqrt(hs[3]) <= rtol * bnorm;
        while (!done && k < maxit) {
            apply(p.as<double>(), q.as<double>());
            hipLaunchKernelGGL(k_cg_xr, dim3(gM), dim3(256), 0, c.stream, z, p.as<double>(), res.as<double>(),
                               q.as<double>(), M, (const double *)xpart.as<double>(), nq, sc, slot,
                               lowrank ? nullptr : static_cast<const double *>(pinv.as<double>()),
                               zp.as<double>(), p2);
            int n2 = gM;
            if (lowrank) {
                precondition(res.as<double>(), zp.as<double>());
                hipLaunchKernelGGL(k_dot2, dim3(DOT_BLOCKS), dim3(256), 0, c.stream, res.as<double>(),
                                   zp.as<double>(), M, p2);
                n2 = DOT_BLOCKS;
            }
            hipLaunchKernelGGL(k_cg_p, dim3(gM), dim3(256), 0, c.stream, zp.as<double>(), p.as<double>(), M,
                               (const double *)p2, n2, sc, 1 - slot, slot);
            slot = 1 - slot;
            ++k;
            if (k % CHECK == 0 || k == maxit) {
                MGRT_HIP(hipMemcpyAsync(hs, sc, sizeof(hs), hipMemcpyDeviceToHost, c.stream));
                MGRT_HIP(hipStreamSynchronize(c.stream));
                MGRT_REQUIRE(std::isfinite(hs[3]), MGRT_E_NONFINITE, "non-finite CG residual");
                done = std::sqrt(hs[3]) <= rtol * bnorm;
                MGRT_REQUIRE(done || hs[4] == 0.0, MGRT_E_NONFINITE,
                             "normal matrix not positive definite (CG breakdown)");
            }
        }
        MGRT_HIP(hipGetLastError());
        return k;
    }
};

std::vector<double> to_host(const DevBuf &b, int64_t n, hipStream_t s) {
    std::vector<double> h(n);
    if (n) MGRT_HIP(hipMemcpyAsync(h.data(), b.p, n * 8, hipMemcpyDeviceToHost, s));
    MGRT_HIP(hipStreamSynchronize(s));
    for (double v : h) MGRT_REQUIRE(std::isfinite(v), MGRT_E_NONFINITE, "non-finite iterate");
    return h;
}

// L on the device: the caller's pointer, or a copy of the host matrix
const void *device_matrix(Ctx &c, const void *L, int on_device, int64_t rows, int64_t M, size_t esz,
                          DevBuf &own) {
    if (on_device) return L;
    own.alloc((size_t)rows * M * esz);
    MGRT_HIP(hipMemcpy(own.p, L, (size_t)rows * M * esz, hipMemcpyHostToDevice));
    (void)c;
    return own.p;
}

// L R for a sparse combination matrix R (CSC, M x K) into a new FP64 matrix (rows x K)
void combine_columns(Ctx &c, const void *L, int prec, int64_t rows, int64_t M,
                     const std::vector<int64_t> &cptr, const std::vector<int32_t> &cidx,
                     const std::vector<double> &cw, DevBuf &out) {
    const int64_t K = (int64_t)cptr.size() - 1;
    out.alloc((size_t)rows * K * 8);
    if (K == 0) return;
    DevBuf dp = upload(cptr, c.stream), di = upload(cidx, c.stream), dw = upload(cw, c.stream);
    const int64_t blocks = rows * ((K + 255) / 256);
    if (prec == 32)
        hipLaunchKernelGGL(k_colcomb<float>, dim3(blocks), dim3(256), 0, c.stream,
                           static_cast<const float *>(L), rows, M, dp.as<int64_t>(), di.as<int32_t>(),
                           dw.as<double>(), K, out.as<double>());
    else
        hipLaunchKernelGGL(k_colcomb<double>, dim3(blocks), dim3(256), 0, c.stream,
                           static_cast<const double *>(L), rows, M, dp.as<int64_t>(), di.as<int32_t>(),
                           dw.as<double>(), K, out.as<double>());
    MGRT_HIP(hipGetLastError());
    MGRT_HIP(hipStreamSynchronize(c.stream));
}

// Fine-fluctuation basis of one parent (Sec. II-D, Fig. 3): +1/-1 on adjacent siblings
// (sharing a facet), the edges of a spanning tree of the siblings' facet adjacency
// rooted at the sibling with most sibling neighbours (lowest id on ties); in 2D the
// middle triangle, so every pair is corner/middle.
struct Pair {
    int32_t plus, minus;
};

std::vector<std::vector<Pair>> pair_basis(int dim, int64_t M, int64_t M2, const int32_t *verts,
                                          const std::vector<std::vector<int32_t>> &kids) {
    const int nv = dim + 1;
    auto share_facet = [&](int32_t a, int32_t b) {
        int common = 0;
        for (int i = 0; i < nv; ++i)
            for (int j = 0; j < nv; ++j) common += verts[(int64_t)a * nv + i] == verts[(int64_t)b * nv + j];
        return common == dim;
    };
    (void)M;
    std::vector<std::vector<Pair>> out(M2);
    for (int64_t P = 0; P < M2; ++P) {
        const auto &ch = kids[P];   // ascending ids
        const size_t nk = ch.size();
        if (nk <= 1) continue;
        std::vector<std::vector<int>> adj(nk);
        for (size_t a = 0; a < nk; ++a)
            for (size_t b = 0; b < nk; ++b)
                if (a != b && share_facet(ch[a], ch[b])) adj[a].push_back((int)b);
        size_t root = 0;
        for (size_t a = 1; a < nk; ++a)
            if (adj[a].size() > adj[root].size()) root = a;
        std::vector<char> seen(nk, 0);
        std::vector<size_t> queue{root};
        seen[root] = 1;
        for (size_t qi = 0; qi < queue.size(); ++qi) {
            const size_t a = queue[qi];
            for (int b : adj[a]) {
                if (seen[b]) continue;
                seen[b] = 1;
                queue.push_back(b);
                out[P].push_back({ch[b], ch[a]});
            }
        }
        MGRT_REQUIRE(queue.size() == nk, MGRT_E_MESH,
                     "the children of a coarse element are not connected through shared facets");
    }
    return out;
}

}  // namespace

}  // namespace mgrt

using namespace mgrt;

extern "C" int mgrt_tv_invert_level(mgrt_ctx *ctx, int64_t rows, int64_t M, const void *L,
                                    int L_precision, int L_on_device, const double *r,
                                    const int64_t *D_rowptr, const int32_t *D_col,
                                    const double *D_val, double alpha, int iters, double cg_rtol,
                                    int cg_maxit, int solver, double *z_out, int32_t *cg_iters) {
    return mgrt_guarded(ctx, [&](Ctx &c) {
        MGRT_REQUIRE(rows >= 1 && M >= 1 && L && r && z_out, MGRT_E_ARG, "bad sizes or null pointers");
        MGRT_REQUIRE(L_precision == 32 || L_precision == 64, MGRT_E_ARG, "L precision must be 32 or 64");
        MGRT_REQUIRE(iters >= 1 && cg_maxit >= 1 && cg_rtol > 0, MGRT_E_ARG, "bad iteration limits");
        MGRT_REQUIRE(solver == MGRT_TV_AUTO || solver == MGRT_TV_CG, MGRT_E_ARG, "unknown solver");
        MGRT_REQUIRE(std::isfinite(alpha) && alpha >= 0, MGRT_E_ARG, "alpha must be >= 0");
        Csr D = checked_csr(M, M, D_rowptr, D_col, D_val, "D");
        for (int64_t k = 0; k < rows; ++k) MGRT_REQUIRE(std::isfinite(r[k]), MGRT_E_NONFINITE, "non-finite r");
        const size_t esz = L_precision == 32 ? 4 : 8;
        DevBuf Lown;
        const void *Ld = device_matrix(c, L, L_on_device, rows, M, esz, Lown);
        TvSystem S(c);
        S.init(rows, M, Ld, L_precision, D, alpha);
        DevBuf dr = upload(std::vector<double>(r, r + rows), c.stream);
        DevBuf b(M * 8), z(M * 8);
        S.Ltx(dr.as<double>(), b.as<double>());
        MGRT_HIP(hipMemsetAsync(z.p, 0, M * 8, c.stream));
        std::vector<double> hz(M, 0.0);
        for (int it = 0; it < iters; ++it) {
            // Gamma_0 = I; Gamma_l from |D z_l| floored at tau
            const std::vector<double> gam = it == 0 ? std::vector<double>(M, 1.0) : tv_weights(D.mul(hz));
            const int k = S.solve_step(b.as<double>(), z.as<double>(), gam, cg_rtol, cg_maxit,
                                       solver == MGRT_TV_AUTO);
            if (cg_iters) cg_iters[it] = k;
            hz = to_host(z, M, c.stream);
            std::copy(hz.begin(), hz.end(), z_out + (int64_t)it * M);
        }
    });
}

// Coarse-to-fine TV inversion over two nested levels (Sec. II-D, eqs. decomposition,
// tv_iteration_0 and tv_iteration_2; compression of Sec. II-E).  The coarse step solves
// on L_c = L R_c with D_c; the kept fine fluctuations (pair basis of the n_keep parents
// with the largest |z_c|) on L_f = L R_f with the T' matrix D_f applied to the fine field
// R_f z_f, against the data left by the coarse step.  Gamma of each level comes from its
// previous iterate (the fine one from the previous fine field on T').
extern "C" int mgrt_tv_invert_two_level(
    mgrt_ctx *ctx, int64_t rows, int64_t M, const void *L, int L_precision, int L_on_device,
    const double *r, int dim, const int32_t *elem_verts, int64_t M2, const int32_t *parent,
    const int64_t *Dc_rowptr, const int32_t *Dc_col, const double *Dc_val,
    const int64_t *Df_rowptr, const int32_t *Df_col, const double *Df_val, double alpha,
    int iters, int64_t n_keep, double cg_rtol, int cg_maxit, int solver, double *x_out,
    double *zc_out, int32_t *kept_out, int32_t *cg_iters) {
    return mgrt_guarded(ctx, [&](Ctx &c) {
        MGRT_REQUIRE(rows >= 1 && M >= 1 && M2 >= 1 && L && r && x_out && elem_verts && parent,
                     MGRT_E_ARG, "bad sizes or null pointers");
        MGRT_REQUIRE(dim == 2 || dim == 3, MGRT_E_ARG, "dim must be 2 or 3");
        MGRT_REQUIRE(L_precision == 32 || L_precision == 64, MGRT_E_ARG, "L precision must be 32 or 64");
        MGRT_REQUIRE(iters >= 1 && cg_maxit >= 1 && cg_rtol > 0 && n_keep >= 0, MGRT_E_ARG,
                     "bad iteration limits or n_keep");
        MGRT_REQUIRE(solver == MGRT_TV_AUTO || solver == MGRT_TV_CG, MGRT_E_ARG, "unknown solver");
        MGRT_REQUIRE(std::isfinite(alpha) && alpha >= 0, MGRT_E_ARG, "alpha must be >= 0");
        Csr Dc = checked_csr(M2, M2, Dc_rowptr, Dc_col, Dc_val, "D_c");
        Csr Df = checked_csr(M, M, Df_rowptr, Df_col, Df_val, "D_f");
        for (int64_t k = 0; k < rows; ++k) MGRT_REQUIRE(std::isfinite(r[k]), MGRT_E_NONFINITE, "non-finite r");
        std::vector<std::vector<int32_t>> kids(M2);
        for (int64_t e = 0; e < M; ++e) {
            MGRT_REQUIRE(parent[e] >= 0 && parent[e] < M2, MGRT_E_ARG, "parent id out of range");
            kids[parent[e]].push_back((int32_t)e);
        }
        for (int64_t P = 0; P < M2; ++P) MGRT_REQUIRE(!kids[P].empty(), MGRT_E_MESH, "coarse element without children");
        const auto pairs = pair_basis(dim, M, M2, elem_verts, kids);
        const int64_t keep = std::min(n_keep, M2);

        const size_t esz = L_precision == 32 ? 4 : 8;
        DevBuf Lown;
        const void *Ld = device_matrix(c, L, L_on_device, rows, M, esz, Lown);
        DevBuf dr = upload(std::vector<double>(r, r + rows), c.stream);

        // coarse level: L_c = L R_c
        std::vector<int64_t> cp{0};
        std::vector<int32_t> ci;
        std::vector<double> cwt;
        for (int64_t P = 0; P < M2; ++P) {
            for (int32_t e : kids[P]) { ci.push_back(e); cwt.push_back(1.0); }
            cp.push_back((int64_t)ci.size());
        }
        DevBuf Lc;
        combine_columns(c, Ld, L_precision, rows, M, cp, ci, cwt, Lc);
        TvSystem Sc(c);
        Sc.init(rows, M2, Lc.p, 64, Dc, alpha);
        DevBuf bc(M2 * 8), zc(M2 * 8), rf(rows * 8), tmp(rows * 8);
        Sc.Ltx(dr.as<double>(), bc.as<double>());
        MGRT_HIP(hipMemsetAsync(zc.p, 0, M2 * 8, c.stream));
        std::vector<double> hzc(M2, 0.0), f(M, 0.0);
        for (int it = 0; it < iters; ++it) {
            // (2) coarse step
            const std::vector<double> gc = it == 0 ? std::vector<double>(M2, 1.0) : tv_weights(Dc.mul(hzc));
            const int kc = Sc.solve_step(bc.as<double>(), zc.as<double>(), gc, cg_rtol, cg_maxit,
                                         solver == MGRT_TV_AUTO);
            hzc = to_host(zc, M2, c.stream);
            // compression: parents with the largest |z_c| (ties: lower id)
            std::vector<int32_t> order(M2);
            for (int64_t P = 0; P < M2; ++P) order[P] = (int32_t)P;
            std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
                return std::fabs(hzc[a]) > std::fabs(hzc[b]);
            });
            std::vector<int32_t> kept(order.begin(), order.begin() + keep);
            std::sort(kept.begin(), kept.end());
            // R_f restricted to the kept parents (CSC) and the columns of every element
            std::vector<int64_t> fp{0};
            std::vector<int32_t> fi;
            std::vector<double> fw;
            std::vector<std::vector<std::pair<int32_t, double>>> in_cols(M);
            for (int32_t P : kept)
                for (const Pair &pr : pairs[P]) {
                    const int32_t k = (int32_t)(fp.size() - 1);
                    fi.push_back(pr.plus); fw.push_back(1.0);
                    fi.push_back(pr.minus); fw.push_back(-1.0);
                    fp.push_back((int64_t)fi.size());
                    in_cols[pr.plus].push_back({k, 1.0});
                    in_cols[pr.minus].push_back({k, -1.0});
                }
            const int64_t K = (int64_t)fp.size() - 1;
            int kf = 0;
            std::vector<double> fnew(M, 0.0);
            if (K > 0) {
                // (3) fine step against the data left by the coarse step
                Sc.Lx(zc.as<double>(), tmp.as<double>());
                hipLaunchKernelGGL(k_axpy, dim3((rows + 255) / 256), dim3(256), 0, c.stream,
                                   dr.as<double>(), -1.0, tmp.as<double>(), rows, rf.as<double>());
                DevBuf Lf;
                combine_columns(c, Ld, L_precision, rows, M, fp, fi, fw, Lf);
                // D_f R_f (M x K, CSR)
                Csr DR;
                DR.nrows = M;
                DR.ncols = K;
                DR.rp.assign(1, 0);
                std::vector<std::pair<int32_t, double>> acc;
                for (int64_t i = 0; i < M; ++i) {
                    acc.clear();
                    for (int64_t q = Df.rp[i]; q < Df.rp[i + 1]; ++q)
                        for (const auto &cv : in_cols[Df.col[q]]) acc.push_back({cv.first, Df.val[q] * cv.second});
                    std::sort(acc.begin(), acc.end(),
                              [](const std::pair<int32_t, double> &a, const std::pair<int32_t, double> &b) {
                                  return a.first < b.first;
                              });
                    for (size_t q = 0; q < acc.size(); ++q) {
                        if (q > 0 && acc[q].first == DR.col.back() && (int64_t)DR.col.size() > DR.rp.back()) {
                            DR.val.back() += acc[q].second;
                        } else {
                            DR.col.push_back(acc[q].first);
                            DR.val.push_back(acc[q].second);
                        }
                    }
                    DR.rp.push_back((int64_t)DR.col.size());
                }
                TvSystem Sf(c);
                Sf.init(rows, K, Lf.p, 64, std::move(DR), alpha);
                DevBuf bf(K * 8), zf(K * 8);
                Sf.Ltx(rf.as<double>(), bf.as<double>());
                MGRT_HIP(hipMemsetAsync(zf.p, 0, K * 8, c.stream));
                const std::vector<double> gf = it == 0 ? std::vector<double>(M, 1.0) : tv_weights(Df.mul(f));
                kf = Sf.solve_step(bf.as<double>(), zf.as<double>(), gf, cg_rtol, cg_maxit,
                                   solver == MGRT_TV_AUTO);
                const std::vector<double> hzf = to_host(zf, K, c.stream);
                for (int64_t k = 0; k < K; ++k) {
                    fnew[fi[2 * k]] += hzf[k];
                    fnew[fi[2 * k + 1]] -= hzf[k];
                }
            }
            f.swap(fnew);
            // (4) x_{l+1} - x0 = R_c z_c + R_f z_f
            for (int64_t e = 0; e < M; ++e) x_out[(int64_t)it * M + e] = hzc[parent[e]] + f[e];
            if (zc_out) std::copy(hzc.begin(), hzc.end(), zc_out + (int64_t)it * M2);
            if (kept_out) std::copy(kept.begin(), kept.end(), kept_out + (int64_t)it * keep);
            if (cg_iters) {
                cg_iters[2 * it] = kc;
                cg_iters[2 * it + 1] = kf;
            }
        }
        MGRT_HIP(hipGetLastError());
    });
}
