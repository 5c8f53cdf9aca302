// TV-regularised linearised inversion on one level (Sec. II-C, eq. tv_iteration):
//   z_{l+1} = (L^T L + alpha D^T Gamma_l D)^{-1} L^T r,   Gamma_0 = I,
//   Gamma_l = diag(1 / max(|D z_l|, tau)),  tau = 1e-8 max|D z_l|.
// Each system is solved by Jacobi-preconditioned conjugate gradients (warm-started from
// z_l; preconditioner diag(L^T L) + alpha diag(D^T Gamma D)) with FP64 vectors and
// reductions.  Products with L stream the matrix row-major: y = L x with one
// workgroup per row block, x = L^T y with thread-per-column partial sums over row chunks
// reduced in a fixed order (deterministic).  When the normal matrix G = L^T L (M x M, FP64)
// is smaller than two passes over L, it is formed once per call on the FP64 matrix cores and
// each CG product reads G instead of L.
#include <algorithm>
#include <cmath>

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
// 2 x 2 MFMA tiles.  L streams through LDS in panels of SYRK_KT rows (converted to FP64).
// MFMA operand layout (wave64): lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// of the 16x4 and 4x16 operands and receives D[4 v + l / 16][l % 16] in slot v.
// Off-diagonal blocks are mirrored by k_mirror_lower.
constexpr int SYRK_KT = 16;
constexpr int SYRK_PAD = 4;
typedef double d4v __attribute__((ext_vector_type(4)));

template <typename T>
__global__ __launch_bounds__(256) void k_syrk(const T *__restrict__ L, int64_t rows, int64_t M,
                                              double *__restrict__ G) {
    const int64_t bi = blockIdx.y, bj = blockIdx.x;
    if (bj < bi) return;
    __shared__ double As[SYRK_KT][64 + SYRK_PAD];
    __shared__ double Bs[SYRK_KT][64 + SYRK_PAD];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int wy = wave >> 1, wx = wave & 1;
    const int64_t i0 = bi * 64, j0 = bj * 64;
    d4v acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4v{0.0, 0.0, 0.0, 0.0};
    for (int64_t r0 = 0; r0 < rows; r0 += SYRK_KT) {
        for (int e = tid; e < SYRK_KT * 64; e += 256) {
            const int kr = e >> 6, cc = e & 63;
            const int64_t r = r0 + kr;
            As[kr][cc] = (r < rows && i0 + cc < M) ? (double)L[r * M + i0 + cc] : 0.0;
            Bs[kr][cc] = (r < rows && j0 + cc < M) ? (double)L[r * M + j0 + cc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < SYRK_KT; kk += 4) {
            const int kr = kk + (lane >> 4), cc = lane & 15;
            const double a0 = As[kr][32 * wy + cc], a1 = As[kr][32 * wy + 16 + cc];
            const double b0 = Bs[kr][32 * wx + cc], b1 = Bs[kr][32 * wx + 16 + cc];
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
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
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
        if (threadIdx.x < o) {
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

struct TvSolver {
    Ctx &c;
    int64_t rows, M;
    int prec;
    const void *L;
    DevBuf Lown;
    DevBuf drp, dcol, dval, dtrp, dtcol, dtval;
    DevBuf gam;
    DevBuf t_rows, t_M1, t_M2, part, dpart;
    int64_t nchunk;
    double alpha;
    static constexpr int DOT_BLOCKS = 256;

    TvSolver(Ctx &cc) : c(cc) {}

    int64_t g(int64_t n) const { return (n + 255) / 256; }

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

    // G = L^T L formed once when a CG iteration then reads fewer bytes (M^2 FP64 vs
    // two passes over L)
    DevBuf Gm;
    bool use_G = false;

    void form_normal_matrix() {
        Gm.alloc((size_t)M * M * 8);
        const int64_t nb = (M + 63) / 64;
        if (prec == 32)
            hipLaunchKernelGGL(k_syrk<float>, dim3(nb, nb), dim3(256), 0, c.stream,
                               static_cast<const float *>(L), rows, M, Gm.as<double>());
        else
            hipLaunchKernelGGL(k_syrk<double>, dim3(nb, nb), dim3(256), 0, c.stream,
                               static_cast<const double *>(L), rows, M, Gm.as<double>());
        hipLaunchKernelGGL(k_mirror_lower, dim3(nb, nb), dim3(256), 0, c.stream, Gm.as<double>(), M);
        MGRT_HIP(hipGetLastError());
        use_G = true;
    }

    // out = L^T L x + alpha D^T (gamma (.) D x)
    void apply(const double *x, double *out) {
        if (use_G) {
            const int64_t gr = (M + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK;
            hipLaunchKernelGGL(k_gemv_n<double>, dim3(gr), dim3(256), 0, c.stream,
                               static_cast<const double *>(Gm.as<double>()), M, M, x, out);
        } else {
            Lx(x, t_rows.as<double>());
            Ltx(t_rows.as<double>(), out);
        }
        hipLaunchKernelGGL(k_spmv, dim3(g(M)), dim3(256), 0, c.stream, drp.as<int64_t>(), dcol.as<int32_t>(),
                           dval.as<double>(), M, x, gam.as<double>(), t_M1.as<double>());
        hipLaunchKernelGGL(k_spmv, dim3(g(M)), dim3(256), 0, c.stream, dtrp.as<int64_t>(), dtcol.as<int32_t>(),
                           dtval.as<double>(), M, t_M1.as<double>(), (const double *)nullptr, t_M2.as<double>());
        hipLaunchKernelGGL(k_axpy, dim3(g(M)), dim3(256), 0, c.stream, out, alpha, t_M2.as<double>(), M, out);
    }
};

}  // namespace

}  // namespace mgrt

using namespace mgrt;

extern "C" int mgrt_tv_invert_level(mgrt_ctx *ctx, int64_t rows, int64_t M, const void *L,
                                    int L_precision, int L_on_device, const double *r,
                                    const int64_t *D_rowptr, const int32_t *D_col,
                                    const double *D_val, double alpha, int iters, double cg_rtol,
                                    int cg_maxit, double *z_out, int32_t *cg_iters) {
    return mgrt_guarded(ctx, [&](Ctx &c) {
        MGRT_REQUIRE(rows >= 1 && M >= 1 && L && r && z_out, MGRT_E_ARG, "bad sizes or null pointers");
        MGRT_REQUIRE(D_rowptr && D_col && D_val, MGRT_E_ARG, "null regularisation matrix");
        MGRT_REQUIRE(L_precision == 32 || L_precision == 64, MGRT_E_ARG, "L precision must be 32 or 64");
        MGRT_REQUIRE(iters >= 1 && cg_maxit >= 1 && cg_rtol > 0, MGRT_E_ARG, "bad iteration limits");
        MGRT_REQUIRE(std::isfinite(alpha) && alpha >= 0, MGRT_E_ARG, "alpha must be >= 0");
        const int64_t nnz = D_rowptr[M];
        MGRT_REQUIRE(D_rowptr[0] == 0 && nnz >= 0, MGRT_E_ARG, "bad CSR row pointer");
        for (int64_t i = 0; i < M; ++i)
            MGRT_REQUIRE(D_rowptr[i + 1] >= D_rowptr[i], MGRT_E_ARG, "CSR row pointer not monotone");
        for (int64_t k = 0; k < nnz; ++k) {
            MGRT_REQUIRE(D_col[k] >= 0 && D_col[k] < M, MGRT_E_ARG, "CSR column out of range");
            MGRT_REQUIRE(std::isfinite(D_val[k]), MGRT_E_NONFINITE, "non-finite D entry");
        }
        for (int64_t k = 0; k < rows; ++k) MGRT_REQUIRE(std::isfinite(r[k]), MGRT_E_NONFINITE, "non-finite r");
        TvSolver S(c);
        S.rows = rows;
        S.M = M;
        S.prec = L_precision;
        S.alpha = alpha;
        const size_t esz = L_precision == 32 ? 4 : 8;
        if (L_on_device) {
            S.L = L;
        } else {
            S.Lown.alloc((size_t)rows * M * esz);
            MGRT_HIP(hipMemcpy(S.Lown.p, L, (size_t)rows * M * esz, hipMemcpyHostToDevice));
            S.L = S.Lown.p;
        }
        // D and its transpose (CSR)
        std::vector<int64_t> rp(D_rowptr, D_rowptr + M + 1), trp(M + 1, 0);
        std::vector<int32_t> cl(D_col, D_col + nnz), tcl(nnz);
        std::vector<double> vl(D_val, D_val + nnz), tvl(nnz);
        for (int64_t k = 0; k < nnz; ++k) trp[cl[k] + 1]++;
        for (int64_t i = 0; i < M; ++i) trp[i + 1] += trp[i];
        {
            std::vector<int64_t> fill(trp.begin(), trp.end() - 1);
            for (int64_t i = 0; i < M; ++i)
                for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
                    const int64_t p = fill[cl[k]]++;
                    tcl[p] = (int32_t)i;
                    tvl[p] = vl[k];
                }
        }
        S.drp = upload(rp, c.stream); S.dcol = upload(cl, c.stream); S.dval = upload(vl, c.stream);
        S.dtrp = upload(trp, c.stream); S.dtcol = upload(tcl, c.stream); S.dtval = upload(tvl, c.stream);
        S.nchunk = (rows + TCHUNK - 1) / TCHUNK;
        S.part.alloc((size_t)S.nchunk * M * 8);
        S.dpart.alloc(2 * TvSolver::DOT_BLOCKS * 8);
        S.t_rows.alloc((size_t)rows * 8);
        S.t_M1.alloc((size_t)M * 8);
        S.t_M2.alloc((size_t)M * 8);
        S.gam.alloc((size_t)M * 8);
        std::vector<double> ones(M, 1.0);
        MGRT_HIP(hipMemcpy(S.gam.p, ones.data(), M * 8, hipMemcpyHostToDevice));
        DevBuf dr = upload(std::vector<double>(r, r + rows), c.stream);
        DevBuf b(M * 8), z(M * 8), res(M * 8), p(M * 8), q(M * 8), Dz(M * 8), zp(M * 8), pinv(M * 8);
        S.Ltx(dr.as<double>(), b.as<double>());
        MGRT_HIP(hipMemsetAsync(z.p, 0, M * 8, c.stream));
        const double bnorm = std::sqrt(S.dot(b.as<double>(), b.as<double>()));
        // Jacobi preconditioner: diag(L^T L) + alpha diag(D^T Gamma D)
        DevBuf ltl(M * 8);
        S.colsq(ltl.as<double>());
        // normal matrix when one product with it moves fewer bytes than two passes over L
        // and it fits the free memory
        {
            size_t fr = 0, tot = 0;
            MGRT_HIP(hipMemGetInfo(&fr, &tot));
            const double gbytes = (double)M * M * 8;
            if (gbytes < 2.0 * rows * M * esz && gbytes + (2ull << 30) < (double)fr)
                S.form_normal_matrix();
        }
        std::vector<double> hltl(M), hz(M), hDz(M), hg(M, 1.0), hp(M);
        MGRT_HIP(hipMemcpyAsync(hltl.data(), ltl.p, M * 8, hipMemcpyDeviceToHost, c.stream));
        MGRT_HIP(hipStreamSynchronize(c.stream));
        for (int it = 0; it < iters; ++it) {
            if (it > 0) {
                // Gamma_l from |D z_l|, floored at tau
                hipLaunchKernelGGL(k_spmv, dim3(S.g(M)), dim3(256), 0, c.stream, S.drp.as<int64_t>(),
                                   S.dcol.as<int32_t>(), S.dval.as<double>(), M, z.as<double>(),
                                   (const double *)nullptr, Dz.as<double>());
                MGRT_HIP(hipMemcpyAsync(hDz.data(), Dz.p, M * 8, hipMemcpyDeviceToHost, c.stream));
                MGRT_HIP(hipStreamSynchronize(c.stream));
                double amax = 0;
                for (int64_t i = 0; i < M; ++i) amax = std::max(amax, std::fabs(hDz[i]));
                const double tau = 1e-8 * amax;
                for (int64_t i = 0; i < M; ++i) hg[i] = 1.0 / std::max(std::fabs(hDz[i]), tau);
                MGRT_HIP(hipMemcpy(S.gam.p, hg.data(), M * 8, hipMemcpyHostToDevice));
            }
            for (int64_t j = 0; j < M; ++j) {
                double dd = 0;
                for (int64_t k = trp[j]; k < trp[j + 1]; ++k) dd += hg[tcl[k]] * tvl[k] * tvl[k];
                const double dj = hltl[j] + alpha * dd;
                hp[j] = dj > 0 ? 1.0 / dj : 1.0;
            }
            MGRT_HIP(hipMemcpy(pinv.p, hp.data(), M * 8, hipMemcpyHostToDevice));
            // preconditioned CG on A z = b from the current z
            S.apply(z.as<double>(), q.as<double>());
            hipLaunchKernelGGL(k_axpy, dim3(S.g(M)), dim3(256), 0, c.stream, b.as<double>(), -1.0,
                               q.as<double>(), M, res.as<double>());
            hipLaunchKernelGGL(k_mul, dim3(S.g(M)), dim3(256), 0, c.stream, pinv.as<double>(),
                               res.as<double>(), M, zp.as<double>());
            MGRT_HIP(hipMemcpyAsync(p.p, zp.p, M * 8, hipMemcpyDeviceToDevice, c.stream));
            double rz, rr;
            S.dot2(res.as<double>(), zp.as<double>(), rz, rr);
            int k = 0;
            while (k < cg_maxit && std::sqrt(rr) > cg_rtol * bnorm) {
                S.apply(p.as<double>(), q.as<double>());
                const double pq = S.dot(p.as<double>(), q.as<double>());
                MGRT_REQUIRE(pq > 0 && std::isfinite(pq), MGRT_E_NONFINITE,
                             "normal matrix not positive definite (CG breakdown)");
                const double a = rz / pq;
                hipLaunchKernelGGL(k_axpy, dim3(S.g(M)), dim3(256), 0, c.stream, z.as<double>(), a,
                                   p.as<double>(), M, z.as<double>());
                hipLaunchKernelGGL(k_axpy, dim3(S.g(M)), dim3(256), 0, c.stream, res.as<double>(), -a,
                                   q.as<double>(), M, res.as<double>());
                hipLaunchKernelGGL(k_mul, dim3(S.g(M)), dim3(256), 0, c.stream, pinv.as<double>(),
                                   res.as<double>(), M, zp.as<double>());
                double rz2;
                S.dot2(res.as<double>(), zp.as<double>(), rz2, rr);
                hipLaunchKernelGGL(k_axpy, dim3(S.g(M)), dim3(256), 0, c.stream, zp.as<double>(),
                                   rz2 / rz, p.as<double>(), M, p.as<double>());
                rz = rz2;
                ++k;
            }
            if (cg_iters) cg_iters[it] = k;
            MGRT_HIP(hipMemcpyAsync(hz.data(), z.p, M * 8, hipMemcpyDeviceToHost, c.stream));
            MGRT_HIP(hipStreamSynchronize(c.stream));
            for (int64_t i = 0; i < M; ++i) {
                MGRT_REQUIRE(std::isfinite(hz[i]), MGRT_E_NONFINITE, "non-finite iterate");
                z_out[(int64_t)it * M + i] = hz[i];
            }
        }
        MGRT_HIP(hipGetLastError());
    });
}
