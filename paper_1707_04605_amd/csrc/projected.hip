// Projected data and projected Jacobian rows (Sec. II-F).  The time-weighted inner
// products <a, b>_j = sum_k q_j[k] a_k b_k (quadrature weights q given by the caller)
// reduce every trace's sampled rows to n_proj rows:
//   P[i][j][c] = sum_k q[j][k] u[i][k] J[i n_samples + k][c].
// With J = the Jacobian this is d/dc <u, u0>_j; with J = a trace (one column) it is the
// projected data itself.  One thread per (trace, column): loads of J are coalesced along
// the row, the weights (same for the whole workgroup) are broadcast, sums in FP64.  The
// main kernel reads 16-byte vectors (4 FP32 or 2 FP64 columns per lane), PU of them in
// flight per lane, with the weights staged in LDS in chunks of PCH samples, and splits the
// samples over the 4 waves of a workgroup (wave w takes k = w mod 4), whose partial sums
// are added in a fixed order through LDS; rows whose length or alignment does not allow
// 16-byte loads take the scalar kernel (sample order).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "mgrt_internal.hpp"

namespace mgrt {

namespace {

constexpr int MAX_PROJ = 8;

template <typename T, int NP>
__global__ __launch_bounds__(256) void k_project(const T *__restrict__ J, int64_t ns, int64_t M,
                                                 const double *__restrict__ coef,
                                                 double *__restrict__ P) {
    const int64_t i = blockIdx.y;
    const int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (c >= M) return;
    const T *col = J + i * ns * M + c;
    const double *w = coef + i * NP * ns;
    double acc[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) acc[j] = 0.0;
#pragma unroll 8
    for (int64_t k = 0; k < ns; ++k) {
        const double v = (double)col[k * M];
#pragma unroll
        for (int j = 0; j < NP; ++j) acc[j] += w[j * ns + k] * v;
    }
#pragma unroll
    for (int j = 0; j < NP; ++j) P[(i * NP + j) * M + c] = acc[j];
}

template <typename T> struct Vec16;
typedef float pf4 __attribute__((ext_vector_type(4)));
typedef double pd2 __attribute__((ext_vector_type(2)));
template <> struct Vec16<float> { typedef pf4 type; static constexpr int n = 4; };
template <> struct Vec16<double> { typedef pd2 type; static constexpr int n = 2; };

constexpr int PCH = 512;   // samples per weight chunk staged in LDS
constexpr int PU = 8;      // 16-byte loads in flight per lane

template <typename T, int NP>
__global__ __launch_bounds__(256) void k_project_vec(const T *__restrict__ J, int64_t ns,
                                                     int64_t M, const double *__restrict__ coef,
                                                     double *__restrict__ P) {
    typedef typename Vec16<T>::type V;
    constexpr int VN = Vec16<T>::n;
    __shared__ double sw[NP][PCH];
    __shared__ double sh[4][64 * VN];
    const int64_t i = blockIdx.y;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t c0 = (int64_t)blockIdx.x * 64 * VN + lane * VN;   // first column of this lane
    const bool live = c0 < M;                                         // M % VN == 0
    const V *base = reinterpret_cast<const V *>(J + i * ns * M + (live ? c0 : 0));
    const int64_t vstride = M / VN;
    const double *w = coef + i * NP * ns;
    double acc[NP][VN];
#pragma unroll
    for (int j = 0; j < NP; ++j)
#pragma unroll
        for (int v = 0; v < VN; ++v) acc[j][v] = 0.0;
    for (int64_t k0 = 0; k0 < ns; k0 += PCH) {
        const int64_t nk = ns - k0 < PCH ? ns - k0 : PCH;
        __syncthreads();
        for (int e = threadIdx.x; e < NP * PCH; e += 256) {
            const int j = e / PCH, kk = e % PCH;
            sw[j][kk] = kk < nk ? w[j * ns + k0 + kk] : 0.0;
        }
        __syncthreads();
        if (!live) continue;
        // this wave takes samples kk = wave, wave + 4, ...; PU loads issued before use
        for (int64_t kb = wave; kb < nk; kb += 4 * PU) {
            V x[PU];
#pragma unroll
            for (int u = 0; u < PU; ++u) {
                const int64_t kk = kb + 4 * u;
                x[u] = kk < nk ? __builtin_nontemporal_load(base + (k0 + kk) * vstride) : V{};
            }
#pragma unroll
            for (int u = 0; u < PU; ++u) {
                const int64_t kk = kb + 4 * u;
                if (kk < nk) {
#pragma unroll
                    for (int j = 0; j < NP; ++j) {
                        const double wk = sw[j][kk];
#pragma unroll
                        for (int v = 0; v < VN; ++v) acc[j][v] += wk * (double)x[u][v];
                    }
                }
            }
        }
    }
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        __syncthreads();
#pragma unroll
        for (int v = 0; v < VN; ++v) sh[wave][lane * VN + v] = acc[j][v];
        __syncthreads();
        if (wave == 0 && live) {
#pragma unroll
            for (int v = 0; v < VN; ++v) {
                const int e = lane * VN + v;
                P[(i * NP + j) * M + c0 + v] = ((sh[0][e] + sh[1][e]) + sh[2][e]) + sh[3][e];
            }
        }
    }
}

template <typename T, int NP>
void launch_project(const void *J, int64_t nt, int64_t ns, int64_t M, const double *coef, double *P,
                    hipStream_t s) {
    constexpr int VN = Vec16<T>::n;
    if (M % VN == 0 && reinterpret_cast<uintptr_t>(J) % 16 == 0)
        hipLaunchKernelGGL((k_project_vec<T, NP>), dim3((M + 64 * VN - 1) / (64 * VN), nt), dim3(256), 0,
                           s, static_cast<const T *>(J), ns, M, coef, P);
    else
        hipLaunchKernelGGL((k_project<T, NP>), dim3((M + 255) / 256, nt), dim3(256), 0, s,
                           static_cast<const T *>(J), ns, M, coef, P);
}

template <typename T>
void project_t(const void *J, int np, int64_t nt, int64_t ns, int64_t M, const double *coef,
               double *P, hipStream_t s) {
    switch (np) {
    case 1: launch_project<T, 1>(J, nt, ns, M, coef, P, s); break;
    case 2: launch_project<T, 2>(J, nt, ns, M, coef, P, s); break;
    case 3: launch_project<T, 3>(J, nt, ns, M, coef, P, s); break;
    case 4: launch_project<T, 4>(J, nt, ns, M, coef, P, s); break;
    default: launch_project<T, MAX_PROJ>(J, nt, ns, M, coef, P, s); break;
    }
}

}  // namespace

}  // namespace mgrt

using namespace mgrt;

// Quadrature weights of the two inner products on the sample grid: sample k holds the
// field at t_k = (s_k + 1) dt (trace[l] is the field after step l), rectangle rule with
// widths w_k = t_k - t_{k-1}, t_{-1} = 0, T = n_steps dt:
//   q[0][k] = w_k,  q[1][k] = (t_k / T) w_k.
extern "C" int mgrt_projection_weights(const int64_t *sample_steps, int32_t n_samples, double dt,
                                       int64_t n_steps, double *q) {
    if (!sample_steps || !q || n_samples < 1 || n_steps < 1 || !std::isfinite(dt) || !(dt > 0))
        return MGRT_E_ARG;
    for (int32_t k = 0; k < n_samples; ++k) {
        if (sample_steps[k] < 0 || sample_steps[k] >= n_steps) return MGRT_E_ARG;
        if (k && sample_steps[k] <= sample_steps[k - 1]) return MGRT_E_ARG;
    }
    const double T = (double)n_steps * dt;
    double tprev = 0.0;
    for (int32_t k = 0; k < n_samples; ++k) {
        const double t = ((double)sample_steps[k] + 1.0) * dt;
        const double w = t - tprev;
        q[k] = w;
        q[n_samples + k] = t * w / T;
        tprev = t;
    }
    return MGRT_OK;
}

extern "C" int mgrt_project_rows(mgrt_ctx *ctx, int64_t n_traces, int32_t n_samples, int64_t M,
                                 const void *J, int J_precision, int J_on_device,
                                 const double *u, int32_t n_proj, const double *q, double *P) {
    return mgrt_guarded(ctx, [&](Ctx &c) {
        MGRT_REQUIRE(n_traces >= 1 && n_samples >= 1 && M >= 1 && J && u && q && P, MGRT_E_ARG,
                     "bad sizes or null pointers");
        MGRT_REQUIRE(n_traces <= 65535, MGRT_E_ARG, "at most 65535 traces per call");
        MGRT_REQUIRE(n_proj >= 1 && n_proj <= MAX_PROJ, MGRT_E_ARG, "n_proj must be 1..8");
        MGRT_REQUIRE(J_precision == 32 || J_precision == 64, MGRT_E_ARG, "J precision must be 32 or 64");
        const int64_t ns = n_samples;
        for (int64_t k = 0; k < (int64_t)n_proj * ns; ++k)
            MGRT_REQUIRE(std::isfinite(q[k]), MGRT_E_NONFINITE, "non-finite quadrature weight");
        // coef[i][j][k] = q[j][k] u[i][k], padded to the instantiated projection count
        const int npi = n_proj <= 4 ? n_proj : MAX_PROJ;
        std::vector<double> coef((size_t)n_traces * npi * ns, 0.0);
        for (int64_t i = 0; i < n_traces; ++i)
            for (int64_t k = 0; k < ns; ++k) {
                const double ui = u[i * ns + k];
                MGRT_REQUIRE(std::isfinite(ui), MGRT_E_NONFINITE, "non-finite weighting trace");
                for (int j = 0; j < n_proj; ++j) coef[(i * npi + j) * ns + k] = q[j * ns + k] * ui;
            }
        const size_t esz = J_precision == 32 ? 4 : 8;
        const size_t jbytes = (size_t)n_traces * ns * M * esz;
        DevBuf Jown;
        const void *Jd = J;
        if (!J_on_device) {
            Jown.alloc(jbytes);
            MGRT_HIP(hipMemcpy(Jown.p, J, jbytes, hipMemcpyHostToDevice));
            Jd = Jown.p;
        }
        DevBuf dcoef = upload(coef, c.stream);
        DevBuf dP((size_t)n_traces * npi * M * 8);
        hipEvent_t e0, e1;
        MGRT_HIP(hipEventCreate(&e0));
        MGRT_HIP(hipEventCreate(&e1));
        MGRT_HIP(hipEventRecord(e0, c.stream));
        if (J_precision == 32)
            project_t<float>(Jd, npi, n_traces, ns, M, dcoef.as<double>(), dP.as<double>(), c.stream);
        else
            project_t<double>(Jd, npi, n_traces, ns, M, dcoef.as<double>(), dP.as<double>(), c.stream);
        MGRT_HIP(hipGetLastError());
        MGRT_HIP(hipEventRecord(e1, c.stream));
        MGRT_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        MGRT_HIP(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        c.timing = mgrt_timing{};
        c.timing.call_ms = ms;
        c.timing.step_ms_total = 0;
        std::vector<double> h((size_t)n_traces * npi * M);
        MGRT_HIP(hipMemcpy(h.data(), dP.p, h.size() * 8, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n_traces; ++i)
            for (int j = 0; j < n_proj; ++j)
                std::copy(h.begin() + (i * npi + j) * M, h.begin() + (i * npi + j + 1) * M,
                          P + (i * n_proj + j) * M);
    });
}
