// Jacobian of sampled traces w.r.t. the coarse permittivity coordinates (Sec. II-B,
// eqs. approx_1 / approx_2; App. A-1 auxiliary source, App. A-3 multigrid source).
//
// A permittivity perturbation dEps changes only the lumped mass: dM.  Differentiating
// the leap-frog recurrence gives the auxiliary (tangent) system -- the same recurrence
// with the load h_l = dM (.) b_l, b_l = -(p_{l+1} - p_l)/dt (the exact form of the
// auxiliary source of App. A-1).
//
// MG mode (eq. approx_2): dM for coarse column j is |T'_j|/(d+1) at each of the d+1
// coarse vertices (the coarse mass derivative, lumped).  The trace response at receiver
// r to a unit load at node i applied at step m is G_{r,i}(l - m); the transition
// operators of the scheme are symmetric, so G_{r,i}(k) is also the response at node i
// to a unit load at the receiver stencil at step 0 (reciprocity).  Hence
//   J2[(s,r,k), j] = |T'_j|/(d+1) sum_{v in vert(T'_j)} sum_{m<=l_k} lambda_{r,v}(l_k - m) b_{s,v}(m)
// with b_s recorded at the coarse nodes in one batched forward run per source batch and
// lambda_r (= p_{k+1} at the coarse nodes of an impulse run from receiver r) in one
// batched impulse run per receiver batch.  The lagged sums run in k_corr, FP64
// accumulation; k_restrict forms the columns.
//
// EXACT mode (eq. approx_1): for each listed column j, dM_i = W_ij = sum of |T|/(d+1)
// over the fine elements T of T'_j that contain node i; the tangent system is stepped
// directly for every (source, column) pair with the recorded b_s as its load.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "mgrt_internal.hpp"
#include "series_filter.hpp"

namespace mgrt {

namespace {

// A second stream, with events, for work that overlaps the stepping stream (default
// priority, non-blocking); it is joined and released when it goes out of scope, also while
// an exception unwinds, so buffers declared before it outlive its work.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    SideStream() {
        try {
            MGRT_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
            for (auto &e : ev) MGRT_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        } catch (...) {
            release();
            throw;
        }
    }
    ~SideStream() { release(); }
    SideStream(const SideStream &) = delete;
    SideStream &operator=(const SideStream &) = delete;
    void release() {
        if (s) (void)hipStreamSynchronize(s);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
        if (s) (void)hipStreamDestroy(s);
        s = nullptr;
        for (auto &e : ev) e = nullptr;
    }
};

constexpr int CORR_R = 4;     // outputs per thread per pass (256 * 4 sample steps per pass)
constexpr int CORR_CH = 512;  // impulse-response samples staged in LDS per chunk

// C[(pair)*K + k][c] = sum_{u=0}^{l_k} lam[c][q][u] * b[c][fcol][l_k - u]
// One workgroup per (coarse node, receiver column).  The forward velocity series b sits
// in LDS for the whole kernel (in its own precision); the impulse response lam streams
// through LDS two chunks at a time, widened to FP64 as it is staged, and is read with the
// same address by every lane.  Output k of a thread reads b backwards from l_k, so the
// inner loop is two LDS reads, one conversion (none for FP64 fields) and one FP64 FMA,
// branch-free.  Outputs are dealt folded (k and 511 - k style) so every wave gets short
// and long sums.  The workgroup's two halves (256 threads each, the same outputs) take
// the even and the odd chunks, which doubles the waves that hide LDS latency at the same
// LDS footprint; their sums are added in a fixed order (even half + odd half) at the end.
template <typename T>
__global__ __launch_bounds__(512) void k_corr(const T *__restrict__ bh, const T *__restrict__ lh,
                                              int64_t N, int64_t Bf, int64_t Bi, int64_t nc,
                                              const int32_t *__restrict__ fcol_of,
                                              const int32_t *__restrict__ pair_of,
                                              const int64_t *__restrict__ lk, int K,
                                              double *__restrict__ C) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *bl = reinterpret_cast<T *>(smem_raw);
    double *ls2 = reinterpret_cast<double *>(bl + ((N + 3) & ~(int64_t)3));   // 2 chunks
    __shared__ double odd[CORR_R][256];
    const int64_t c = blockIdx.x;
    const int q = blockIdx.y;
    const int fcol = fcol_of[q];
    if (fcol < 0) return;
    const T *bser = bh + (c * Bf + fcol) * N;
    const T *lser = lh + (c * Bi + q) * N;
    for (int64_t t = threadIdx.x; t < N; t += 512) bl[t] = bser[t];
    const int64_t pair = pair_of[q];
    const int half = threadIdx.x >> 8;
    const int tid = threadIdx.x & 255;
    const double *ls = ls2 + half * CORR_CH;
    for (int k0 = 0; k0 < K; k0 += 256 * CORR_R) {
        int64_t lr[CORR_R];
        int kr[CORR_R];
        double acc[CORR_R];
#pragma unroll
        for (int r = 0; r < CORR_R; ++r) {
            const int k = k0 + r * 256 + ((r & 1) ? 255 - tid : tid);
            kr[r] = k;
            lr[r] = k < K ? lk[k] : -1;
            acc[r] = 0.0;
        }
        const int64_t umax = lk[std::min(K, k0 + 256 * CORR_R) - 1];
        for (int64_t u2 = 0; u2 <= umax; u2 += 2 * CORR_CH) {
            __syncthreads();   // previous chunks consumed (and b staged, first time)
            for (int t = threadIdx.x; t < 2 * CORR_CH; t += 512)
                ls2[t] = u2 + t < N ? (double)lser[u2 + t] : 0.0;
            __syncthreads();
            const int64_t u0 = u2 + half * CORR_CH;
#pragma unroll
            for (int r = 0; r < CORR_R; ++r) {
                const int64_t l = lr[r];
                if (l < u0) continue;
                const int ue = (int)std::min<int64_t>(CORR_CH, l - u0 + 1);
                const T *bp = bl + (l - u0);            // b[l - u0 - j] = bp[-j]
                double a = acc[r];
                int j = 0;
                for (; j + 8 <= ue; j += 8) {
#pragma unroll
                    for (int e = 0; e < 8; ++e) a = fma(ls[j + e], (double)bp[-(j + e)], a);
                }
                for (; j < ue; ++j) a = fma(ls[j], (double)bp[-j], a);
                acc[r] = a;
            }
        }
        __syncthreads();
        if (half == 1) {
#pragma unroll
            for (int r = 0; r < CORR_R; ++r) odd[r][tid] = acc[r];
        }
        __syncthreads();
        if (half == 0) {
#pragma unroll
            for (int r = 0; r < CORR_R; ++r)
                if (kr[r] < K) C[(pair * K + kr[r]) * nc + c] = acc[r] + odd[r][tid];
        }
    }
}

// J[row][j] = cvol_j/(d+1) * sum_a C[row][cvi(j,a)]
__global__ __launch_bounds__(256) void k_restrict(const double *__restrict__ C, int64_t nc,
                                                  const int32_t *__restrict__ cvi,
                                                  const double *__restrict__ cvol, int V,
                                                  int64_t M, double *__restrict__ J) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t row = blockIdx.y;
    if (j >= M) return;
    double s = 0.0;
    for (int a = 0; a < V; ++a) s += C[row * nc + cvi[j * V + a]];
    J[row * M + j] = s * cvol[j] / V;
}

// series[e][l] = (b[e][l] - b[e][l-1]) / dt from histories hist[e][l] (b[-1] = 0)
template <typename T>
__global__ void k_diff_series(const T *__restrict__ hist, int64_t E, int64_t N, double inv_dt,
                              double *__restrict__ out) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= E * N) return;
    const int64_t l = idx % N;
    const double cur = (double)hist[idx];
    const double prev = l > 0 ? (double)hist[idx - 1] : 0.0;
    out[idx] = (cur - prev) * inv_dt;
}

size_t free_bytes(const mgrt_run_opts *o) {
    size_t fr = 0, tot = 0;
    MGRT_HIP(hipMemGetInfo(&fr, &tot));
    size_t cap = fr > (size_t)(2ull << 30) ? fr - (size_t)(2ull << 30) : fr / 2;   // keep 2 GiB
    if (o && o->mem_budget_gb > 0) cap = std::min(cap, (size_t)(o->mem_budget_gb * (1ull << 30)));
    return cap;
}

std::vector<Record> receiver_taps(const Acquisition &aq, int64_t s, int col, int V, int dst0) {
    std::vector<Record> rec;
    for (int r = 0; r < aq.n_rec; ++r) {
        const Stencil &rs = aq.rec[s * aq.n_rec + r];
        for (int a = 0; a < V; ++a) rec.push_back(Record{rs.node[a], col, dst0 + r * V + a, rs.w[a]});
    }
    return rec;
}

// Exact split of the source function between the two runs of the reciprocity pairing.
// J2 = lambda * b with b = beta * w (beta: the velocity response to a unit load at the
// source, w the wavelet) and * causal convolution over steps, so J2 = (lambda * w1) *
// (beta * w2) for any causal w1, w2 with w1 * w2 = w.  The impulse response lambda carries
// the scheme's whole spectrum up to the grid scale, and paired with it the FP32 rounding
// noise of b, which is broadband, is amplified by the ratio of lambda's total to its
// in-band content; splitting w leaves both runs band-limited.  Here
//   w1 = ((1 - rho) / (1 - rho z^-1))^2 delta    (two first-order low-pass stages),
//   w2 = ((1 - rho z^-1) / (1 - rho))^2 w         (their FIR inverse applied to w),
// rho = exp(-omega_c dt), omega_c = 3 times the wavelet's RMS angular frequency
// sqrt(sum ((w_l - w_{l-1})/dt)^2 / sum w_l^2), so omega_c dt comes from the samples alone.  Each first-order stage is evaluated as
// (w_l - w_{l-1})/(1 - rho) + w_{l-1}, which keeps the cancellation of the difference out
// of the small divisor.  The split is exact for any omega_c; unless forced it is skipped
// (returns false) when omega_c dt > 0.5, where the wavelet itself already reaches the
// grid scale and nothing is gained, and forced splits clamp omega_c dt to 2.  An all-zero
// wavelet is never split.  h2 (optional) receives w1^-1 * w2, the filter that turns the
// response to w1 into the response to w2.
bool split_wavelet(const std::vector<double> &w, bool forced, std::vector<double> &w1,
                   std::vector<double> &w2, std::vector<double> *h2 = nullptr) {
    const int64_t N = (int64_t)w.size();
    double e0 = 0, e1 = 0, prev = 0;
    for (int64_t l = 0; l < N; ++l) {
        e0 += w[l] * w[l];
        e1 += (w[l] - prev) * (w[l] - prev);
        prev = w[l];
    }
    if (!(e0 > 0)) return false;
    double wc_dt = 3.0 * std::sqrt(e1 / e0);         // omega_c * dt
    if (!(wc_dt > 0)) return false;
    if (wc_dt > 0.5) {
        if (!forced) return false;
        wc_dt = std::min(wc_dt, 2.0);
    }
    const double rho = std::exp(-wc_dt), omr = -std::expm1(-wc_dt);   // 1 - rho
    w1.assign(N, 0.0);
    double rn = 1.0;                                  // rho^l
    for (int64_t l = 0; l < N; ++l) {
        w1[l] = omr * omr * (double)(l + 1) * rn;
        rn *= rho;
    }
    auto stage = [&](const std::vector<double> &x) {
        std::vector<double> y(N);
        double xp = 0.0;
        for (int64_t l = 0; l < N; ++l) {
            y[l] = (x[l] - xp) / omr + xp;
            xp = x[l];
        }
        return y;
    };
    w2 = stage(stage(w));
    // w1^-1 = ((1 - rho z^-1) / (1 - rho))^2 is the FIR of the two stages, so w1^-1 * w2
    // is w through all four of them
    if (h2) *h2 = stage(stage(w2));
    return true;
}

// MG mode (eq. approx_2 through discrete reciprocity).  With deconv, the receiver runs
// carry the source function itself and their records are Tikhonov-deconvolved by it
// before the correlation (the paper's route of App. A-2, delta relative to max |F|^2).
// With split, the source runs carry w2 and the receiver runs w1 (split_wavelet); with
// split and monostatic pairs one run with w1 serves both (the one-run pairing below).
template <typename T>
void jacobian_mg(Ctx &c, const Acquisition &aq, const std::vector<double> &g,
                 const std::vector<double> &wav, double dt, int64_t N,
                 const std::vector<int64_t> &ss, const mgrt_run_opts *opts, double *J_out,
                 bool dev_out, bool deconv, double delta, bool split) {
    const HostMesh &hm = c.hm;
    const int prec = sizeof(T) == 4 ? 32 : 64;
    const int flags = opts ? opts->flags : 0;
    const int V = hm.d + 1;
    const int64_t n = hm.n, nc_nodes = (int64_t)hm.cnodes.size(), M = hm.nc;
    const int K = (int)ss.size();
    const int64_t n_pairs = aq.n_src * aq.n_rec;
    const int64_t rows = n_pairs * K;
    const size_t esz = sizeof(T);
    const size_t lds = (size_t)((N + 3) & ~(int64_t)3) * esz + (size_t)2 * CORR_CH * sizeof(double);
    MGRT_REQUIRE(lds <= 150 * 1024, MGRT_E_OOM_PLAN,
                 "trace length too long for the correlation kernel's LDS staging");

    std::vector<double> w1, w2, h2;
    const bool did_split = split && split_wavelet(wav, (flags & MGRT_F_JAC_SPLIT) != 0, w1, w2, &h2);
    // One run per monostatic pair: when every source has one receiver at its own point
    // (the same P1 stencil), the receiver's impulse run and the source run see the same
    // Green's function G of that point.  The scheme is linear and time invariant from zero
    // state, so the run with w1 records both lambda * w1 = G * w1 (its field) and, after
    // the filter h2 = w1^-1 * w2 (FFT, FP64), beta * w2 (its velocity convolved with h2).
    bool mono = did_split && !deconv && aq.n_rec == 1 && !(flags & MGRT_F_JAC_PAIRED);
    for (int64_t s = 0; s < aq.n_src && mono; ++s)
        for (int a = 0; a < V; ++a)
            mono = mono && aq.src[s].node[a] == aq.rec[s].node[a] && aq.src[s].w[a] == aq.rec[s].w[a];
    c.timing.jac_runs = mono ? 1 : 2;

    // memory plan: histories for Bf sources and Bi receivers, correlations, J
    int Bf = pick_batch(c, prec, aq.n_src, opts ? opts->batch : 0, dt, flags);
    const size_t fixed = (size_t)n_pairs * K * nc_nodes * 8 + (size_t)rows * M * 8;
    const size_t cap = free_bytes(opts);
    // (de)convolution scratch: padded rows of 2 (L/2 + 1) reals (FP64 for the one-run
    // filter), chunked to at most 128 MiB (at least one row), so that a chunk stays in the
    // 256 MB Infinity Cache between the transforms' passes (C3's one-run filter: 128 MiB
    // chunks 2.58 s per Jacobian, 1 GiB 2.62 s, 32 MiB 2.58 s with more launches)
    int64_t Lfft = 1;
    while (Lfft < 2 * N) Lfft *= 2;
    const size_t dscratch = deconv || mono ? std::max<size_t>((size_t)(Lfft + 2) * 8, (size_t)128 << 20) : 0;
    auto need = [&](int bf, int bi) {
        return fixed + (size_t)nc_nodes * N * esz * (bf + bi) + (size_t)n * esz * 2 * std::max(bf, bi) +
               dscratch;
    };
    int Bi = mono ? Bf : pick_batch(c, prec, std::min<int64_t>(n_pairs, (int64_t)Bf * aq.n_rec), 0, dt, flags);
    while (need(Bf, Bi) > cap && (Bf > 1 || Bi > 1)) {
        if (mono) Bi = Bf = Bf == 4 && prec == 32 ? 1 : Bf / 2;
        else if (Bi >= Bf && Bi > 1) Bi = Bi == 4 && prec == 32 ? 1 : Bi / 2;
        else Bf = Bf == 4 && prec == 32 ? 1 : Bf / 2;
    }
    MGRT_REQUIRE(need(Bf, Bi) <= cap, MGRT_E_OOM_PLAN, "Jacobian histories do not fit device memory");

    // the one-run pairing overlaps batch b's filter and sums with the stepping of batch
    // b + 1; a second set of histories (when it fits) lets the run of b + 1 start at once
    const int64_t n_batches = (aq.n_src + Bf - 1) / Bf;
    const size_t set_bytes = (size_t)nc_nodes * N * esz * 2 * Bf;
    const int nsets = mono && n_batches > 1 && need(Bf, Bi) + set_bytes <= cap ? 2 : 1;
    c.timing.jac_sets = mono ? nsets : 0;

    DevBuf Cbuf((size_t)n_pairs * K * nc_nodes * 8);
    DevBuf Jdev((size_t)rows * M * 8);
    DevBuf bh((size_t)nc_nodes * Bf * N * esz), lh((size_t)nc_nodes * Bi * N * esz);
    DevBuf bh2, lh2;
    if (nsets == 2) {
        bh2.alloc((size_t)nc_nodes * Bf * N * esz);
        lh2.alloc((size_t)nc_nodes * Bf * N * esz);
    }
    DevBuf stA((size_t)n * std::max(Bf, Bi) * esz), stB((size_t)n * std::max(Bf, Bi) * esz);
    DevBuf dss = upload(ss, c.stream);
    std::vector<double> imp(N, 0.0);   // unit load at step 0 in load-difference form
    imp[0] = 1.0 / dt;
    if (N > 1) imp[1] = -1.0 / dt;
    if (did_split) imp = load_series(w1.data(), N, dt);
    c.timing.jac_split = did_split ? 1 : 0;
    DevBuf series = upload(did_split ? load_series(w2.data(), N, dt) : g, c.stream);
    DevBuf impulse = upload(imp, c.stream);
    std::vector<int64_t> hist_nodes(hm.cnodes.begin(), hm.cnodes.end());

    StepOp &opf = get_step_op(c, tile_nodes(prec, Bf), prec, dt);
    MGRT_HIP(hipFuncSetAttribute((const void *)k_corr<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    if (mono) {
        // One run per source batch with w1 at the source points: the field to lh, the
        // velocity to bh.  The filter h2 of bh and the lagged sums go to a second stream;
        // the run of batch b + nsets waits only for the sums of batch b (its set).
        SeriesFilter filt(c, prec, nc_nodes * Bf, N, h2, dscratch);
        std::vector<int32_t> fcol((size_t)n_batches * Bf, -1), pair((size_t)n_batches * Bf, 0);
        for (int64_t s = 0; s < aq.n_src; ++s) {
            fcol[s] = (int32_t)(s % Bf);
            pair[s] = (int32_t)s;
        }
        DevBuf dfcol = upload(fcol, c.stream), dpair = upload(pair, c.stream);
        T *bset[2] = {bh.as<T>(), bh2.as<T>()}, *lset[2] = {lh.as<T>(), lh2.as<T>()};
        SideStream side;   // after the buffers: joined before any of them is freed
        for (int64_t bi = 0; bi < n_batches; ++bi) {
            const int64_t s0 = bi * Bf;
            const int nb = (int)std::min<int64_t>(Bf, aq.n_src - s0);
            const int set = (int)(bi % nsets);
            if (bi >= nsets) MGRT_HIP(hipStreamWaitEvent(c.stream, side.ev[set], 0));
            BatchRun mr;
            mr.prec = prec; mr.B = Bf; mr.flags = flags; mr.launch = opts ? opts->launch : 0; mr.n_steps = N;
            mr.d_series = impulse.as<double>(); mr.series_len = N;
            for (int b = 0; b < nb; ++b) {
                const Stencil &st = aq.src[s0 + b];
                for (int a = 0; a < V; ++a)
                    mr.inj.push_back(Injection{st.node[a], b, 0, opf.gamma[st.node[a]] * st.w[a]});
            }
            mr.hist = true; mr.hist_mode = 2; mr.d_hist = lset[set]; mr.d_hist2 = bset[set]; mr.hist_len = N;
            mr.hist_nodes = hist_nodes;
            MGRT_HIP(hipMemsetAsync(stA.p, 0, (size_t)n * Bf * esz, c.stream));
            MGRT_HIP(hipMemsetAsync(stB.p, 0, (size_t)n * Bf * esz, c.stream));
            mr.d_p = stA.p; mr.d_pm = stB.p;
            run_batch(c, opf, mr);
            MGRT_HIP(hipEventRecord(side.ev[2], c.stream));
            MGRT_HIP(hipStreamWaitEvent(side.s, side.ev[2], 0));
            filt.enqueue(bset[set], side.s);
            hipLaunchKernelGGL(k_corr<T>, dim3(nc_nodes, Bf), dim3(512), lds, side.s, bset[set], lset[set], N,
                               (int64_t)Bf, (int64_t)Bf, nc_nodes, dfcol.as<int32_t>() + s0,
                               dpair.as<int32_t>() + s0, dss.as<int64_t>(), K, Cbuf.as<double>());
            MGRT_HIP(hipGetLastError());
            MGRT_HIP(hipEventRecord(side.ev[set], side.s));
        }
        MGRT_HIP(hipStreamSynchronize(side.s));
    }
    for (int64_t s0 = 0; s0 < aq.n_src && !mono; s0 += Bf) {
        const int nb = (int)std::min<int64_t>(Bf, aq.n_src - s0);
        // forward: b_s at the coarse nodes
        BatchRun fr;
        fr.prec = prec; fr.B = Bf; fr.flags = flags; fr.launch = opts ? opts->launch : 0; fr.n_steps = N;
        fr.d_series = series.as<double>(); fr.series_len = N;
        for (int b = 0; b < nb; ++b) {
            const Stencil &st = aq.src[s0 + b];
            for (int a = 0; a < V; ++a)
                fr.inj.push_back(Injection{st.node[a], b, 0, opf.gamma[st.node[a]] * st.w[a]});
        }
        fr.hist = true; fr.hist_mode = 1; fr.d_hist = bh.p; fr.hist_len = N;
        fr.hist_nodes = hist_nodes;
        MGRT_HIP(hipMemsetAsync(stA.p, 0, (size_t)n * Bf * esz, c.stream));
        MGRT_HIP(hipMemsetAsync(stB.p, 0, (size_t)n * Bf * esz, c.stream));
        fr.d_p = stA.p; fr.d_pm = stB.p;
        run_batch(c, opf, fr);

        // impulse runs from the receivers of this source batch
        const int64_t P = (int64_t)nb * aq.n_rec;
        StepOp &opi = get_step_op(c, tile_nodes(prec, Bi), prec, dt);
        for (int64_t q0 = 0; q0 < P; q0 += Bi) {
            const int nq = (int)std::min<int64_t>(Bi, P - q0);
            BatchRun ir;
            ir.prec = prec; ir.B = Bi; ir.flags = flags; ir.launch = opts ? opts->launch : 0; ir.n_steps = N;
            ir.d_series = deconv ? series.as<double>() : impulse.as<double>(); ir.series_len = N;
            std::vector<int32_t> fcol(Bi, -1), pair(Bi, 0);
            for (int q = 0; q < nq; ++q) {
                const int64_t pl = q0 + q;            // local pair: b * n_rec + r
                const int b = (int)(pl / aq.n_rec);
                const int r = (int)(pl % aq.n_rec);
                const Stencil &rs = aq.rec[(s0 + b) * aq.n_rec + r];
                for (int a = 0; a < V; ++a)
                    ir.inj.push_back(Injection{rs.node[a], q, 0, opi.gamma[rs.node[a]] * rs.w[a]});
                fcol[q] = b;
                pair[q] = (int32_t)((s0 + b) * aq.n_rec + r);
            }
            ir.hist = true; ir.hist_mode = 0; ir.d_hist = lh.p; ir.hist_len = N;
            ir.hist_nodes = hist_nodes;
            MGRT_HIP(hipMemsetAsync(stA.p, 0, (size_t)n * Bi * esz, c.stream));
            MGRT_HIP(hipMemsetAsync(stB.p, 0, (size_t)n * Bi * esz, c.stream));
            ir.d_p = stA.p; ir.d_pm = stB.p;
            run_batch(c, opi, ir);
            if (deconv) deconvolve_series(c, lh.p, prec, nc_nodes * Bi, N, wav, delta, dscratch);
            DevBuf dfcol = upload(fcol, c.stream), dpair = upload(pair, c.stream);
            hipLaunchKernelGGL(k_corr<T>, dim3(nc_nodes, Bi), dim3(512), lds, c.stream,
                               bh.as<T>(), lh.as<T>(), N, (int64_t)Bf, (int64_t)Bi, nc_nodes,
                               dfcol.as<int32_t>(), dpair.as<int32_t>(), dss.as<int64_t>(), K,
                               Cbuf.as<double>());
            MGRT_HIP(hipGetLastError());
            MGRT_HIP(hipStreamSynchronize(c.stream));
        }
    }
    const int64_t gx = (M + 255) / 256;
    for (int64_t r0 = 0; r0 < rows; r0 += 65535) {
        const int64_t nr = std::min<int64_t>(65535, rows - r0);
        hipLaunchKernelGGL(k_restrict, dim3(gx, nr), dim3(256), 0, c.stream,
                           Cbuf.as<double>() + r0 * nc_nodes, nc_nodes, c.dm.cvert_idx.as<int32_t>(),
                           c.dm.cvol.as<double>(), V, M, Jdev.as<double>() + r0 * M);
    }
    MGRT_HIP(hipGetLastError());
    MGRT_HIP(hipStreamSynchronize(c.stream));
    MGRT_HIP(hipMemcpy(J_out, Jdev.p, (size_t)rows * M * 8,
                       dev_out ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost));
    c.timing.batch = Bf;
}

// EXACT mode: tangent-linear runs, one column per (source, listed coarse column).
template <typename T>
void jacobian_exact(Ctx &c, const Acquisition &aq, const std::vector<double> &g, double dt,
                    int64_t N, const std::vector<int64_t> &ss, const std::vector<int64_t> &cols,
                    const mgrt_run_opts *opts, double *J_out, bool dev_out) {
    const HostMesh &hm = c.hm;
    const int prec = sizeof(T) == 4 ? 32 : 64;
    const int flags = opts ? opts->flags : 0;
    const int V = hm.d + 1;
    const int64_t n = hm.n;
    const int K = (int)ss.size();
    const int64_t ncol = (int64_t)cols.size();
    const int64_t rows = aq.n_src * aq.n_rec * K;
    const size_t esz = sizeof(T);

    // W_ij per listed column: (node, weight) lists
    std::vector<std::vector<std::pair<int64_t, double>>> wcol(ncol);
    std::vector<int64_t> support;
    for (int64_t q = 0; q < ncol; ++q) {
        const int64_t j = cols[q];
        std::vector<std::pair<int64_t, double>> ent;
        for (int64_t k = hm.c2f_ptr[j]; k < hm.c2f_ptr[j + 1]; ++k) {
            const int64_t t = hm.c2f_idx[k];
            for (int a = 0; a < V; ++a) ent.emplace_back(hm.elems[t * V + a], hm.vol[t] / V);
        }
        std::sort(ent.begin(), ent.end());
        for (size_t e = 0; e < ent.size();) {
            const int64_t i = ent[e].first;
            double s = 0;
            while (e < ent.size() && ent[e].first == i) s += ent[e++].second;
            wcol[q].emplace_back(i, s);
            support.push_back(i);
        }
    }
    std::sort(support.begin(), support.end());
    support.erase(std::unique(support.begin(), support.end()), support.end());
    const int64_t ns = (int64_t)support.size();
    auto sidx = [&](int64_t i) {
        return (int64_t)(std::lower_bound(support.begin(), support.end(), i) - support.begin());
    };

    // tangent columns: (source s, listed column q) pairs in batches of Bt; the sources of a
    // batch are stepped forward first, recording b at the support nodes.
    const int64_t n_tl = aq.n_src * ncol;
    const int Bt = choose_batch(prec, n_tl, opts ? opts->batch : 0);
    const int64_t src_per = std::max<int64_t>(1, Bt / std::max<int64_t>(1, ncol));
    const int Bf = choose_batch(prec, std::min<int64_t>(aq.n_src, src_per), 0);
    std::vector<double> Jh((size_t)rows * ncol, 0.0);
    DevBuf series = upload(g, c.stream);
    DevBuf stA((size_t)n * std::max(Bt, Bf) * esz), stB((size_t)n * std::max(Bt, Bf) * esz);
    DevBuf bh((size_t)ns * Bf * N * esz);
    DevBuf bser((size_t)ns * Bf * N * 8);
    const int64_t n_parts = (int64_t)Bt * aq.n_rec * V;
    DevBuf parts((size_t)N * n_parts * 8);
    std::vector<double> hp((size_t)N * n_parts);
    StepOp &opf = get_step_op(c, tile_nodes(prec, Bf), prec, dt);
    StepOp &opt = get_step_op(c, tile_nodes(prec, Bt), prec, dt);

    // the tangent columns of one source batch are (s in batch) x (all listed columns)
    for (int64_t s0 = 0; s0 < aq.n_src; s0 += Bf) {
        const int nb = (int)std::min<int64_t>(Bf, aq.n_src - s0);
        BatchRun fr;
        fr.prec = prec; fr.B = Bf; fr.flags = flags; fr.launch = opts ? opts->launch : 0; fr.n_steps = N;
        fr.d_series = series.as<double>(); fr.series_len = N;
        for (int b = 0; b < nb; ++b) {
            const Stencil &st = aq.src[s0 + b];
            for (int a = 0; a < V; ++a)
                fr.inj.push_back(Injection{st.node[a], b, 0, opf.gamma[st.node[a]] * st.w[a]});
        }
        fr.hist = true; fr.hist_mode = 1; fr.d_hist = bh.p; fr.hist_len = N;
        fr.hist_nodes = support;
        MGRT_HIP(hipMemsetAsync(stA.p, 0, (size_t)n * Bf * esz, c.stream));
        MGRT_HIP(hipMemsetAsync(stB.p, 0, (size_t)n * Bf * esz, c.stream));
        fr.d_p = stA.p; fr.d_pm = stB.p;
        run_batch(c, opf, fr);
        // load series of the tangent system: (h_l - h_{l-1})/dt per unit weight
        const int64_t E = ns * Bf;
        hipLaunchKernelGGL(k_diff_series<T>, dim3((E * N + 255) / 256), dim3(256), 0, c.stream,
                           bh.as<T>(), E, N, 1.0 / dt, bser.as<double>());
        MGRT_HIP(hipGetLastError());
        MGRT_HIP(hipStreamSynchronize(c.stream));

        const int64_t T_here = (int64_t)nb * ncol;
        for (int64_t t0 = 0; t0 < T_here; t0 += Bt) {
            const int nt = (int)std::min<int64_t>(Bt, T_here - t0);
            BatchRun tr;
            tr.prec = prec; tr.B = Bt; tr.flags = flags; tr.launch = opts ? opts->launch : 0; tr.n_steps = N;
            tr.d_series = bser.as<double>(); tr.series_len = N;
            for (int q = 0; q < nt; ++q) {
                const int64_t tl = t0 + q;
                const int b = (int)(tl / ncol);
                const int64_t cq = tl % ncol;
                for (const auto &iw : wcol[cq]) {
                    const int64_t si = sidx(iw.first);
                    tr.inj.push_back(Injection{iw.first, q, (int32_t)(si * Bf + b),
                                               opt.gamma[iw.first] * iw.second});
                }
                auto taps = receiver_taps(aq, s0 + b, q, V, q * aq.n_rec * V);
                tr.rec.insert(tr.rec.end(), taps.begin(), taps.end());
            }
            tr.d_parts = parts.as<double>(); tr.n_parts = n_parts;
            MGRT_HIP(hipMemsetAsync(stA.p, 0, (size_t)n * Bt * esz, c.stream));
            MGRT_HIP(hipMemsetAsync(stB.p, 0, (size_t)n * Bt * esz, c.stream));
            tr.d_p = stA.p; tr.d_pm = stB.p;
            run_batch(c, opt, tr);
            MGRT_HIP(hipMemcpy(hp.data(), parts.p, hp.size() * 8, hipMemcpyDeviceToHost));
            for (int q = 0; q < nt; ++q) {
                const int64_t tl = t0 + q;
                const int64_t s = s0 + tl / ncol;
                const int64_t cq = tl % ncol;
                for (int r = 0; r < aq.n_rec; ++r)
                    for (int k = 0; k < K; ++k) {
                        double v = 0;
                        for (int a = 0; a < V; ++a) v += hp[ss[k] * n_parts + (q * aq.n_rec + r) * V + a];
                        Jh[((s * aq.n_rec + r) * K + k) * ncol + cq] = v;
                    }
            }
        }
    }
    if (dev_out) MGRT_HIP(hipMemcpy(J_out, Jh.data(), Jh.size() * 8, hipMemcpyHostToDevice));
    else std::memcpy(J_out, Jh.data(), Jh.size() * 8);
    c.timing.batch = Bt;
}

}  // namespace

}  // namespace mgrt

using namespace mgrt;

extern "C" int mgrt_jacobian_coarse(mgrt_ctx *ctx, int64_t n_src, const double *src_xyz,
                                    int32_t n_rec, const double *rec_xyz, const double *wavelet,
                                    double dt, int64_t n_steps, int32_t n_samples,
                                    const int64_t *sample_steps, int mode, int64_t n_cols,
                                    const int64_t *cols, const mgrt_run_opts *opts, double *J) {
    return mgrt_guarded(ctx, [&](Ctx &c) {
        MGRT_REQUIRE(J && sample_steps, MGRT_E_ARG, "null output or sample steps");
        MGRT_REQUIRE(n_steps >= 1 && n_samples >= 1, MGRT_E_ARG, "need n_steps, n_samples >= 1");
        MGRT_REQUIRE(c.hm.nc > 0, MGRT_E_STATE, "mesh was uploaded without a coarse level");
        std::vector<int64_t> ss(sample_steps, sample_steps + n_samples);
        for (int k = 0; k < n_samples; ++k) {
            MGRT_REQUIRE(ss[k] >= 0 && ss[k] < n_steps, MGRT_E_ARG, "sample step out of range");
            if (k) MGRT_REQUIRE(ss[k] > ss[k - 1], MGRT_E_ARG, "sample steps must increase");
        }
        const int flags = opts ? opts->flags : 0;
        const int prec = run_precision(opts);
        Acquisition aq = make_acquisition(c, n_src, src_xyz, n_rec, rec_xyz);
        check_stability(c, dt, flags);
        std::vector<double> g = load_series(wavelet, n_steps, dt);
        const std::vector<double> wav(wavelet, wavelet + n_steps);
        c.timing = mgrt_timing{};
        c.timing.nodes = c.hm.n;
        c.timing.precision = prec;
        auto t0 = std::chrono::steady_clock::now();
        const bool dev_out = (flags & MGRT_F_DEVICE_OUT) != 0;
        if (mode == MGRT_JAC_MG || mode == MGRT_JAC_DECONV) {
            MGRT_REQUIRE(cols == nullptr && n_cols == 0, MGRT_E_ARG, "MG modes return all columns");
            const bool dc = mode == MGRT_JAC_DECONV;
            const double delta = opts ? opts->deconv_delta : 0.0;
            MGRT_REQUIRE(!dc || (std::isfinite(delta) && delta >= 0), MGRT_E_ARG,
                         "deconv_delta must be finite and >= 0");
            // exact wavelet split: by default for FP32 fields in MG mode, forced either way
            // by the flags
            MGRT_REQUIRE(!((flags & MGRT_F_JAC_SPLIT) && (flags & MGRT_F_JAC_DIRECT)), MGRT_E_ARG,
                         "MGRT_F_JAC_SPLIT and MGRT_F_JAC_DIRECT exclude each other");
            MGRT_REQUIRE(!(dc && (flags & MGRT_F_JAC_SPLIT)), MGRT_E_ARG,
                         "the deconvolution route pairs the physical runs (no split)");
            const bool split = !dc && ((flags & MGRT_F_JAC_SPLIT) ||
                                       (prec == 32 && !(flags & MGRT_F_JAC_DIRECT)));
            if (prec == 32) jacobian_mg<float>(c, aq, g, wav, dt, n_steps, ss, opts, J, dev_out, dc, delta, split);
            else jacobian_mg<double>(c, aq, g, wav, dt, n_steps, ss, opts, J, dev_out, dc, delta, split);
            c.timing.node_updates = c.hm.n * n_steps * (aq.n_src + (c.timing.jac_runs == 1 ? 0 : aq.n_src * aq.n_rec));
        } else {
            MGRT_REQUIRE(mode == MGRT_JAC_EXACT, MGRT_E_ARG, "unknown Jacobian mode");
            MGRT_REQUIRE(cols && n_cols >= 1, MGRT_E_ARG, "EXACT mode needs a column list");
            std::vector<int64_t> cl(cols, cols + n_cols);
            for (int64_t j : cl) MGRT_REQUIRE(j >= 0 && j < c.hm.nc, MGRT_E_ARG, "column out of range");
            if (prec == 32) jacobian_exact<float>(c, aq, g, dt, n_steps, ss, cl, opts, J, dev_out);
            else jacobian_exact<double>(c, aq, g, dt, n_steps, ss, cl, opts, J, dev_out);
            c.timing.node_updates = c.hm.n * n_steps * (aq.n_src + aq.n_src * n_cols);
        }
        c.timing.call_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (!dev_out) {
            const int64_t nout = (mode == MGRT_JAC_EXACT ? n_cols : c.hm.nc) * aq.n_src * aq.n_rec * n_samples;
            for (int64_t k = 0; k < nout; ++k)
                MGRT_REQUIRE(std::isfinite(J[k]), MGRT_E_NONFINITE, "non-finite Jacobian entry");
        }
    });
}
