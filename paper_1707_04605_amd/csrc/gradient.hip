// Misfit gradient g = J1^T rho by a reverse-time adjoint run (the transpose of the
// auxiliary system of App. A-1, eq. linearized1/2).
//
// With y_l = phi_r . p_{l+1}, a permittivity direction changes the traces by
// dy_l = sum_{m<=l} phi_r . Phi(l-m) h_m, h_m = dM (.) b_m, b_m = -(p_{m+1} - p_m)/dt,
// where Phi(k) is the (symmetric) response of the recurrence to a unit load k steps
// earlier.  So sum_l rho_l dy_l = sum_m lambda_m . h_m with
// lambda_m = sum_{l>=m} Phi(l-m) phi_r rho_l, which is the state after N-m steps of
// the SAME recurrence driven by the time-reversed residual at the receivers.  For every
// node i the adjoint sweep accumulates acc_i = sum_m sum_sources lambda_{m,i} b_{m,i};
// then d/d eps_T = |T|/(d+1) sum_{i in T} acc_i and d/dc_j = sum_{T in T'_j} d/d eps_T.
//
// The adjoint runs forward in its own time while it needs b_m backwards in m: the
// forward sweep keeps checkpoints (p_a, p_{a-1}) every K steps; segments are then
// recomputed last-to-first, their velocities stored in HBM, and consumed in reverse by
// the adjoint steps.  K ~ sqrt(2N) minimises memory; the batch width shrinks until the
// plan fits the device.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "mgrt_internal.hpp"

namespace mgrt {

namespace {

// acc is indexed in stepping order: iperm maps the caller's node ids into it
__global__ void k_grad_fine(const double *__restrict__ acc, const int32_t *__restrict__ iperm,
                            const int32_t *__restrict__ elems, const double *__restrict__ vol,
                            int V, int64_t m, double *__restrict__ gf) {
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (t >= m) return;
    double s = 0.0;
    for (int a = 0; a < V; ++a) s += acc[iperm[elems[t * V + a]]];
    gf[t] = s * vol[t] / V;
}

__global__ void k_grad_coarse(const double *__restrict__ gf, const int64_t *__restrict__ ptr,
                              const int32_t *__restrict__ idx, int64_t nc,
                              double *__restrict__ gc) {
    const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (j >= nc) return;
    double s = 0.0;
    for (int64_t k = ptr[j]; k < ptr[j + 1]; ++k) s += gf[idx[k]];
    gc[j] = s;
}

size_t free_cap(const mgrt_run_opts *o) {
    size_t fr = 0, tot = 0;
    MGRT_HIP(hipMemGetInfo(&fr, &tot));
    size_t cap = fr > (size_t)(2ull << 30) ? fr - (size_t)(2ull << 30) : fr / 2;
    if (o && o->mem_budget_gb > 0) cap = std::min(cap, (size_t)(o->mem_budget_gb * (1ull << 30)));
    return cap;
}

template <typename T>
void gradient_t(Ctx &c, const Acquisition &aq, const std::vector<double> &g, double dt, int64_t N,
                const double *residual, int level, const mgrt_run_opts *opts, double *grad) {
    const HostMesh &hm = c.hm;
    const int prec = sizeof(T) == 4 ? 32 : 64;
    const int flags = opts ? opts->flags : 0;
    const int V = hm.d + 1;
    const int64_t n = hm.n;
    const size_t esz = sizeof(T);

    // plan: slabs of n*B*esz bytes -- 2 per checkpoint, K for the segment, 4 states; with a
    // PML also its q state (n_ent*B*esz) per checkpoint and for the two running sweeps
    const size_t cap = free_cap(opts);
    const int64_t n_ent = pml_entries(c);
    int B = pick_batch(c, prec, aq.n_src, opts ? opts->batch : 0, dt, flags);
    int64_t K = 1;
    auto slabs = [&](int64_t k) { return 2 * ((N + k - 1) / k) + k + 4; };
    auto plan = [&](int b) {
        int64_t best = 1;
        size_t bm = SIZE_MAX;
        for (int64_t k = std::max<int64_t>(1, (int64_t)std::sqrt(2.0 * N) / 2);
             k <= std::min<int64_t>(N, (int64_t)std::sqrt(2.0 * N) * 2 + 1); ++k) {
            size_t m = (size_t)slabs(k) * n * b * esz + (size_t)((N + k - 1) / k + 2) * n_ent * b * esz;
            if (m < bm) { bm = m; best = k; }
        }
        K = best;
        return bm + (size_t)n * 8;
    };
    while (plan(B) > cap && B > 1) B = (B == 4 && prec == 32) ? 1 : B / 2;
    MGRT_REQUIRE(plan(B) <= cap, MGRT_E_OOM_PLAN,
                 "checkpoints for one source do not fit the device memory budget");
    const int64_t nseg = (N + K - 1) / K;
    const size_t slab = (size_t)n * B * esz;

    DevBuf ck(slab * 2 * nseg), seg(slab * K), fA(slab), fB(slab), aA(slab), aB(slab);
    const size_t qsz = (size_t)n_ent * B * esz;
    DevBuf ckq(qsz * nseg), fq(qsz), aq_state(qsz);
    char *ckqp = static_cast<char *>(ckq.p);
    DevBuf acc((size_t)n * 8);
    MGRT_HIP(hipMemsetAsync(acc.p, 0, acc.bytes, c.stream));
    DevBuf series = upload(g, c.stream);
    StepOp &op = get_step_op(c, tile_nodes(prec, B), prec, dt);
    char *ckp = static_cast<char *>(ck.p);

    for (int64_t s0 = 0; s0 < aq.n_src; s0 += B) {
        const int nb = (int)std::min<int64_t>(B, aq.n_src - s0);
        std::vector<Injection> fwd_inj;
        for (int b = 0; b < nb; ++b) {
            const Stencil &st = aq.src[s0 + b];
            for (int a = 0; a < V; ++a)
                fwd_inj.push_back(Injection{st.node[a], b, 0, op.gamma[st.node[a]] * st.w[a]});
        }
        // forward sweep with checkpoints
        MGRT_HIP(hipMemsetAsync(fA.p, 0, slab, c.stream));
        MGRT_HIP(hipMemsetAsync(fB.p, 0, slab, c.stream));
        if (qsz) MGRT_HIP(hipMemsetAsync(fq.p, 0, qsz, c.stream));
        void *cur = fA.p, *prev = fB.p;
        for (int64_t j = 0; j < nseg; ++j) {
            const int64_t a0 = j * K, a1 = std::min(N, a0 + K);
            MGRT_HIP(hipMemcpyAsync(ckp + (2 * j) * slab, cur, slab, hipMemcpyDeviceToDevice, c.stream));
            MGRT_HIP(hipMemcpyAsync(ckp + (2 * j + 1) * slab, prev, slab, hipMemcpyDeviceToDevice, c.stream));
            if (qsz) MGRT_HIP(hipMemcpyAsync(ckqp + j * qsz, fq.p, qsz, hipMemcpyDeviceToDevice, c.stream));
            if (j == nseg - 1) break;   // the last segment is recomputed first anyway
            BatchRun fr;
            fr.prec = prec; fr.B = B; fr.flags = flags; fr.launch = opts ? opts->launch : 0; fr.n_steps = a1 - a0; fr.step0 = a0;
            fr.d_series = series.as<double>(); fr.series_len = N;
            fr.inj = fwd_inj;
            fr.d_p = cur; fr.d_pm = prev;
            fr.d_q = qsz ? fq.p : nullptr;
            run_batch(c, op, fr);
            cur = fr.d_p; prev = fr.d_pm;
        }
        // adjoint loads: time-reversed residuals in load-difference form
        std::vector<double> rs((size_t)nb * aq.n_rec * N);
        std::vector<Injection> adj_inj;
        for (int b = 0; b < nb; ++b)
            for (int r = 0; r < aq.n_rec; ++r) {
                const double *rho = residual + ((s0 + b) * aq.n_rec + r) * N;
                double *out = &rs[((size_t)b * aq.n_rec + r) * N];
                for (int64_t l = 0; l < N; ++l) {
                    const double cur_v = rho[N - 1 - l];
                    const double prev_v = l > 0 ? rho[N - l] : 0.0;
                    out[l] = (cur_v - prev_v) / dt;
                }
                const Stencil &st = aq.rec[(s0 + b) * aq.n_rec + r];
                for (int a = 0; a < V; ++a)
                    adj_inj.push_back(Injection{st.node[a], b, b * aq.n_rec + r, op.gamma[st.node[a]] * st.w[a]});
            }
        DevBuf aseries = upload(rs, c.stream);
        MGRT_HIP(hipMemsetAsync(aA.p, 0, slab, c.stream));
        MGRT_HIP(hipMemsetAsync(aB.p, 0, slab, c.stream));
        if (qsz) MGRT_HIP(hipMemsetAsync(aq_state.p, 0, qsz, c.stream));
        void *acur = aA.p, *aprev = aB.p;
        for (int64_t j = nseg - 1; j >= 0; --j) {
            const int64_t a0 = j * K, a1 = std::min(N, a0 + K);
            MGRT_HIP(hipMemcpyAsync(fA.p, ckp + (2 * j) * slab, slab, hipMemcpyDeviceToDevice, c.stream));
            MGRT_HIP(hipMemcpyAsync(fB.p, ckp + (2 * j + 1) * slab, slab, hipMemcpyDeviceToDevice, c.stream));
            if (qsz) MGRT_HIP(hipMemcpyAsync(fq.p, ckqp + j * qsz, qsz, hipMemcpyDeviceToDevice, c.stream));
            BatchRun fr;
            fr.prec = prec; fr.B = B; fr.flags = flags; fr.launch = opts ? opts->launch : 0; fr.n_steps = a1 - a0; fr.step0 = a0;
            fr.d_series = series.as<double>(); fr.series_len = N;
            fr.inj = fwd_inj;
            fr.d_p = fA.p; fr.d_pm = fB.p;
            fr.d_q = qsz ? fq.p : nullptr;
            fr.d_vel_out = seg.p;
            run_batch(c, op, fr);
            BatchRun ar;
            ar.prec = prec; ar.B = B; ar.flags = flags; ar.launch = opts ? opts->launch : 0; ar.n_steps = a1 - a0; ar.step0 = N - a1;
            ar.d_series = aseries.as<double>(); ar.series_len = N;
            ar.inj = adj_inj;
            ar.d_p = acur; ar.d_pm = aprev;
            ar.d_q = qsz ? aq_state.p : nullptr;
            ar.d_vel = seg.p; ar.vel_reverse = true;
            ar.d_acc = acc.as<double>();
            run_batch(c, op, ar);
            acur = ar.d_p; aprev = ar.d_pm;
        }
    }
    DevBuf gf((size_t)hm.m * 8);
    hipLaunchKernelGGL(k_grad_fine, dim3((hm.m + 255) / 256), dim3(256), 0, c.stream,
                       acc.as<double>(), c.dm.iperm.as<int32_t>(), c.dm.elems.as<int32_t>(),
                       c.dm.vol.as<double>(), V, hm.m,
                       gf.as<double>());
    MGRT_HIP(hipGetLastError());
    if (level == 1) {
        MGRT_HIP(hipStreamSynchronize(c.stream));
        MGRT_HIP(hipMemcpy(grad, gf.p, (size_t)hm.m * 8, hipMemcpyDeviceToHost));
    } else {
        DevBuf gc((size_t)hm.nc * 8);
        hipLaunchKernelGGL(k_grad_coarse, dim3((hm.nc + 255) / 256), dim3(256), 0, c.stream,
                           gf.as<double>(), c.dm.c2f_ptr.as<int64_t>(), c.dm.c2f_idx.as<int32_t>(),
                           hm.nc, gc.as<double>());
        MGRT_HIP(hipGetLastError());
        MGRT_HIP(hipStreamSynchronize(c.stream));
        MGRT_HIP(hipMemcpy(grad, gc.p, (size_t)hm.nc * 8, hipMemcpyDeviceToHost));
    }
    c.timing.batch = B;
    c.timing.node_updates = n * N * aq.n_src * 3;   // forward, recomputation, adjoint
}

}  // namespace

}  // namespace mgrt

using namespace mgrt;

extern "C" int mgrt_misfit_gradient(mgrt_ctx *ctx, int64_t n_src, const double *src_xyz,
                                    int32_t n_rec, const double *rec_xyz, const double *wavelet,
                                    double dt, int64_t n_steps, const double *residual, int level,
                                    const mgrt_run_opts *opts, double *grad) {
    return mgrt_guarded(ctx, [&](Ctx &c) {
        MGRT_REQUIRE(grad && residual, MGRT_E_ARG, "null residual or gradient output");
        MGRT_REQUIRE(n_steps >= 1, MGRT_E_ARG, "n_steps must be >= 1");
        MGRT_REQUIRE(level == 0 || level == 1, MGRT_E_ARG, "level must be 0 (coarse) or 1 (fine)");
        MGRT_REQUIRE(level == 1 || c.hm.nc > 0, MGRT_E_STATE, "no coarse level uploaded");
        MGRT_REQUIRE(!(opts && (opts->flags & MGRT_F_DEVICE_OUT)), MGRT_E_ARG,
                     "gradient output is a host array");
        const int flags = opts ? opts->flags : 0;
        const int prec = run_precision(opts);
        Acquisition aq = make_acquisition(c, n_src, src_xyz, n_rec, rec_xyz);
        check_stability(c, dt, flags);
        for (int64_t k = 0; k < n_src * n_rec * n_steps; ++k)
            MGRT_REQUIRE(std::isfinite(residual[k]), MGRT_E_NONFINITE, "non-finite residual");
        std::vector<double> g = load_series(wavelet, n_steps, dt);
        c.timing = mgrt_timing{};
        c.timing.nodes = c.hm.n;
        c.timing.precision = prec;
        auto t0 = std::chrono::steady_clock::now();
        if (prec == 32) gradient_t<float>(c, aq, g, dt, n_steps, residual, level, opts, grad);
        else gradient_t<double>(c, aq, g, dt, n_steps, residual, level, opts, grad);
        c.timing.call_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        const int64_t nout = level == 0 ? c.hm.nc : c.hm.m;
        for (int64_t k = 0; k < nout; ++k)
            MGRT_REQUIRE(std::isfinite(grad[k]), MGRT_E_NONFINITE, "non-finite gradient entry");
    });
}
