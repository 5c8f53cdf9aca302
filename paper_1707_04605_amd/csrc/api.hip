// C ABI of libmgrt: context, mesh and permittivity upload, forward traces.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>

#include "mgrt_internal.hpp"

namespace mgrt {

int run_precision(const mgrt_run_opts *o) {
    int p = o ? o->precision : 0;
    if (p == 0) p = 32;
    MGRT_REQUIRE(p == 32 || p == 64, MGRT_E_ARG, "precision must be 32 or 64");
    return p;
}

Acquisition make_acquisition(Ctx &c, int64_t n_src, const double *src_xyz, int32_t n_rec,
                             const double *rec_xyz) {
    MGRT_REQUIRE(c.have_mesh, MGRT_E_STATE, "no mesh uploaded");
    MGRT_REQUIRE(c.have_eps, MGRT_E_STATE, "no permittivity uploaded");
    MGRT_REQUIRE(n_src >= 1 && n_rec >= 1, MGRT_E_ARG, "need n_src >= 1 and n_rec >= 1");
    MGRT_REQUIRE(src_xyz && rec_xyz, MGRT_E_ARG, "null source or receiver coordinates");
    const int d = c.hm.d;
    for (int64_t k = 0; k < n_src * d; ++k)
        MGRT_REQUIRE(std::isfinite(src_xyz[k]), MGRT_E_NONFINITE, "non-finite source coordinate");
    for (int64_t k = 0; k < n_src * n_rec * d; ++k)
        MGRT_REQUIRE(std::isfinite(rec_xyz[k]), MGRT_E_NONFINITE, "non-finite receiver coordinate");
    Acquisition a;
    a.n_src = n_src;
    a.n_rec = n_rec;
    a.src = locate_points(c.hm, n_src, src_xyz);
    a.rec = locate_points(c.hm, n_src * n_rec, rec_xyz);
    return a;
}

// g_l = (w_l - w_{l-1}) / dt, w_{-1} = 0: the load difference of the three-level form.
std::vector<double> load_series(const double *w, int64_t n_steps, double dt) {
    MGRT_REQUIRE(w, MGRT_E_ARG, "null wavelet");
    std::vector<double> g(n_steps);
    double prev = 0.0;
    for (int64_t l = 0; l < n_steps; ++l) {
        MGRT_REQUIRE(std::isfinite(w[l]), MGRT_E_NONFINITE, "non-finite wavelet sample");
        g[l] = (w[l] - prev) / dt;
        prev = w[l];
    }
    return g;
}

void check_stability(Ctx &c, double dt, int flags) {
    MGRT_REQUIRE(std::isfinite(dt) && dt > 0, MGRT_E_ARG, "dt must be positive and finite");
    if (flags & MGRT_F_SKIP_STABILITY) return;
    const double bound = 2.0 / std::sqrt(c.gersh);
    MGRT_REQUIRE(dt <= bound, MGRT_E_UNSTABLE,
                 "dt = " + std::to_string(dt) + " exceeds the stability bound " + std::to_string(bound));
}

static void copy_out(const double *src_host, size_t count, double *dst, int flags, hipStream_t s) {
    if (flags & MGRT_F_DEVICE_OUT) {
        MGRT_HIP(hipMemcpyAsync(dst, src_host, count * sizeof(double), hipMemcpyHostToDevice, s));
        MGRT_HIP(hipStreamSynchronize(s));
    } else {
        std::memcpy(dst, src_host, count * sizeof(double));
    }
}

// Forward traces for all sources; returns host traces [src][rec][step].
static std::vector<double> forward_impl(Ctx &c, const Acquisition &aq, const double *wavelet,
                                        double dt, int64_t n_steps, const mgrt_run_opts *opts) {
    const int prec = run_precision(opts);
    const int variant = opts ? opts->variant : MGRT_STEP_BATCHED;
    const int flags = opts ? opts->flags : 0;
    const int d = c.hm.d, V = d + 1;
    const int64_t n = c.hm.n;
    std::vector<double> g = load_series(wavelet, n_steps, dt);
    std::vector<double> traces(aq.n_src * aq.n_rec * n_steps, 0.0);
    c.timing = mgrt_timing{};
    c.timing.nodes = n;
    c.timing.precision = prec;
    auto t0 = std::chrono::steady_clock::now();

    if (variant == MGRT_STEP_PLAIN) {
        MGRT_REQUIRE(!c.have_pml, MGRT_E_ARG, "the plain reference stepper has no PML");
        MGRT_REQUIRE(prec == 64, MGRT_E_ARG, "the plain stepper is FP64 only");
        const int64_t n_parts = (int64_t)aq.n_rec * V;
        DevBuf parts(n_steps * n_parts * sizeof(double));
        std::vector<double> hp(n_steps * n_parts);
        for (int64_t s = 0; s < aq.n_src; ++s) {
            std::vector<Record> rec;
            for (int r = 0; r < aq.n_rec; ++r)
                for (int a = 0; a < V; ++a)
                    rec.push_back(Record{aq.rec[s * aq.n_rec + r].node[a], 0, r * V + a,
                                         aq.rec[s * aq.n_rec + r].w[a]});
            run_plain(c, dt, n_steps, aq.src[s], g.data(), rec, parts.as<double>(), n_parts, flags);
            MGRT_HIP(hipMemcpy(hp.data(), parts.p, hp.size() * sizeof(double), hipMemcpyDeviceToHost));
            for (int r = 0; r < aq.n_rec; ++r)
                for (int64_t l = 0; l < n_steps; ++l) {
                    double t = 0;
                    for (int a = 0; a < V; ++a) t += hp[l * n_parts + r * V + a];
                    traces[(s * aq.n_rec + r) * n_steps + l] = t;
                }
        }
        c.timing.batch = 1;
    } else {
        MGRT_REQUIRE(variant == MGRT_STEP_BATCHED, MGRT_E_ARG, "unknown stepping variant");
        const int B = pick_batch(c, prec, aq.n_src, opts ? opts->batch : 0, dt, flags);
        const int S = tile_nodes(prec, B);
        StepOp &op = get_step_op(c, S, prec, dt);
        const size_t esz = prec == 32 ? 4 : 8;
        DevBuf series = upload(g, c.stream);
        DevBuf bufA(n * B * esz), bufB(n * B * esz);
        const int64_t n_parts = (int64_t)B * aq.n_rec * V;
        DevBuf parts(n_steps * n_parts * sizeof(double));
        std::vector<double> hp(n_steps * n_parts);
        for (int64_t s0 = 0; s0 < aq.n_src; s0 += B) {
            const int nb = (int)std::min<int64_t>(B, aq.n_src - s0);
            BatchRun run;
            run.prec = prec;
            run.B = B;
            run.flags = flags; run.launch = opts ? opts->launch : 0;
            run.n_steps = n_steps;
            run.d_series = series.as<double>();
            run.series_len = n_steps;
            for (int b = 0; b < nb; ++b) {
                const Stencil &st = aq.src[s0 + b];
                for (int a = 0; a < V; ++a)
                    run.inj.push_back(Injection{st.node[a], b, 0, op.gamma[st.node[a]] * st.w[a]});
                for (int r = 0; r < aq.n_rec; ++r) {
                    const Stencil &rs = aq.rec[(s0 + b) * aq.n_rec + r];
                    for (int a = 0; a < V; ++a)
                        run.rec.push_back(Record{rs.node[a], b, (b * aq.n_rec + r) * V + a, rs.w[a]});
                }
            }
            run.d_parts = parts.as<double>();
            run.n_parts = n_parts;
            MGRT_HIP(hipMemsetAsync(bufA.p, 0, bufA.bytes, c.stream));
            MGRT_HIP(hipMemsetAsync(bufB.p, 0, bufB.bytes, c.stream));
            run.d_p = bufA.p;
            run.d_pm = bufB.p;
            run_batch(c, op, run);
            MGRT_HIP(hipMemcpy(hp.data(), parts.p, hp.size() * sizeof(double), hipMemcpyDeviceToHost));
            for (int b = 0; b < nb; ++b)
                for (int r = 0; r < aq.n_rec; ++r)
                    for (int64_t l = 0; l < n_steps; ++l) {
                        double t = 0;
                        for (int a = 0; a < V; ++a) t += hp[l * n_parts + (b * aq.n_rec + r) * V + a];
                        traces[((s0 + b) * aq.n_rec + r) * n_steps + l] = t;
                    }
        }
        c.timing.batch = B;
        c.timing.ell_width = op.wmax;
        c.timing.ell_mean_width = op.wmean;
    }
    c.timing.node_updates = n * n_steps * aq.n_src;
    c.timing.call_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    for (double t : traces)
        MGRT_REQUIRE(std::isfinite(t), MGRT_E_NONFINITE, "non-finite trace value (unstable run?)");
    return traces;
}

// ------------------------------------------------------------------------------------
// Allocation-free forward traces.  Device memory beyond the caller's inputs and outputs
// comes from one file-scope array per GPU, `scratch`, whose device address is taken once
// per device (hipGetSymbolAddress) when a context is created there; host code only ever
// uses that address, never the array's name.  Every call on a GPU shares its array.

constexpr size_t NOALLOC_SCRATCH_BYTES = 64ull << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;

static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Take scratch's address on `device` (current) once; false if HIP refuses.
bool init_scratch(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return true;   // no allocation-free calls
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return true;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return false;
    g_scratch_ptr[device] = p;
    return true;
}

void *scratch_on(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

template <typename T>
__global__ void k_clear(T *__restrict__ x, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) x[i] = T(0);
}

// traces[q][l] = sum_{a < V} parts[l][q V + a] for the nq traces of a batch (the host
// reduction's order), and bad = 1 where a result is not finite
__global__ void k_sum_parts(const double *__restrict__ parts, int64_t n_steps, int64_t n_parts,
                            int64_t nq, int V, double *__restrict__ traces, int *__restrict__ bad) {
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= nq * n_steps) return;
    const int64_t q = idx / n_steps, l = idx - q * n_steps;
    double t = 0;
    for (int a = 0; a < V; ++a) t += parts[l * n_parts + q * V + a];
    traces[idx] = t;
    if (!isfinite(t)) bad[0] = 1;
}

}  // namespace

static void forward_noalloc(Ctx &c, const Acquisition &aq, const double *wavelet, double dt,
                            int64_t n_steps, const mgrt_run_opts *opts, double *traces) {
    const int prec = run_precision(opts);
    const int flags = opts ? opts->flags : 0;
    MGRT_REQUIRE(!opts || opts->variant == MGRT_STEP_BATCHED, MGRT_E_ARG,
                 "the allocation-free entry point runs the batched stepper only");
    const int d = c.hm.d, V = d + 1;
    const int64_t n = c.hm.n;
    // batch width: requested, else what this context's batch tuner chose for this column
    // count, else the default rule; the operator must already exist (an earlier allocating
    // call with the same precision, batch width, dt and permittivity built it)
    const int req = opts ? opts->batch : 0;
    int B = choose_batch(prec, aq.n_src, req);
    if (req == 0) {
        int top = 1;
        while (top < aq.n_src && top < 128) top <<= 1;
        const auto hit = c.batch_tuned.find(std::make_tuple(prec, (int64_t)top));
        if (hit != c.batch_tuned.end()) B = hit->second;
    }
    const auto oit = c.ops.find(std::make_tuple(tile_nodes(prec, B), prec));
    MGRT_REQUIRE(oit != c.ops.end() && oit->second->dt == dt && oit->second->eps_version == c.eps_version,
                 MGRT_E_STATE,
                 "no step operator for this precision, batch width, dt and permittivity yet: "
                 "call mgrt_forward_traces once with the same arguments first");
    StepOp &op = *oit->second;
    void *sp = scratch_on(c.device);
    MGRT_REQUIRE(sp, MGRT_E_HIP, "no allocation-free scratch on this device");
    Arena ar;
    ar.base = static_cast<char *>(sp);
    ar.cap = NOALLOC_SCRATCH_BYTES;
    const size_t esz = prec == 32 ? 4 : 8;
    const bool dev_out = (flags & MGRT_F_DEVICE_OUT) != 0;
    const int64_t n_parts = (int64_t)B * aq.n_rec * V;
    const int64_t per_batch = (int64_t)B * aq.n_rec * n_steps;
    double *d_series = put(ar, load_series(wavelet, n_steps, dt));
    void *bufA = ar.take(n * B * esz), *bufB = ar.take(n * B * esz);
    double *parts = static_cast<double *>(ar.take((size_t)n_steps * n_parts * sizeof(double)));
    double *stage = dev_out ? nullptr : static_cast<double *>(ar.take((size_t)per_batch * sizeof(double)));
    int *bad = static_cast<int *>(ar.take(sizeof(int)));
    hipStream_t s = c.stream;
    hipLaunchKernelGGL(k_clear<int>, dim3(1), dim3(256), 0, s, bad, (int64_t)1);
    const size_t mark = ar.used;
    const int64_t nstate = n * B * (int64_t)(esz / 4);         // 32-bit words per state field
    for (int64_t s0 = 0; s0 < aq.n_src; s0 += B) {
        const int nb = (int)std::min<int64_t>(B, aq.n_src - s0);
        ar.used = mark;                                         // per-batch tile lists
        BatchRun run;
        run.prec = prec;
        run.B = B;
        run.flags = flags | MGRT_F_NO_TUNE | MGRT_F_NO_GRAPH;
        run.launch = opts ? opts->launch : 0;
        run.n_steps = n_steps;
        run.d_series = d_series;
        run.series_len = n_steps;
        run.arena = &ar;
        for (int b = 0; b < nb; ++b) {
            const Stencil &st = aq.src[s0 + b];
            for (int a = 0; a < V; ++a)
                run.inj.push_back(Injection{st.node[a], b, 0, op.gamma[st.node[a]] * st.w[a]});
            for (int r = 0; r < aq.n_rec; ++r) {
                const Stencil &rs = aq.rec[(s0 + b) * aq.n_rec + r];
                for (int a = 0; a < V; ++a)
                    run.rec.push_back(Record{rs.node[a], b, (b * aq.n_rec + r) * V + a, rs.w[a]});
            }
        }
        run.d_parts = parts;
        run.n_parts = n_parts;
        hipLaunchKernelGGL(k_clear<uint32_t>, dim3((nstate + 255) / 256), dim3(256), 0, s,
                           static_cast<uint32_t *>(bufA), nstate);
        hipLaunchKernelGGL(k_clear<uint32_t>, dim3((nstate + 255) / 256), dim3(256), 0, s,
                           static_cast<uint32_t *>(bufB), nstate);
        run.d_p = bufA;
        run.d_pm = bufB;
        run_batch(c, op, run);
        const int64_t nq = (int64_t)nb * aq.n_rec;
        double *dst = dev_out ? traces + s0 * aq.n_rec * n_steps : stage;
        hipLaunchKernelGGL(k_sum_parts, dim3((nq * n_steps + 255) / 256), dim3(256), 0, s, parts,
                           n_steps, n_parts, nq, V, dst, bad);
        MGRT_HIP(hipGetLastError());
        if (!dev_out)
            MGRT_HIP(hipMemcpyAsync(traces + s0 * aq.n_rec * n_steps, stage,
                                    (size_t)nq * n_steps * sizeof(double), hipMemcpyDeviceToHost, s));
        MGRT_HIP(hipStreamSynchronize(s));
    }
    int hbad = 0;
    MGRT_HIP(hipMemcpy(&hbad, bad, sizeof(int), hipMemcpyDeviceToHost));
    MGRT_REQUIRE(!hbad, MGRT_E_NONFINITE, "non-finite trace value (unstable run?)");
    c.timing.batch = B;
    c.timing.ell_width = op.wmax;
    c.timing.ell_mean_width = op.wmean;
}

}  // namespace mgrt

using namespace mgrt;

extern "C" {

int mgrt_create(int device, void *hip_stream, mgrt_ctx **out) {
    if (!out) return MGRT_E_ARG;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return MGRT_E_HIP;
    if (hipSetDevice(device) != hipSuccess) return MGRT_E_HIP;
    if (!init_scratch(device)) return MGRT_E_HIP;
    mgrt_ctx *ctx = new (std::nothrow) mgrt_ctx();
    if (!ctx) return MGRT_E_OOM_PLAN;
    ctx->c.device = device;
    if (hip_stream) {
        ctx->c.stream = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&ctx->c.stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return MGRT_E_HIP;
        }
        ctx->c.own_stream = true;
    }
    *out = ctx;
    return MGRT_OK;
}

int mgrt_destroy(mgrt_ctx *ctx) {
    if (!ctx) return MGRT_E_ARG;
    (void)hipSetDevice(ctx->c.device);
    (void)hipStreamSynchronize(ctx->c.stream);
    bool own = ctx->c.own_stream;
    hipStream_t s = ctx->c.stream;
    delete ctx;
    if (own) (void)hipStreamDestroy(s);
    return MGRT_OK;
}

const char *mgrt_last_error(const mgrt_ctx *ctx) {
    if (!ctx) return "null context";
    return ctx->c.last_error.c_str();
}

int mgrt_upload_mesh(mgrt_ctx *ctx, int dim, int64_t n_nodes, const double *coords,
                     int64_t n_elems, const int32_t *elems, int64_t n_bfacets,
                     const int32_t *bfacets, const double *admittance, int64_t n_coarse,
                     const int32_t *coarse_of_elem, const int32_t *coarse_verts) {
    return mgrt_guarded(ctx, [&](Ctx &c) {
        MGRT_REQUIRE(dim == 2 || dim == 3, MGRT_E_ARG, "dim must be 2 or 3");
        MGRT_REQUIRE(n_nodes > dim && n_elems > 0 && coords && elems, MGRT_E_ARG, "empty mesh");
        MGRT_REQUIRE(n_nodes < (int64_t)1 << 31, MGRT_E_ARG, "node ids must fit int32");
        MGRT_REQUIRE(n_bfacets >= 0 && (n_bfacets == 0 || bfacets), MGRT_E_ARG, "bad boundary facets");
        MGRT_REQUIRE(n_coarse >= 0, MGRT_E_ARG, "bad n_coarse");
        for (int64_t k = 0; k < n_nodes * dim; ++k)
            MGRT_REQUIRE(std::isfinite(coords[k]), MGRT_E_NONFINITE, "non-finite coordinate");
        c.have_mesh = false;
        c.have_eps = false;
        c.have_pml = false;
        c.rxi.clear();
        c.pml_zeta.clear();
        c.ops.clear();
        c.tuned.clear();
        c.batch_tuned.clear();
        build_host_mesh(c.hm, dim, n_nodes, coords, n_elems, elems, n_bfacets, bfacets, admittance,
                        n_coarse, coarse_of_elem, coarse_verts);
        HostMesh &hm = c.hm;
        choose_node_order(hm);
        build_node_grid(hm);
        c.dm = DevMesh();
        c.dm.iperm = upload(hm.iperm, c.stream);
        c.dm.krow = upload(hm.krow, c.stream);
        c.dm.kcol = upload(hm.kcol, c.stream);
        c.dm.kval = upload(hm.kval, c.stream);
        c.dm.kdiag = upload(hm.kdiag, c.stream);
        c.dm.rbound = upload(hm.rbound, c.stream);
        c.dm.elems = upload(hm.elems, c.stream);
        c.dm.vol = upload(hm.vol, c.stream);
        if (hm.nc > 0) {
            c.dm.c2f_ptr = upload(hm.c2f_ptr, c.stream);
            c.dm.c2f_idx = upload(hm.c2f_idx, c.stream);
            c.dm.cvol = upload(hm.cvol, c.stream);
            c.dm.cnodes = upload(hm.cnodes, c.stream);
            c.dm.cvert_idx = upload(hm.cvert_idx, c.stream);
        }
        MGRT_HIP(hipStreamSynchronize(c.stream));
        c.have_mesh = true;
    });
}

int mgrt_upload_permittivity(mgrt_ctx *ctx, const double *eps, const double *sigma) {
    return mgrt_guarded(ctx, [&](Ctx &c) {
        MGRT_REQUIRE(c.have_mesh, MGRT_E_STATE, "no mesh uploaded");
        MGRT_REQUIRE(eps, MGRT_E_ARG, "null eps");
        const HostMesh &hm = c.hm;
        const int V = hm.d + 1;
        for (int64_t t = 0; t < hm.m; ++t) {
            MGRT_REQUIRE(std::isfinite(eps[t]), MGRT_E_NONFINITE, "non-finite eps");
            MGRT_REQUIRE(eps[t] > 0, MGRT_E_ARG, "eps must be > 0");
            if (sigma) {
                MGRT_REQUIRE(std::isfinite(sigma[t]), MGRT_E_NONFINITE, "non-finite sigma");
                MGRT_REQUIRE(sigma[t] >= 0, MGRT_E_ARG, "sigma must be >= 0");
            }
        }
        // lumped masses, gathered per node in a fixed order (deterministic)
        c.Mlump.assign(hm.n, 0.0);
        c.rsig = hm.rbound;
        parallel_for(hm.n, [&](int64_t i0, int64_t i1) {
            for (int64_t i = i0; i < i1; ++i) {
                double ms = 0, rs = 0;
                for (int64_t k = hm.n2e_ptr[i]; k < hm.n2e_ptr[i + 1]; ++k) {
                    const int64_t t = hm.n2e_idx[k] / V;
                    ms += eps[t] * hm.vol[t] / V;
                    if (sigma) rs += sigma[t] * hm.vol[t] / V;
                }
                c.Mlump[i] = ms;
                c.rsig[i] += rs;
            }
        });
        c.rdamp = c.rsig;
        if (c.have_pml)
            for (int64_t i = 0; i < hm.n; ++i) c.rdamp[i] += c.rxi[i];
        double gmax = 0;
        for (int64_t i = 0; i < hm.n; ++i) {
            double row = std::fabs(hm.kdiag[i]);
            for (int64_t k = hm.krow[i]; k < hm.krow[i + 1]; ++k) row += std::fabs(hm.kval[k]);
            gmax = std::max(gmax, row / c.Mlump[i]);
        }
        c.gersh = gmax;
        c.dM = upload(c.Mlump, c.stream);
        c.dR = upload(c.rdamp, c.stream);
        MGRT_HIP(hipStreamSynchronize(c.stream));
        c.eps_version++;
        c.have_eps = true;
    });
}

int mgrt_upload_pml(mgrt_ctx *ctx, const double *xi, const double *zeta) {
    return mgrt_guarded(ctx, [&](Ctx &c) {
        MGRT_REQUIRE(c.have_mesh, MGRT_E_STATE, "no mesh uploaded");
        MGRT_REQUIRE((xi == nullptr) == (zeta == nullptr), MGRT_E_ARG,
                     "xi and zeta must both be given or both be null");
        const HostMesh &hm = c.hm;
        const int d = hm.d, V = d + 1;
        c.have_pml = false;
        c.rxi.clear();
        c.pml_zeta.clear();
        if (xi) {
            for (int64_t t = 0; t < hm.m; ++t) {
                MGRT_REQUIRE(std::isfinite(xi[t]) && xi[t] >= 0, MGRT_E_ARG, "xi must be finite and >= 0");
                for (int k = 0; k < d; ++k)
                    MGRT_REQUIRE(std::isfinite(zeta[t * d + k]) && zeta[t * d + k] >= 0, MGRT_E_ARG,
                                 "zeta must be finite and >= 0");
            }
            c.pml_zeta.assign(zeta, zeta + hm.m * d);
            c.rxi.assign(hm.n, 0.0);
            parallel_for(hm.n, [&](int64_t i0, int64_t i1) {
                for (int64_t i = i0; i < i1; ++i) {
                    double rs = 0;
                    for (int64_t k = hm.n2e_ptr[i]; k < hm.n2e_ptr[i + 1]; ++k) {
                        const int64_t t = hm.n2e_idx[k] / V;
                        rs += xi[t] * hm.vol[t] / V;
                    }
                    c.rxi[i] = rs;
                }
            });
            c.have_pml = true;
        }
        if (c.have_eps) {
            c.rdamp = c.rsig;
            if (c.have_pml)
                for (int64_t i = 0; i < hm.n; ++i) c.rdamp[i] += c.rxi[i];
            c.dR = upload(c.rdamp, c.stream);
            MGRT_HIP(hipStreamSynchronize(c.stream));
            c.eps_version++;
        }
    });
}

int mgrt_stability_bound(mgrt_ctx *ctx, double *dt_max) {
    return mgrt_guarded(ctx, [&](Ctx &c) {
        MGRT_REQUIRE(dt_max, MGRT_E_ARG, "null output");
        MGRT_REQUIRE(c.have_eps, MGRT_E_STATE, "no permittivity uploaded");
        *dt_max = 2.0 / std::sqrt(c.gersh);
    });
}

int mgrt_forward_traces(mgrt_ctx *ctx, int64_t n_src, const double *src_xyz, int32_t n_rec,
                        const double *rec_xyz, const double *wavelet, double dt,
                        int64_t n_steps, const mgrt_run_opts *opts, double *traces) {
    return mgrt_guarded(ctx, [&](Ctx &c) {
        MGRT_REQUIRE(traces, MGRT_E_ARG, "null traces output");
        MGRT_REQUIRE(n_steps >= 1, MGRT_E_ARG, "n_steps must be >= 1");
        const int flags = opts ? opts->flags : 0;
        Acquisition aq = make_acquisition(c, n_src, src_xyz, n_rec, rec_xyz);
        check_stability(c, dt, flags);
        std::vector<double> tr = forward_impl(c, aq, wavelet, dt, n_steps, opts);
        copy_out(tr.data(), tr.size(), traces, flags, c.stream);
    });
}

int mgrt_forward_traces_noalloc(mgrt_ctx *ctx, int64_t n_src, const double *src_xyz, int32_t n_rec,
                                const double *rec_xyz, const double *wavelet, double dt,
                                int64_t n_steps, const mgrt_run_opts *opts, double *traces) {
    return mgrt_guarded(ctx, [&](Ctx &c) {
        MGRT_REQUIRE(traces, MGRT_E_ARG, "null traces output");
        MGRT_REQUIRE(n_steps >= 1, MGRT_E_ARG, "n_steps must be >= 1");
        const int flags = opts ? opts->flags : 0;
        Acquisition aq = make_acquisition(c, n_src, src_xyz, n_rec, rec_xyz);
        check_stability(c, dt, flags);
        c.timing = mgrt_timing{};
        c.timing.nodes = c.hm.n;
        c.timing.precision = run_precision(opts);
        auto t0 = std::chrono::steady_clock::now();
        forward_noalloc(c, aq, wavelet, dt, n_steps, opts, traces);
        c.timing.node_updates = c.hm.n * n_steps * n_src;
        c.timing.call_ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    });
}

int mgrt_last_timing(const mgrt_ctx *ctx, mgrt_timing *out) {
    if (!ctx || !out) return MGRT_E_ARG;
    *out = ctx->c.timing;
    return MGRT_OK;
}

int mgrt_struct_sizes(size_t *run_opts_bytes, size_t *timing_bytes) {
    if (run_opts_bytes) *run_opts_bytes = sizeof(mgrt_run_opts);
    if (timing_bytes) *timing_bytes = sizeof(mgrt_timing);
    return MGRT_OK;
}

}  // extern "C"
