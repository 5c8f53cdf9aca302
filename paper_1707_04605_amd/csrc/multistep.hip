// Several leap-frog steps per launch on small meshes (App. A eqs. leap-frog1/2 in the
// nodal three-level form of the batched stepper, step.hip).
//
// A small mesh (tens of thousands of nodes) steps in a few microseconds, most of it launch
// and dispatch latency, and its state lives in L2.  Here each workgroup takes its tile of
// S nodes together with every node within graph distance k of the tile (its k-ring in the
// stiffness graph) into LDS, advances them k steps and writes the tile's two newest levels
// back: one launch per k steps.  A node at distance d from the tile is still exact after
// k - d steps, so sub-step s updates the nodes within distance k - 1 - s and the tile is
// exact after all k; neighbouring tiles recompute their shared rings instead of exchanging
// them.  Every node update is the batched stepper's, term by term: the increment
// beta (p_l - p_{l-1}) + sum_j c_ij (p_{l,j} - p_{l,i}) over the row's padded entries in
// the same order, the nodal loads in list order, then the receiver taps.
//
// Used for one column (B = 1) of a forward run without PML, histories, adjoint
// correlation or velocity output, on meshes of at most 256 tiles, with the largest k in
// {8, 6, 4, 2} whose largest region fits the LDS budget; MGRT_F_ONE_STEP turns it off.
#include <algorithm>
#include <memory>
#include <vector>

#include "mgrt_internal.hpp"

namespace mgrt {

namespace {

constexpr int MS_THREADS = 1024;
constexpr int MS_MAX_TILES = 256;           // larger meshes step one launch per step
constexpr int MS_LIST = 64;                 // nodal loads / taps per tile held in LDS
constexpr size_t MS_LDS = 150 * 1024;       // LDS budget per workgroup
constexpr int MS_K[] = {8, 6, 4, 2};

// Region tables of one step operator (stepping order, one column), built on first use
// and kept until the operator's values change.
struct Regions {
    int k = 0, W = 0, S = 0, rmax = 0;
    int64_t n_tiles = 0;
    DevBuf ptr;      // int32 n_tiles+1: first entry of each tile's region
    DevBuf cnt;      // int32 n_tiles*(k+1): entries of the tile within distance d
    DevBuf node;     // int32 per entry: stepping-order node (the tile's nodes first, in order)
    DevBuf nbr;      // uint16 per entry and slot: local index of the row's neighbour
    DevBuf beta;     // T per entry
    DevBuf val;      // T per entry and slot: -dt^2 K_ij / D_i (0 on padding slots)
    std::vector<std::vector<int32_t>> h_nodes;   // per tile: stepping-order node of each entry
};

int padded_width(int wmax) {
    for (int w : {4, 6, 8, 12, 16})
        if (wmax <= w) return w;
    return 0;
}

// LDS of one workgroup: p_l, p_{l-1}, beta and the W coefficients per entry (T), the W
// neighbour slots (uint16), then the nodal loads and taps; each part starts 8-byte aligned
__host__ __device__ inline size_t round8(size_t b) { return (b + 7) & ~(size_t)7; }
__host__ __device__ inline size_t region_nb_off(int rmax, int W, size_t esz) {
    return round8((size_t)rmax * esz * (3 + (size_t)W));
}
__host__ __device__ inline size_t region_tail_off(int rmax, int W, size_t esz) {
    return region_nb_off(rmax, W, esz) + round8((size_t)rmax * W * 2);
}
size_t region_lds(int rmax, int W, size_t esz) {
    return region_tail_off(rmax, W, esz) + (size_t)2 * MS_LIST * (8 + 4 + 4);
}

template <typename T>
struct RegionArgs {
    const T *p, *pm;                 // p_l, p_{l-1} (stepping order)
    T *out_p, *out_pm;               // p_{l+k}, p_{l+k-1}
    const int32_t *ptr, *cnt, *node;
    const uint16_t *nbr;
    const T *beta, *val;
    const int32_t *ld_ptr, *ld_loc, *ld_sid;   // per-tile nodal loads (local entry, series)
    const double *ld_w;
    const int32_t *tp_ptr, *tp_loc, *tp_dst;   // per-tile receiver taps (local entry, part)
    const double *tp_w;
    const double *series;
    int64_t series_len, t0;          // series index of sub-step 0
    double *parts;                   // parts row of sub-step 0 (null: no taps)
    // replayed launches: t0 and the parts row are offsets from *step_base steps, which a
    // small kernel advances at the end of every replay; null for direct launches
    const int64_t *step_base;
    int64_t n_parts, n;
    int W, k, ksteps, S, rmax;
};

template <typename T>
__global__ __launch_bounds__(MS_THREADS) void k_region_steps(const RegionArgs<T> a) {
    extern __shared__ __align__(16) unsigned char sm[];
    const int t = blockIdx.x;
    const int r0 = a.ptr[t], R = a.ptr[t + 1] - r0;
    const int W = a.W;
    T *u0 = reinterpret_cast<T *>(sm);
    T *u1 = u0 + a.rmax;
    T *be = u1 + a.rmax;
    T *vv = be + a.rmax;
    uint16_t *nb = reinterpret_cast<uint16_t *>(sm + region_nb_off(a.rmax, W, sizeof(T)));
    double *lw = reinterpret_cast<double *>(sm + region_tail_off(a.rmax, W, sizeof(T)));
    double *tw = lw + MS_LIST;
    int32_t *lloc = reinterpret_cast<int32_t *>(tw + MS_LIST);
    int32_t *lsid = lloc + MS_LIST;
    int32_t *tloc = lsid + MS_LIST;
    int32_t *tdst = tloc + MS_LIST;

    for (int e = threadIdx.x; e < R; e += MS_THREADS) {
        const int64_t g = a.node[r0 + e];
        u0[e] = a.p[g];
        u1[e] = a.pm[g];
        be[e] = a.beta[r0 + e];
        for (int w = 0; w < W; ++w) {
            vv[e * W + w] = a.val[(int64_t)(r0 + e) * W + w];
            nb[e * W + w] = a.nbr[(int64_t)(r0 + e) * W + w];
        }
    }
    const int l0 = a.ld_ptr[t], nl = a.ld_ptr[t + 1] - l0;
    const int q0 = a.tp_ptr[t], nq = a.parts ? a.tp_ptr[t + 1] - q0 : 0;
    for (int i = threadIdx.x; i < nl; i += MS_THREADS) {
        lloc[i] = a.ld_loc[l0 + i];
        lsid[i] = a.ld_sid[l0 + i];
        lw[i] = a.ld_w[l0 + i];
    }
    for (int i = threadIdx.x; i < nq; i += MS_THREADS) {
        tloc[i] = a.tp_loc[q0 + i];
        tdst[i] = a.tp_dst[q0 + i];
        tw[i] = a.tp_w[q0 + i];
    }
    __syncthreads();
    const int64_t sb = a.step_base ? a.step_base[0] : 0;
    double *parts = a.parts ? a.parts + sb * a.n_parts : nullptr;
    const int64_t tser = a.t0 + sb;
    const int64_t tile0 = (int64_t)t * a.S;
    const int ntile = (int)std::min<int64_t>(a.S, a.n - tile0);
    T *pc = u0, *pv = u1;
    for (int s = 0; s < a.ksteps; ++s) {
        const int act = a.cnt[t * (a.k + 1) + (a.ksteps - 1 - s)];
        for (int e = threadIdx.x; e < act; e += MS_THREADS) {
            const T c0 = pc[e];
            T inc = be[e] * (c0 - pv[e]);
            for (int w = 0; w < W; ++w) inc += vv[e * W + w] * (pc[nb[e * W + w]] - c0);
            for (int i = 0; i < nl; ++i)
                if (lloc[i] == e) inc += (T)(lw[i] * a.series[(int64_t)lsid[i] * a.series_len + tser + s]);
            const T out = c0 + inc;
            pv[e] = out;                               // p_{l+1} over p_{l-1}
            if (e < ntile)
                for (int i = 0; i < nq; ++i)
                    if (tloc[i] == e) parts[(int64_t)s * a.n_parts + tdst[i]] = tw[i] * (double)out;
        }
        __syncthreads();
        T *x = pc;
        pc = pv;
        pv = x;
    }
    for (int e = threadIdx.x; e < ntile; e += MS_THREADS) {
        a.out_p[tile0 + e] = pc[e];
        a.out_pm[tile0 + e] = pv[e];
    }
}

__global__ void k_region_base(int64_t *__restrict__ base, int64_t value, int advance) {
    if (blockIdx.x == 0 && threadIdx.x == 0) base[0] = advance ? base[0] + value : value;
}

// k-rings of every tile, the neighbour slots in the row's CSR order padded to W (the
// batched stepper's order), and beta and the coefficients as the stepper computes them.
template <typename T>
std::shared_ptr<Regions> build_regions(Ctx &c, const StepOp &op) {
    const HostMesh &hm = c.hm;
    const int64_t n = hm.n;
    const int S = op.S;
    const int W = padded_width(op.wmax);
    if (W == 0 || op.n_tiles > MS_MAX_TILES || n >= (1 << 30)) return nullptr;
    const int kmax = MS_K[0];
    // one breadth-first search per tile to distance kmax
    std::vector<std::vector<int32_t>> ents(op.n_tiles), depth(op.n_tiles);
    std::vector<int32_t> stamp(n, -1);
    for (int64_t t = 0; t < op.n_tiles; ++t) {
        auto &E = ents[t];
        auto &D = depth[t];
        for (int64_t ii = t * S; ii < std::min<int64_t>(n, (t + 1) * S); ++ii) {
            stamp[ii] = (int32_t)t;
            E.push_back((int32_t)ii);
            D.push_back(0);
        }
        size_t f0 = 0;
        for (int d = 1; d <= kmax; ++d) {
            const size_t f1 = E.size();
            for (size_t f = f0; f < f1; ++f) {
                const int64_t i = hm.perm[E[f]];
                for (int64_t q = hm.krow[i]; q < hm.krow[i + 1]; ++q) {
                    const int32_t jj = hm.iperm[hm.kcol[q]];
                    if (stamp[jj] == (int32_t)t) continue;
                    stamp[jj] = (int32_t)t;
                    E.push_back(jj);
                    D.push_back(d);
                }
            }
            f0 = f1;
        }
    }
    // the largest k whose largest region fits
    int k = 0, rmax = 0;
    for (int kk : MS_K) {
        int rm = 0;
        for (int64_t t = 0; t < op.n_tiles; ++t) {
            int r = 0;
            while (r < (int)depth[t].size() && depth[t][r] <= kk) ++r;
            rm = std::max(rm, r);
        }
        if (rm < 65536 && region_lds(rm, W, sizeof(T)) <= MS_LDS) {
            k = kk;
            rmax = rm;
            break;
        }
    }
    if (k == 0) return nullptr;
    auto R = std::make_shared<Regions>();
    R->k = k;
    R->W = W;
    R->S = S;
    R->rmax = rmax;
    R->n_tiles = op.n_tiles;
    std::vector<int32_t> ptr(op.n_tiles + 1, 0), cnt((size_t)op.n_tiles * (k + 1), 0), node;
    std::vector<uint16_t> nbr;
    std::vector<T> beta, val;
    std::vector<int32_t> loc(n, -1);
    R->h_nodes.resize(op.n_tiles);
    const double dt = op.dt;
    for (int64_t t = 0; t < op.n_tiles; ++t) {
        int r = 0;
        while (r < (int)depth[t].size() && depth[t][r] <= k) ++r;
        for (int e = 0; e < r; ++e) loc[ents[t][e]] = e;
        for (int d = 0; d <= k; ++d) {
            int m = 0;
            while (m < r && depth[t][m] <= d) ++m;
            cnt[(size_t)t * (k + 1) + d] = m;
        }
        ptr[t + 1] = ptr[t] + r;
        for (int e = 0; e < r; ++e) {
            const int32_t ii = ents[t][e];
            const int64_t i = hm.perm[ii];
            const double M = c.Mlump[i], h = 0.5 * dt * c.rdamp[i];
            const double Dg = M + h;
            node.push_back(ii);
            beta.push_back((T)((M - h) / Dg));
            const int64_t len = hm.krow[i + 1] - hm.krow[i];
            for (int w = 0; w < W; ++w) {
                // rows at distance k are never updated: own slots, value 0
                if (w < len && depth[t][e] < k) {
                    const int32_t jj = hm.iperm[hm.kcol[hm.krow[i] + w]];
                    MGRT_REQUIRE(loc[jj] >= 0, MGRT_E_STATE, "region table: neighbour outside its region");
                    nbr.push_back((uint16_t)loc[jj]);
                    val.push_back((T)(-dt * dt * hm.kval[hm.krow[i] + w] / Dg));
                } else {
                    nbr.push_back((uint16_t)e);
                    val.push_back((T)0);
                }
            }
        }
        R->h_nodes[t].assign(ents[t].begin(), ents[t].begin() + r);
        for (int e = 0; e < r; ++e) loc[ents[t][e]] = -1;
    }
    R->ptr = upload(ptr, c.stream);
    R->cnt = upload(cnt, c.stream);
    R->node = upload(node, c.stream);
    R->nbr = upload(nbr, c.stream);
    R->beta = upload(beta, c.stream);
    R->val = upload(val, c.stream);
    MGRT_HIP(hipStreamSynchronize(c.stream));
    return R;
}

template <typename T>
bool run_multistep_t(Ctx &c, StepOp &op, BatchRun &run) {
    const HostMesh &hm = c.hm;
    const int64_t n = hm.n;
    // the operator drops its tables whenever its values change (step.hip, get_step_op)
    if (!op.multi) {
        op.multi = build_regions<T>(c, op);
        if (!op.multi) op.multi = std::make_shared<Regions>();   // k = 0: not usable
    }
    const Regions &R = *std::static_pointer_cast<Regions>(op.multi);
    if (R.k == 0 || run.n_steps < R.k) return false;
    const int S = R.S;
    // per-tile nodal loads (every region entry that carries one, in the run's order; those
    // at distance k are never updated, so theirs never apply) and receiver taps (tile
    // nodes), held in LDS; more than MS_LIST of either in a tile: one launch per step
    std::vector<int32_t> ld_ptr(R.n_tiles + 1, 0), ld_loc, ld_sid, tp_ptr(R.n_tiles + 1, 0), tp_loc, tp_dst;
    std::vector<double> ld_w, tp_w;
    std::vector<int32_t> loc(n, -1);
    for (int64_t t = 0; t < R.n_tiles; ++t) {
        const auto &E = R.h_nodes[t];
        for (size_t e = 0; e < E.size(); ++e) loc[E[e]] = (int32_t)e;
        for (const Injection &j : run.inj) {
            const int32_t e = loc[hm.iperm[j.node]];
            if (e < 0) continue;
            ld_loc.push_back(e);
            ld_sid.push_back(j.sid);
            ld_w.push_back(j.weight);
        }
        for (const Record &q : run.rec) {
            const int32_t ii = hm.iperm[q.node];
            if (ii < t * S || ii >= (t + 1) * S) continue;
            tp_loc.push_back(ii - (int32_t)(t * S));
            tp_dst.push_back(q.dst);
            tp_w.push_back(q.weight);
        }
        ld_ptr[t + 1] = (int32_t)ld_loc.size();
        tp_ptr[t + 1] = (int32_t)tp_loc.size();
        if (ld_ptr[t + 1] - ld_ptr[t] > MS_LIST || tp_ptr[t + 1] - tp_ptr[t] > MS_LIST) return false;
        for (size_t e = 0; e < E.size(); ++e) loc[E[e]] = -1;
    }
    if (ld_loc.empty()) { ld_loc.push_back(0); ld_sid.push_back(0); ld_w.push_back(0.0); }
    if (tp_loc.empty()) { tp_loc.push_back(0); tp_dst.push_back(0); tp_w.push_back(0.0); }
    hipStream_t s = c.stream;
    DevBuf d_ldp = upload(ld_ptr, s), d_ldl = upload(ld_loc, s), d_lds = upload(ld_sid, s), d_ldw = upload(ld_w, s);
    DevBuf d_tpp = upload(tp_ptr, s), d_tpl = upload(tp_loc, s), d_tpd = upload(tp_dst, s), d_tpw = upload(tp_w, s);
    DevBuf xa((size_t)n * sizeof(T)), xb((size_t)n * sizeof(T));

    RegionArgs<T> a{};
    a.ptr = R.ptr.as<int32_t>();
    a.cnt = R.cnt.as<int32_t>();
    a.node = R.node.as<int32_t>();
    a.nbr = R.nbr.as<uint16_t>();
    a.beta = R.beta.as<T>();
    a.val = R.val.as<T>();
    a.ld_ptr = d_ldp.as<int32_t>();
    a.ld_loc = d_ldl.as<int32_t>();
    a.ld_sid = d_lds.as<int32_t>();
    a.ld_w = d_ldw.as<double>();
    a.tp_ptr = d_tpp.as<int32_t>();
    a.tp_loc = d_tpl.as<int32_t>();
    a.tp_dst = d_tpd.as<int32_t>();
    a.tp_w = d_tpw.as<double>();
    a.series = run.d_series;
    a.series_len = run.series_len;
    a.n_parts = run.n_parts;
    a.n = n;
    a.W = R.W;
    a.k = R.k;
    a.S = S;
    a.rmax = R.rmax;
    if (run.d_series == nullptr) MGRT_REQUIRE(run.inj.empty(), MGRT_E_ARG, "loads without series");
    const size_t lds = region_lds(R.rmax, R.W, sizeof(T));
    MGRT_HIP(hipFuncSetAttribute((const void *)k_region_steps<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds));
    const bool timing = (run.flags & MGRT_F_TIMING) != 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (timing) {
        MGRT_HIP(hipEventCreate(&e0));
        MGRT_HIP(hipEventCreate(&e1));
        MGRT_HIP(hipEventRecord(e0, s));
    }
    // the pair (p_l, p_{l-1}) alternates between the caller's buffers and (xa, xb): a launch
    // reads one pair while its workgroups write the other
    T *src_p = static_cast<T *>(run.d_p), *src_pm = static_cast<T *>(run.d_pm);
    T *alt_p = xa.as<T>(), *alt_pm = xb.as<T>();
    int64_t launches = 0;
    // launch of ks steps starting at step l (an offset from *base when base is set)
    auto issue = [&](int64_t l, int ks, const int64_t *base) {
        a.p = src_p;
        a.pm = src_pm;
        a.out_p = alt_p;
        a.out_pm = alt_pm;
        a.ksteps = ks;
        a.t0 = run.step0 + l;
        a.parts = run.d_parts ? run.d_parts + l * run.n_parts : nullptr;
        a.step_base = base;
        hipLaunchKernelGGL(k_region_steps<T>, dim3((unsigned)R.n_tiles), dim3(MS_THREADS), lds, s, a);
        std::swap(src_p, alt_p);
        std::swap(src_pm, alt_pm);
        ++launches;
    };
    // runs of G launches of k steps (G even: the buffer pairs are back in place after each)
    // are captured once into a graph and replayed, as the one-step launches are; the steps
    // left over and MGRT_F_NO_GRAPH take direct launches
    int64_t l = 0;
    constexpr int64_t G = 64;
    const int64_t nrep = run.n_steps / (G * R.k);
    if (!(run.flags & MGRT_F_NO_GRAPH) && nrep >= 2) {
        DevBuf dbase(sizeof(int64_t));
        int64_t *base = dbase.as<int64_t>();
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            try {
                for (int64_t j = 0; j < G; ++j) issue(j * R.k, R.k, base);
                hipLaunchKernelGGL(k_region_base, dim3(1), dim3(64), 0, s, base, G * R.k, 1);
            } catch (...) {
                hipGraph_t g2 = nullptr;
                (void)hipStreamEndCapture(s, &g2);
                if (g2) (void)hipGraphDestroy(g2);
                throw;
            }
            MGRT_HIP(hipStreamEndCapture(s, &graph));
            hipGraphExec_t exec = nullptr;
            const hipError_t ie = hipGraphInstantiateWithFlags(&exec, graph, 0);
            (void)hipGraphDestroy(graph);
            MGRT_HIP(ie);
            hipLaunchKernelGGL(k_region_base, dim3(1), dim3(64), 0, s, base, (int64_t)0, 0);
            launches = 0;
            hipError_t le = hipSuccess;
            for (int64_t r = 0; r < nrep && le == hipSuccess; ++r) le = hipGraphLaunch(exec, s);
            const hipError_t se = hipStreamSynchronize(s);
            (void)hipGraphExecDestroy(exec);
            MGRT_HIP(le);
            MGRT_HIP(se);
            l = nrep * G * R.k;
            launches = nrep * G;
            c.timing.graph_steps += l;
        } else {
            (void)hipGetLastError();
        }
    }
    for (; l < run.n_steps;) {
        const int ks = (int)std::min<int64_t>(R.k, run.n_steps - l);
        issue(l, ks, nullptr);
        l += ks;
    }
    MGRT_HIP(hipGetLastError());
    if (timing) MGRT_HIP(hipEventRecord(e1, s));
    // leave p_N, p_{N-1} in the caller's buffers
    if (src_p != run.d_p) {
        MGRT_HIP(hipMemcpyAsync(run.d_p, src_p, (size_t)n * sizeof(T), hipMemcpyDeviceToDevice, s));
        MGRT_HIP(hipMemcpyAsync(run.d_pm, src_pm, (size_t)n * sizeof(T), hipMemcpyDeviceToDevice, s));
    }
    MGRT_HIP(hipStreamSynchronize(s));
    if (timing) {
        float ms = 0;
        MGRT_HIP(hipEventElapsedTime(&ms, e0, e1));
        c.timing.step_ms_total += ms;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    c.timing.step_launches += launches;
    c.timing.steps_per_launch = R.k;
    // per step: the three state words per node and the operator, as for one-step launches
    c.timing.step_bytes += (3.0 * sizeof(T) * (double)n + op.oper_bytes) * run.n_steps;
    c.timing.batch = 1;
    c.timing.ell_width = op.wmax;
    c.timing.ell_mean_width = op.wmean;
    return true;
}

}  // namespace

bool run_multistep(Ctx &c, StepOp &op, BatchRun &run) {
    if (run.B != 1 || run.arena || run.hist || run.d_acc || run.d_vel || run.d_vel_out || run.launch != 0 ||
        (run.flags & MGRT_F_ONE_STEP) || op.pml.n_ent > 0 || op.n_tiles > MS_MAX_TILES)
        return false;
    for (const Injection &j : run.inj)
        if (j.col != 0) return false;
    for (const Record &q : run.rec)
        if (q.col != 0) return false;
    return op.prec == 32 ? run_multistep_t<float>(c, op, run) : run_multistep_t<double>(c, op, run);
}

}  // namespace mgrt
