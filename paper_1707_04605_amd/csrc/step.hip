// Leap-frog stepping kernels (App. A, eqs. leap-frog1/2) in the equivalent nodal
// three-level form.  Eliminating the element gradient field q (q_{l+1/2} - q_{l-1/2} =
// dt A^-1 B p_l) from two consecutive steps gives, with D = M + dt r/2, E = M - dt r/2,
//
//   D p_{l+1} = 2 M p_l - E p_{l-1} - dt^2 K p_l + dt (f_l - f_{l-1}),
//
// K = sum_k B^(k)T A^-1 B^(k).  Every node update reads p_l (own row and neighbours),
// reads p_{l-1} and overwrites it with p_{l+1}: three state words per node and column.
//
// The update is evaluated as an increment of p_l.  K annihilates constants (the P1
// gradients of a constant vanish), so K_ii = -sum_{j != i} K_ij and
//
//   p_{l+1} = p_l + inc,  inc = beta (p_l - p_{l-1}) + sum_{j != i} c_ij (p_{l,j} - p_{l,i})
//                               + gamma g_l,
//
// beta = E/D, c_ij = -dt^2 K_ij / D, gamma = dt^2 / D.  In exact arithmetic this is the
// recurrence above; in FP32 it keeps the operator's null space exact whatever the
// rounding of the coefficients, and every rounded term is small next to p_l (the
// differences are O(h) and O(dt) of it), where the expanded form
// 2 M/D p_l - beta p_{l-1} + sum_j c_ij p_j rounds terms of the size of p_l and lets the
// solution drift in phase over long runs.  The recorded velocity -(p_{l+1} - p_l)/dt is
// -inc/dt, taken before inc is rounded into p_{l+1}.
//
// Layout: state [n][B], nodes in mesh order, the B independent columns (sources)
// innermost so that one node's row is one contiguous 16-byte-per-lane vector load.
// A workgroup of 256 lanes owns a tile of S = 256 / LPN consecutive nodes (LPN lanes per
// node, VEC columns per lane); the stiffness rows of a tile form one SELL slice stored
// column-major (entry k of the tile's rows is contiguous).  Tiles are dealt to the 8 XCDs
// in contiguous ranges (or linearly) so that the p rows a tile shares with its
// neighbours stay in one XCD's L2.
//
// The kernels and their launch mapping are in step_kernels.hpp.  This file is the host
// side: the operator in SELL slices and packed records, the tile lists of loads, taps and
// histories, the launch variants and batch widths and their tuning, and runs of steps
// captured and replayed as graphs; small one-column runs go to multistep.hip first.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <type_traits>

#include "mgrt_internal.hpp"
#include "step_kernels.hpp"

namespace mgrt {

// ------------------------------------------------------------------------------------
// Host side.

int tile_nodes(int prec, int B) {
    int vec = (prec == 32) ? (B >= 4 ? 4 : 1) : (B >= 2 ? 2 : 1);
    int lpn = B / vec;
    return 256 / lpn;
}

int choose_batch(int prec, int64_t n_src, int requested) {
    auto ok = [&](int b) {
        if (b < 1 || b > 128 || (b & (b - 1))) return false;
        if (prec == 32 && b == 2) return false;
        return true;
    };
    if (requested > 0) {
        MGRT_REQUIRE(ok(requested), MGRT_E_ARG,
                     "batch must be a power of two in 1..128 (not 2 in FP32)");
        return requested;
    }
    int bmax = prec == 32 ? 64 : 32;
    int b = 1;
    while (b < n_src && b < bmax) b <<= 1;
    if (prec == 32 && b == 2) b = 4;
    return b;
}


// Compile-time slice width: the stiffness rows of every tile are padded to it.
static int pick_w(int wmax) {
    for (int w : {4, 6, 8, 12, 16})
        if (wmax <= w) return w;
    return 0;
}

template <typename T>
static void fill_values(Ctx &c, StepOp &op) {
    const HostMesh &hm = c.hm;
    const int64_t n = hm.n;
    const int S = op.S;
    const double dt = op.dt;
    std::vector<T> beta(n);
    op.gamma.resize(n);
    std::vector<int64_t> sptr(op.n_tiles + 1);
    MGRT_HIP(hipMemcpy(sptr.data(), op.slice_ptr.p, sptr.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    std::vector<T> vals(sptr[op.n_tiles], T(0));
    parallel_for(op.n_tiles, [&](int64_t t0, int64_t t1) {
        for (int64_t t = t0; t < t1; ++t) {
            for (int r = 0; r < S; ++r) {
                const int64_t ii = t * S + r;       // stepping order
                if (ii >= n) break;
                const int64_t i = hm.perm[ii];      // caller's node id
                const double M = c.Mlump[i], h = 0.5 * dt * c.rdamp[i];
                const double D = M + h;
                beta[ii] = (T)((M - h) / D);
                op.gamma[i] = dt * dt / D;
                const int64_t len = hm.krow[i + 1] - hm.krow[i];
                for (int64_t k = 0; k < len; ++k)
                    vals[sptr[t] + k * S + r] = (T)(-dt * dt * hm.kval[hm.krow[i] + k] / D);
            }
        }
    }, 64);
    op.beta = upload(beta, c.stream);
    op.vals = upload(vals, c.stream);
    // packed per-node records for the packed launches: beta, the coefficient shared by all
    // W entries (0 when they differ: then the first column id carries REC_GENERAL and the
    // kernel reads the slice values), W column ids; values in the working precision (FP64
    // as two 32-bit words)
    op.meta = DevBuf();
    op.meta_words = 0;
    op.uniform_rows = 0;
    op.oper_bytes = (double)hm.krow[n] * (4.0 + sizeof(T)) + (double)sizeof(T) * n;
    const int Wp = pick_w(op.wmax);
    if (Wp > 0) {
        constexpr int VW = sizeof(T) / 4;
        const int MW = 2 * VW + Wp;
        std::vector<uint32_t> meta((size_t)n * MW, 0u);
        std::vector<int64_t> uni(op.n_tiles, 0), gen_nnz(op.n_tiles, 0);
        parallel_for(op.n_tiles, [&](int64_t t0, int64_t t1) {
            for (int64_t t = t0; t < t1; ++t)
                for (int64_t r = 0; r < S && t * S + r < n; ++r) {
                    const int64_t ii = t * S + r;
                    uint32_t *rec = &meta[(size_t)ii * MW];
                    std::memcpy(&rec[0], &beta[ii], sizeof(T));
                    const int64_t i = hm.perm[ii];
                    const int64_t len = hm.krow[i + 1] - hm.krow[i];
                    const T v0 = vals[sptr[t] + r];
                    bool same = len == Wp;
                    for (int k = 1; k < Wp && same; ++k) same = vals[sptr[t] + (int64_t)k * S + r] == v0;
                    const T cu = same ? v0 : T(0);
                    std::memcpy(&rec[VW], &cu, sizeof(T));
                    for (int k = 0; k < Wp; ++k)
                        rec[2 * VW + k] = (uint32_t)(k < len ? hm.iperm[hm.kcol[hm.krow[i] + k]] : ii);
                    if (!same) {
                        rec[2 * VW] |= REC_GENERAL;
                        gen_nnz[t] += len;
                    }
                    uni[t] += same;
                }
        }, 64);
        int64_t gnnz = 0;
        for (int64_t t = 0; t < op.n_tiles; ++t) {
            op.uniform_rows += uni[t];
            gnnz += gen_nnz[t];
        }
        // operator bytes a step needs in this representation: beta, the column ids, one
        // coefficient per uniform row and every coefficient of the other rows
        op.oper_bytes = (double)sizeof(T) * (double)(n + op.uniform_rows + gnnz) + 4.0 * (double)hm.krow[n];
        op.meta = upload(meta, c.stream);
        op.meta_words = MW;
        // the most common pattern of neighbour offsets (record columns minus the node, over
        // a sample of every 7th node); speculative gathers need it on at least half of them
        std::map<std::vector<int32_t>, int64_t> freq;
        int64_t sampled = 0;
        for (int64_t ii = 0; ii < n; ii += 7, ++sampled) {
            std::vector<int32_t> off(Wp);
            for (int k = 0; k < Wp; ++k)
                off[k] = (int32_t)((int64_t)(meta[(size_t)ii * MW + 2 * VW + k] & ~REC_GENERAL) - ii);
            freq[off]++;
        }
        const auto top = std::max_element(freq.begin(), freq.end(),
                                           [](const auto &x, const auto &y) { return x.second < y.second; });
        op.spec_ok = top != freq.end() && 2 * top->second >= sampled;
        for (int k = 0; k < 8; ++k) op.spec_off[k] = op.spec_ok && k < Wp ? top->first[k] : 0;
    }
    op.pml = PmlOp();
    if (c.have_pml) {
        const int d = hm.d, NV = d + 1;
        std::vector<int64_t> et;   // entry -> element * d + direction
        for (int64_t t = 0; t < hm.m; ++t)
            for (int k = 0; k < d; ++k)
                if (c.pml_zeta[t * d + k] > 0) et.push_back(t * d + k);
        const int64_t ne = (int64_t)et.size();
        std::vector<int32_t> enode(ne * NV);
        std::vector<T> eg(ne * NV), edec(ne);
        // per node (stepping order): (entry, coefficient) pairs
        std::vector<int32_t> cnt(n + 1, 0);
        for (int64_t e = 0; e < ne; ++e) {
            const int64_t t = et[e] / d;
            for (int a = 0; a < NV; ++a) cnt[hm.iperm[hm.elems[t * NV + a]] + 1]++;
        }
        std::vector<int32_t> node_row(n, -1);
        std::vector<int32_t> rptr{0};
        std::vector<int64_t> rstart(n, 0);
        int64_t nrows = 0, nnz = 0;
        for (int64_t ii = 0; ii < n; ++ii)
            if (cnt[ii + 1] > 0) {
                node_row[ii] = (int32_t)nrows++;
                rstart[ii] = nnz;
                nnz += cnt[ii + 1];
                rptr.push_back((int32_t)nnz);
            }
        std::vector<int32_t> rent(nnz);
        std::vector<T> rcoef(nnz);
        std::vector<int64_t> fill(rstart);
        for (int64_t e = 0; e < ne; ++e) {
            const int64_t t = et[e] / d;
            const int k = (int)(et[e] % d);
            const double z = c.pml_zeta[t * d + k];
            edec[e] = (T)(1.0 - dt * z);
            for (int a = 0; a < NV; ++a) {
                const int64_t i = hm.elems[t * NV + a];
                const int64_t ii = hm.iperm[i];
                const double gk = hm.grad[(t * NV + a) * d + k];
                enode[e * NV + a] = (int32_t)ii;
                eg[e * NV + a] = (T)(dt * gk);
                const int64_t slot = fill[ii]++;
                rent[slot] = (int32_t)e;
                rcoef[slot] = (T)(op.gamma[i] * z * hm.vol[t] * gk);
            }
        }
        // per entry: its NV nodes, then dt d_k phi_a|_T for them and 1 - dt zeta (values as
        // 1 or 2 words)
        constexpr int VW = sizeof(T) / 4;
        const int MW = NV + (NV + 1) * VW;
        std::vector<uint32_t> erec((size_t)ne * MW);
        for (int64_t e = 0; e < ne; ++e) {
            uint32_t *r = &erec[(size_t)e * MW];
            for (int a = 0; a < NV; ++a) {
                r[a] = (uint32_t)enode[e * NV + a];
                std::memcpy(r + NV + a * VW, &eg[e * NV + a], sizeof(T));
            }
            std::memcpy(r + NV + NV * VW, &edec[e], sizeof(T));
        }
        PmlOp &P = op.pml;
        P.n_ent = ne;
        P.n_rows = nrows;
        P.nnz = nnz;
        P.ent_rec = upload(erec, c.stream);
        P.row_ptr = upload(rptr, c.stream);
        P.row_ent = upload(rent, c.stream);
        P.row_coef = upload(rcoef, c.stream);
        P.node_row = upload(node_row, c.stream);
    }
    MGRT_HIP(hipStreamSynchronize(c.stream));
}

StepOp &get_step_op(Ctx &c, int S, int prec, double dt) {
    auto &slot = c.ops[std::make_tuple(S, prec)];
    const HostMesh &hm = c.hm;
    if (!slot) {
        auto op = std::make_unique<StepOp>();
        op->S = S;
        op->prec = prec;
        op->n_tiles = (hm.n + S - 1) / S;
        std::vector<int64_t> sptr(op->n_tiles + 1, 0);
        std::vector<int32_t> sw(op->n_tiles, 0);
        for (int64_t t = 0; t < op->n_tiles; ++t) {
            int w = 0;
            for (int r = 0; r < S; ++r) {
                int64_t ii = t * S + r;
                if (ii >= hm.n) break;
                const int64_t i = hm.perm[ii];
                w = std::max<int>(w, (int)(hm.krow[i + 1] - hm.krow[i]));
            }
            sw[t] = w;
            op->wmax = std::max(op->wmax, w);
        }
        // narrow rows: one width for all slices (the kernel's unrolled width)
        const int wpad = pick_w(op->wmax);
        for (int64_t t = 0; t < op->n_tiles; ++t) {
            if (wpad > 0) sw[t] = wpad;
            sptr[t + 1] = sptr[t] + (int64_t)sw[t] * S;
        }
        op->wmean = (double)hm.krow[hm.n] / std::max<int64_t>(1, hm.n);
        std::vector<int32_t> cols(sptr[op->n_tiles]);
        parallel_for(op->n_tiles, [&](int64_t t0, int64_t t1) {
            for (int64_t t = t0; t < t1; ++t)
                for (int r = 0; r < S; ++r) {
                    const int64_t ii = t * S + r;
                    const int32_t self = (int32_t)std::min<int64_t>(ii, hm.n - 1);
                    const int64_t i = ii < hm.n ? hm.perm[ii] : -1;
                    const int64_t len = i >= 0 ? hm.krow[i + 1] - hm.krow[i] : 0;
                    for (int k = 0; k < sw[t]; ++k)
                        cols[sptr[t] + (int64_t)k * S + r] =
                            k < len ? hm.iperm[hm.kcol[hm.krow[i] + k]] : self;
                }
        }, 64);
        op->slice_ptr = upload(sptr, c.stream);
        op->slice_w = upload(sw, c.stream);
        op->cols = upload(cols, c.stream);
        MGRT_HIP(hipStreamSynchronize(c.stream));
        op->dt = -1;
        slot = std::move(op);
    }
    StepOp &op = *slot;
    if (op.dt != dt || op.eps_version != c.eps_version) {
        op.dt = dt;
        op.eps_version = c.eps_version;
        op.multi.reset();
        if (prec == 32) fill_values<float>(c, op);
        else fill_values<double>(c, op);
    }
    return op;
}

namespace {

struct TileLists {
    DevBuf own[5];
    const int32_t *ptr = nullptr, *loc = nullptr, *col = nullptr, *aux = nullptr;
    const double *w = nullptr;
};

// Group entries by tile (stable in the given order) and upload (into the arena when one
// is given).  Entries name nodes by the caller's id; they are placed by stepping order.
template <typename Ent, typename AuxFn, typename WFn>
TileLists make_lists(const std::vector<Ent> &ents, int S, int64_t n_tiles,
                     const std::vector<int32_t> &iperm, AuxFn aux, WFn wfn, hipStream_t s,
                     Arena *ar) {
    std::vector<int32_t> ptr(n_tiles + 1, 0);
    for (const auto &e : ents) ptr[iperm[e.node] / S + 1]++;
    for (int64_t t = 0; t < n_tiles; ++t) ptr[t + 1] += ptr[t];
    std::vector<int32_t> loc(ents.size()), col(ents.size()), ax(ents.size());
    std::vector<double> w(ents.size());
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (const auto &e : ents) {
        const int64_t ii = iperm[e.node];
        int32_t k = fill[ii / S]++;
        loc[k] = (int32_t)(ii % S);
        col[k] = e.col;
        ax[k] = aux(e);
        w[k] = wfn(e);
    }
    // keep non-empty allocations so that kernel pointers are always valid
    if (ents.empty()) {
        loc.push_back(0); col.push_back(-1); ax.push_back(0); w.push_back(0);
    }
    TileLists L;
    if (ar) {
        L.ptr = put(*ar, ptr);
        L.loc = put(*ar, loc);
        L.col = put(*ar, col);
        L.aux = put(*ar, ax);
        L.w = put(*ar, w);
        return L;
    }
    L.own[0] = upload(ptr, s);
    L.own[1] = upload(loc, s);
    L.own[2] = upload(col, s);
    L.own[3] = upload(ax, s);
    L.own[4] = upload(w, s);
    L.ptr = L.own[0].as<int32_t>();
    L.loc = L.own[1].as<int32_t>();
    L.col = L.own[2].as<int32_t>();
    L.aux = L.own[3].as<int32_t>();
    L.w = L.own[4].as<double>();
    return L;
}

struct HistEnt {
    int64_t node;
    int32_t col;
    int32_t idx;
};

// Launch variants of one stepping configuration: bit 0 non-temporal p_{l-1} / p_{l+1},
// bit 1 XCD-contiguous tile order, bit 2 packed per-node records, bit 3 (with bit 2, on
// operators with a dominant neighbour-offset pattern) speculative gathers.  All variants
// compute identical results.
constexpr int N_VARIANTS = 16;

int n_variants(int) { return N_VARIANTS; }

// The record mode of variant v for op: 0 plain, 1 packed, 2 packed + speculative.
int pk_mode(int v, const StepOp &op) {
    if (!((v >> 2) & 1)) return 0;
    return ((v >> 3) & 1) && op.spec_ok ? 2 : 1;
}

// Variants worth timing: bit 3 only with bit 2 and a dominant offset pattern.
bool variant_distinct(int v, const StepOp &op) {
    return !((v >> 3) & 1) || (((v >> 2) & 1) && op.spec_ok);
}

// Bounded non-zero scratch fields for the variant timing (all-zero fields time
// differently from the ones a run steps): x_i = (h(i) mod 2^16) / 2^16 - 1/2 for an
// integer hash h
template <typename T>
__global__ void k_fill_pattern(T *__restrict__ x, int64_t count, uint32_t salt) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= count) return;
    uint32_t h = (uint32_t)i * 2654435761u ^ salt;
    h ^= h >> 15;
    h *= 2246822519u;
    h ^= h >> 13;
    x[i] = (T)((double)(h & 0xffffu) * (1.0 / 65536.0) - 0.5);
}

// Time every variant on scratch state (pattern-filled fields, no loads or taps: the cost
// is the memory traffic of the step), two interleaved rounds of a few launches each, and
// return the variant with the fastest round and the per-launch times.
template <typename T>
Tuned tune_variant(Ctx &c, const StepOp &op, const StepArgs<T> &proto, int B, int W, int64_t grid) {
    const size_t slab = (size_t)proto.n * proto.B * sizeof(T);
    DevBuf sa(slab), sb(slab);
    const int64_t cnt = proto.n * proto.B;
    hipLaunchKernelGGL(k_fill_pattern<T>, dim3((cnt + 255) / 256), dim3(256), 0, c.stream,
                       static_cast<T *>(sa.p), cnt, 0x9e3779b9u);
    hipLaunchKernelGGL(k_fill_pattern<T>, dim3((cnt + 255) / 256), dim3(256), 0, c.stream,
                       static_cast<T *>(sb.p), cnt, 0x7f4a7c15u);
    MGRT_HIP(hipGetLastError());
    StepArgs<T> a = proto;
    a.parts = nullptr;
    a.hist = nullptr;
    a.acc = nullptr;
    a.vel_out = nullptr;
    a.inj_ptr = nullptr;
    a.pml_row = nullptr;
    hipEvent_t e0, e1;
    MGRT_HIP(hipEventCreate(&e0));
    MGRT_HIP(hipEventCreate(&e1));
    // two interleaved rounds over the variants; each variant keeps its faster round
    const int nv = n_variants(sizeof(T) == 4 ? 32 : 64);
    std::vector<float> vbest(nv, 1e30f);
    // enough launches per round that a round of a small problem lasts well above the
    // timer's resolution
    const int64_t nb = proto.n * proto.B;
    const int reps = nb > (1 << 22) ? 12 : (int)std::min<int64_t>(200, std::max<int64_t>(24, (1 << 22) / nb));
    for (int round = 0; round < 2; ++round) {
        for (int v = 0; v < nv; ++v) {
            if (!variant_distinct(v, op)) continue;
            a.xcd_map = (v >> 1) & 1;
            for (int r = 0; r < 2 + reps; ++r) {
                if (r == 2) MGRT_HIP(hipEventRecord(e0, c.stream));
                a.p = static_cast<T *>(r & 1 ? sb.p : sa.p);
                a.pm = static_cast<T *>(r & 1 ? sa.p : sb.p);
                launch_step<T>(a, B, W, v & 1, pk_mode(v, op), grid, c.stream);
            }
            MGRT_HIP(hipEventRecord(e1, c.stream));
            MGRT_HIP(hipEventSynchronize(e1));
            float ms = 0;
            MGRT_HIP(hipEventElapsedTime(&ms, e0, e1));
            vbest[v] = std::min(vbest[v], ms);
        }
    }
    Tuned t;
    t.variant = 0;
    for (int v = 1; v < nv; ++v)
        if (vbest[v] < vbest[t.variant]) t.variant = v;
    for (int v = 0; v < nv && v < 16; ++v) t.us[v] = variant_distinct(v, op) ? 1e3 * vbest[v] / reps : 0.0;
    t.best_us = t.us[t.variant];
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return t;
}

// The operator's part of the step arguments (no loads, taps or histories).
template <typename T>
StepArgs<T> op_args(const Ctx &c, const StepOp &op, int B) {
    StepArgs<T> a{};
    a.slice_ptr = op.slice_ptr.as<int64_t>();
    a.slice_w = op.slice_w.as<int32_t>();
    a.cols = op.cols.as<int32_t>();
    a.vals = op.vals.as<T>();
    a.beta = op.beta.as<T>();
    a.meta = op.meta.as<uint32_t>();
    a.n = c.hm.n;
    a.n_tiles = op.n_tiles;
    a.B = B;
    a.per_xcd = (op.n_tiles + 7) / 8;
    a.inv_dt = (T)(1.0 / op.dt);
    for (int k = 0; k < 8; ++k) a.spec_off[k] = op.spec_off[k];
    return a;
}

// Variant timings of (op, B), measured once per context.
template <typename T>
const Tuned &tuned_for(Ctx &c, const StepOp &op, int B) {
    const int W = pick_w(op.wmax);
    const auto key = std::make_tuple(op.prec, B, op.S, W);
    auto it = c.tuned.find(key);
    if (it == c.tuned.end()) {
        const int64_t grid = (op.n_tiles + 7) / 8 * 8;
        it = c.tuned.emplace(key, tune_variant<T>(c, op, op_args<T>(c, op, B), B, W, grid)).first;
    }
    return it->second;
}

template <typename T>
void run_batch_t(Ctx &c, StepOp &op, BatchRun &run) {
    const int S = op.S;
    const int64_t n = c.hm.n;
    hipStream_t s = c.stream;
    MGRT_REQUIRE(tile_nodes(op.prec, run.B) == S, MGRT_E_ARG, "batch width does not match operator tiles");
    if (run_multistep(c, op, run)) return;
    c.timing.steps_per_launch = 1;
    const std::vector<int32_t> &ip = c.hm.iperm;
    TileLists inj = make_lists(run.inj, S, op.n_tiles, ip, [](const Injection &e) { return e.sid; },
                               [](const Injection &e) { return e.weight; }, s, run.arena);
    TileLists rec = make_lists(run.rec, S, op.n_tiles, ip, [](const Record &e) { return e.dst; },
                               [](const Record &e) { return e.weight; }, s, run.arena);
    std::vector<HistEnt> hents;
    if (run.hist)
        for (size_t k = 0; k < run.hist_nodes.size(); ++k)
            hents.push_back(HistEnt{run.hist_nodes[k], 0, (int32_t)k});
    TileLists hl = make_lists(hents, S, op.n_tiles, ip, [](const HistEnt &e) { return e.idx; },
                              [](const HistEnt &) { return 0.0; }, s, run.arena);

    StepArgs<T> a{};
    a.slice_ptr = op.slice_ptr.as<int64_t>();
    a.slice_w = op.slice_w.as<int32_t>();
    a.cols = op.cols.as<int32_t>();
    a.vals = op.vals.as<T>();
    a.beta = op.beta.as<T>();
    a.meta = op.meta.as<uint32_t>();
    a.n = n;
    a.n_tiles = op.n_tiles;
    a.B = run.B;
    const int64_t grid = (op.n_tiles + 7) / 8 * 8;
    a.per_xcd = grid / 8;
    a.inj_ptr = inj.ptr;
    a.inj_loc = inj.loc;
    a.inj_col = inj.col;
    a.inj_sid = inj.aux;
    a.inj_w = inj.w;
    a.series = run.d_series;
    a.series_len = run.series_len;
    a.rec_ptr = rec.ptr;
    a.rec_loc = rec.loc;
    a.rec_col = rec.col;
    a.rec_dst = rec.aux;
    a.rec_w = rec.w;
    a.hist_ptr = hl.ptr;
    a.hist_loc = hl.loc;
    a.hist_idx = hl.aux;
    // histories: staged step-major for chunks of up to 64 steps (at most 256 MB)
    const int64_t hist_nh = run.hist ? (int64_t)run.hist_nodes.size() : 0;
    const int64_t hist_nser = hist_nh * run.B;
    int64_t hist_chunk = 0;
    DevBuf hist_own, hist_own2;
    T *hist_stage = nullptr, *hist_stage2 = nullptr;
    const bool dual = run.hist && run.hist_mode == 2;
    MGRT_REQUIRE(!dual || run.d_hist2, MGRT_E_ARG, "dual history without its second series");
    if (run.hist && hist_nh > 0) {
        hist_chunk = std::max<int64_t>(1, std::min<int64_t>(64, (256ll << 20) / (hist_nser * (int64_t)sizeof(T))));
        const size_t hb = (size_t)hist_chunk * hist_nser * sizeof(T);
        if (run.arena) {
            hist_stage = static_cast<T *>(run.arena->take(hb));
            if (dual) hist_stage2 = static_cast<T *>(run.arena->take(hb));
        } else {
            hist_own.alloc(hb);
            hist_stage = hist_own.as<T>();
            if (dual) {
                hist_own2.alloc(hb);
                hist_stage2 = hist_own2.as<T>();
            }
        }
    }
    a.hist = hist_chunk ? hist_stage : nullptr;
    a.hist2 = hist_chunk ? hist_stage2 : nullptr;
    a.hist_nh = hist_nh;
    a.hist_mode = run.hist_mode;
    a.inv_dt = (T)(1.0 / op.dt);
    a.acc = run.d_acc;
    if (run.d_series == nullptr) MGRT_REQUIRE(run.inj.empty(), MGRT_E_ARG, "loads without series");
    const int W = pick_w(op.wmax);

    // launch variant: tuned once per configuration and context (unless disabled or too small
    // to time), else packed records with speculative gathers where offered, linear order
    int variant = 12;
    MGRT_REQUIRE(run.launch >= 0 && run.launch <= n_variants(op.prec), MGRT_E_ARG,
                 "launch variant must be 0..16");
    for (int k = 0; k < 8; ++k) a.spec_off[k] = op.spec_off[k];
    if (run.launch > 0) {
        variant = run.launch - 1;
    } else {
        const auto key = std::make_tuple(op.prec, run.B, op.S, W);
        auto it = c.tuned.find(key);
        if (it != c.tuned.end()) {
            variant = it->second.variant;
        } else if (!run.arena && !(run.flags & MGRT_F_NO_TUNE) && run.n_steps >= 64 &&
                   n * (int64_t)run.B >= (1 << 14)) {
            const Tuned &t = tuned_for<T>(c, op, run.B);
            variant = t.variant;
            for (int v = 0; v < 16; ++v) c.timing.tune_us[v] = t.us[v];
        }
    }
    a.xcd_map = (variant >> 1) & 1;
    const bool nt = variant & 1;
    const int pk = pk_mode(variant, op);
    c.timing.variant = variant;

    const bool timing = !run.arena && (run.flags & MGRT_F_TIMING) != 0;
    std::vector<hipEvent_t> ev;
    if (timing) {
        ev.resize(2 * run.n_steps);
        for (auto &e : ev) MGRT_HIP(hipEventCreate(&e));
    }
    // split-field PML state of this run: q^(k) of the listed element-directions (zero at
    // the start), ping-pong, and the per-step load rows
    const PmlOp &P = op.pml;
    DevBuf q0, q1;
    T *q0p = nullptr, *q1p = nullptr;
    const size_t qbytes = (size_t)P.n_ent * run.B * sizeof(T);
    if (P.n_ent > 0) {
        if (run.arena) {
            q1p = static_cast<T *>(run.arena->take(qbytes));
            if (!run.d_q) {
                q0p = static_cast<T *>(run.arena->take(qbytes));
                const int64_t cnt = (int64_t)(qbytes / sizeof(T));
                hipLaunchKernelGGL(k_zero<T>, dim3((cnt + 255) / 256), dim3(256), 0, s, q0p, cnt);
            }
        } else {
            if (!run.d_q) {
                q0.alloc(qbytes);
                MGRT_HIP(hipMemsetAsync(q0.p, 0, qbytes, s));
                q0p = q0.as<T>();
            }
            q1.alloc(qbytes);
            q1p = q1.as<T>();
        }
        a.pml_row = P.node_row.as<int32_t>();
        a.pml_ptr = P.row_ptr.as<int32_t>();
        a.pml_ent = P.row_ent.as<int32_t>();
        a.pml_coef = P.row_coef.as<T>();
    }
    T *qa = run.d_q ? static_cast<T *>(run.d_q) : q0p, *qb_ = q1p;
    const int pvec = sizeof(T) == 4 ? (run.B >= 4 ? 4 : 1) : (run.B >= 2 ? 2 : 1);
    const int64_t g_ent = (P.n_ent * (run.B / pvec) + 255) / 256;
    T *bufA = static_cast<T *>(run.d_p);
    T *bufB = static_cast<T *>(run.d_pm);
    const int64_t nB = n * (int64_t)run.B;
    // Issue step l of the run: the PML update, the step and (flush) the history chunk
    // that ends with this step (its slot in the chunk).  With base != null, l is the offset
    // within a replayed run of steps and the kernels add *base to it.
    auto issue = [&](int64_t l, int64_t slot, const int64_t *base, bool flush) {
        a.p = bufA;
        a.pm = bufB;
        a.step_base = base;
        a.series_t = run.step0 + l;
        a.parts = run.d_parts ? run.d_parts + l * run.n_parts : nullptr;
        a.n_parts = run.n_parts;
        a.hist_t = slot;
        if (run.d_vel) {
            const int64_t vl = run.vel_reverse ? run.n_steps - 1 - l : l;
            a.vel = static_cast<const T *>(run.d_vel) + vl * nB;
            a.vel_stride = run.vel_reverse ? -nB : nB;
        }
        if (run.d_vel_out) {
            a.vel_out = static_cast<T *>(run.d_vel_out) + l * nB;
            a.vel_out_stride = nB;
        }
        if (P.n_ent > 0) {
            // the step reads q_{l-1/2} (qa) for its load; the update writes q_{l+1/2} (qb_)
            a.pml_q = qa;
            launch_pml_q<T>(c.hm.d, pvec, P, run.B, g_ent, bufA, qa, qb_, s);
        }
        launch_step<T>(a, run.B, W, nt, pk, grid, s);
        if (P.n_ent > 0) std::swap(qa, qb_);
        if (flush) {
            hipLaunchKernelGGL(k_hist_flush<T>, dim3((hist_nser + 63) / 64), dim3(256), 0, s,
                               static_cast<const T *>(hist_stage), hist_nser, (int)(slot + 1),
                               static_cast<T *>(run.d_hist), run.hist_len, run.hist_off + (l - slot),
                               (int)run.reverse_hist, base);
            if (dual)
                hipLaunchKernelGGL(k_hist_flush<T>, dim3((hist_nser + 63) / 64), dim3(256), 0, s,
                                   static_cast<const T *>(hist_stage2), hist_nser, (int)(slot + 1),
                                   static_cast<T *>(run.d_hist2), run.hist_len, run.hist_off + (l - slot),
                                   (int)run.reverse_hist, base);
        }
        std::swap(bufA, bufB);
    };
    // Runs of G steps (one history chunk, an even count so that the state and PML buffers
    // are back in place after each) are captured once into a graph of kernel nodes and
    // replayed; the remaining steps, a stream that cannot be captured or MGRT_F_NO_GRAPH
    // take direct launches.  With MGRT_F_TIMING one pair of events brackets all replays
    // (kernels plus the gaps between graph nodes) and one pair every direct launch.
    int64_t l0 = 0;
    const int64_t G = hist_chunk ? hist_chunk : 64;
    if (!run.arena && !(run.flags & MGRT_F_NO_GRAPH) && G % 2 == 0 && run.n_steps >= 2 * G) {
        DevBuf dbase(sizeof(int64_t));
        int64_t *base = dbase.as<int64_t>();
        hipGraph_t graph = nullptr;
        if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) == hipSuccess) {
            try {
                for (int64_t j = 0; j < G; ++j) issue(j, j, base, hist_chunk != 0 && j == G - 1);
                hipLaunchKernelGGL(k_step_base, dim3(1), dim3(64), 0, s, base, G, 1);
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
            const int64_t nrep = run.n_steps / G;
            hipLaunchKernelGGL(k_step_base, dim3(1), dim3(64), 0, s, base, (int64_t)0, 0);
            if (timing) MGRT_HIP(hipEventRecord(ev[0], s));
            hipError_t le = hipSuccess;
            for (int64_t r = 0; r < nrep && le == hipSuccess; ++r) le = hipGraphLaunch(exec, s);
            if (timing && le == hipSuccess) le = hipEventRecord(ev[1], s);
            const hipError_t se = hipStreamSynchronize(s);
            (void)hipGraphExecDestroy(exec);
            MGRT_HIP(le);
            MGRT_HIP(se);
            l0 = nrep * G;
            c.timing.graph_steps += l0;
            if (timing) {
                float ms = 0;
                MGRT_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
                c.timing.step_ms_total += ms;
            }
        } else {
            (void)hipGetLastError();
        }
    }
    for (int64_t l = l0; l < run.n_steps; ++l) {
        const int64_t slot = hist_chunk ? l % hist_chunk : 0;
        if (timing) MGRT_HIP(hipEventRecord(ev[2 * l], s));
        issue(l, slot, nullptr, hist_chunk && (slot == hist_chunk - 1 || l == run.n_steps - 1));
        if (timing) MGRT_HIP(hipEventRecord(ev[2 * l + 1], s));
    }
    MGRT_HIP(hipGetLastError());
    // the caller's PML state holds q_{N-1/2}
    if (run.d_q && P.n_ent > 0 && qa != run.d_q)
        MGRT_HIP(hipMemcpyAsync(run.d_q, qa, qbytes, hipMemcpyDeviceToDevice, s));
    // leave d_p = p_N, d_pm = p_{N-1}
    run.d_p = bufA;
    run.d_pm = bufB;
    MGRT_HIP(hipStreamSynchronize(s));
    c.timing.step_launches += run.n_steps;
    {
        const double esz = sizeof(T);
        const double words = 3 + (run.d_vel_out ? 1 : 0) + (run.d_vel ? 1 : 0);
        const int NV = c.hm.d + 1;
        // PML: q read and written once (the step's gathers of q_{l-1/2} are counted once
        // more), entry and row coefficients, the node -> row map
        const double pml_bytes =
            P.n_ent > 0 ? 3.0 * esz * (double)P.n_ent * run.B + (double)P.n_ent * (NV * (4 + esz) + esz) +
                              (double)P.nnz * (4 + esz) + 4.0 * (P.n_rows + 1) + 4.0 * n
                        : 0.0;
        const double per_launch = words * esz * (double)n * run.B + op.oper_bytes +
                                  (run.d_acc ? 16.0 * n : 0.0) + pml_bytes;
        c.timing.step_bytes += per_launch * run.n_steps;
        c.timing.batch = run.B;
        c.timing.ell_width = op.wmax;
        c.timing.ell_mean_width = op.wmean;
    }
    if (timing) {
        double tot = 0;
        for (int64_t l = l0; l < run.n_steps; ++l) {
            float ms = 0;
            MGRT_HIP(hipEventElapsedTime(&ms, ev[2 * l], ev[2 * l + 1]));
            tot += ms;
        }
        c.timing.step_ms_total += tot;
        for (auto &e : ev) (void)hipEventDestroy(e);
    }
}

}  // namespace

// Batch width for n_cols independent columns.  A requested width is checked and used.
// Otherwise, for problems large enough to time (n * B >= 2^20 node-columns), every
// power-of-two width from a quarter of the default up to the column count is timed (its
// fastest launch variant on scratch state, once per context) and the width with the
// smallest estimated run time ceil(n_cols / B) * t_launch(B) is taken (ties: the wider);
// small problems and MGRT_F_NO_TUNE keep the default rule of choose_batch.  The
// candidates and their per-launch times are reported in mgrt_timing.tune_b / tune_b_us.
int pick_batch(Ctx &c, int prec, int64_t n_cols, int requested, double dt, int flags) {
    const int rule = choose_batch(prec, n_cols, requested);
    if (requested > 0 || (flags & MGRT_F_NO_TUNE) || c.hm.n * (int64_t)rule < (1 << 20)) return rule;
    int top = 1;
    while (top < n_cols && top < 128) top <<= 1;
    const auto key = std::make_tuple(prec, (int64_t)top);
    const auto hit = c.batch_tuned.find(key);
    if (hit != c.batch_tuned.end()) return hit->second;
    std::vector<int> cands;
    for (int b = std::max(1, rule / 4); b <= top; b <<= 1)
        if (!(prec == 32 && b == 2)) cands.push_back(b);
    // estimated run time per step: ceil(n_cols / B) launches of the width's fastest variant
    std::vector<double> est;
    int k = 0;
    for (int b : cands) {
        StepOp &op = get_step_op(c, tile_nodes(prec, b), prec, dt);
        const double us = prec == 32 ? tuned_for<float>(c, op, b).best_us : tuned_for<double>(c, op, b).best_us;
        est.push_back((double)((n_cols + b - 1) / b) * us);
        if (k < 6) {
            c.timing.tune_b[k] = b;
            c.timing.tune_b_us[k] = us;
            ++k;
        }
    }
    // the widest width within 2% of the smallest estimate: a narrower width carries costs
    // per batch that the launch timing does not see (a graph capture, buffers, trace
    // copies; in the Jacobian more history flushes, and a working set that shares the
    // Infinity Cache with the transforms overlapping the run)
    const double lo = *std::min_element(est.begin(), est.end());
    int best = rule;
    for (size_t i = 0; i < cands.size(); ++i)
        if (est[i] <= 1.02 * lo) best = cands[i];
    c.batch_tuned[key] = best;
    // the launch variants timed for the chosen width
    const StepOp &bop = get_step_op(c, tile_nodes(prec, best), prec, dt);
    const Tuned &bt = prec == 32 ? tuned_for<float>(c, bop, best) : tuned_for<double>(c, bop, best);
    for (int v = 0; v < 16; ++v) c.timing.tune_us[v] = bt.us[v];
    return best;
}

int64_t pml_entries(const Ctx &c) {
    if (!c.have_pml) return 0;
    int64_t ne = 0;
    for (double z : c.pml_zeta) ne += z > 0;
    return ne;
}

void run_batch(Ctx &c, StepOp &op, BatchRun &run) {
    if (op.prec == 32) run_batch_t<float>(c, op, run);
    else run_batch_t<double>(c, op, run);
}

void run_plain(Ctx &c, double dt, int64_t n_steps, const Stencil &src, const double *h_g,
               const std::vector<Record> &rec, double *d_parts, int64_t n_parts, int flags) {
    const HostMesh &hm = c.hm;
    hipStream_t s = c.stream;
    MGRT_REQUIRE(rec.size() <= 32, MGRT_E_ARG, "plain stepper records at most 32 taps");
    DevBuf bp(hm.n * sizeof(double)), bq(hm.n * sizeof(double));
    MGRT_HIP(hipMemsetAsync(bp.p, 0, bp.bytes, s));
    MGRT_HIP(hipMemsetAsync(bq.p, 0, bq.bytes, s));
    PlainArgs a{};
    a.row = c.dm.krow.as<int64_t>();
    a.col = c.dm.kcol.as<int32_t>();
    a.val = c.dm.kval.as<double>();
    a.kdiag = c.dm.kdiag.as<double>();
    a.M = c.dM.as<double>();
    a.r = c.dR.as<double>();
    a.dt = dt;
    a.n = hm.n;
    for (int q = 0; q < 4; ++q) {
        a.src_node[q] = q <= hm.d ? src.node[q] : -1;
        a.src_w[q] = q <= hm.d ? src.w[q] : 0.0;
    }
    a.n_taps = (int32_t)rec.size();
    for (size_t q = 0; q < rec.size(); ++q) {
        a.tap_node[q] = (int32_t)rec[q].node;
        a.tap_dst[q] = rec[q].dst;
        a.tap_w[q] = rec[q].weight;
    }
    const bool timing = (flags & MGRT_F_TIMING) != 0;
    std::vector<hipEvent_t> ev;
    if (timing) {
        ev.resize(2 * n_steps);
        for (auto &e : ev) MGRT_HIP(hipEventCreate(&e));
    }
    const int64_t grid = (hm.n + 255) / 256;
    double *A = bp.as<double>(), *Bq = bq.as<double>();
    for (int64_t l = 0; l < n_steps; ++l) {
        a.p = A;
        a.pm = Bq;
        a.g = h_g[l];
        a.parts = d_parts + l * n_parts;
        if (timing) MGRT_HIP(hipEventRecord(ev[2 * l], s));
        hipLaunchKernelGGL(k_step_plain, dim3(grid), dim3(256), 0, s, a);
        if (timing) MGRT_HIP(hipEventRecord(ev[2 * l + 1], s));
        std::swap(A, Bq);
    }
    MGRT_HIP(hipGetLastError());
    MGRT_HIP(hipStreamSynchronize(s));
    c.timing.step_launches += n_steps;
    if (timing) {
        double tot = 0;
        for (int64_t l = 0; l < n_steps; ++l) {
            float ms = 0;
            MGRT_HIP(hipEventElapsedTime(&ms, ev[2 * l], ev[2 * l + 1]));
            tot += ms;
        }
        c.timing.step_ms_total += tot;
        for (auto &e : ev) (void)hipEventDestroy(e);
    }
}

}  // namespace mgrt
