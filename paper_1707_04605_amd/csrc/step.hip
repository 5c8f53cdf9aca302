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
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <type_traits>

#include "mgrt_internal.hpp"

namespace mgrt {

template <typename T, int V>
struct VecT {
    typedef T type __attribute__((ext_vector_type(V)));
};

template <typename T>
struct StepArgs {
    const T *__restrict__ p;      // p_l
    T *__restrict__ pm;           // in p_{l-1}, out p_{l+1}
    const int64_t *__restrict__ slice_ptr;
    const int32_t *__restrict__ slice_w;
    const int32_t *__restrict__ cols;
    const T *__restrict__ vals;
    const T *__restrict__ beta;
    int64_t n;
    int64_t n_tiles;
    int64_t B;                    // row stride (columns)
    int64_t per_xcd;              // gridDim.x / 8
    int32_t xcd_map;              // 1: deal contiguous tile ranges to the 8 XCDs
    // nodal loads: p+[node][col] += w * series[sid][t]
    const int32_t *__restrict__ inj_ptr;
    const int32_t *__restrict__ inj_loc;
    const int32_t *__restrict__ inj_col;
    const int32_t *__restrict__ inj_sid;
    const double *__restrict__ inj_w;
    const double *__restrict__ series;
    int64_t series_len;
    int64_t series_t;
    // receiver taps: parts[dst] = w * p+[node][col]
    const int32_t *__restrict__ rec_ptr;
    const int32_t *__restrict__ rec_loc;
    const int32_t *__restrict__ rec_col;
    const int32_t *__restrict__ rec_dst;
    const double *__restrict__ rec_w;
    double *__restrict__ parts;
    // coarse-node histories, staged step-major for a chunk of steps:
    // hist[(hist_t * hist_nh + c) * B + col] (hist_t = the step's slot in the chunk);
    // k_hist_flush moves each chunk to the time-contiguous series
    const int32_t *__restrict__ hist_ptr;
    const int32_t *__restrict__ hist_loc;
    const int32_t *__restrict__ hist_idx;
    T *__restrict__ hist;
    T *__restrict__ hist2;        // mode 2: the velocity's stage (the same layout)
    int64_t hist_nh;
    int64_t hist_t;
    int32_t hist_mode;            // 0: p+,  1: -(p+ - p)/dt,  2: p+ to hist and -(p+ - p)/dt to hist2
    T inv_dt;
    // adjoint correlation: acc[node] += sum_col p+[node][col] * vel[node][col]
    const T *__restrict__ vel;
    double *__restrict__ acc;
    // full velocity field out: vel_out[node][col] = -(p+ - p)/dt
    T *__restrict__ vel_out;
    // split-field PML load of node rows in the layer (pml_row >= 0):
    //   p+[node][:] += sum_{k in row} pml_coef[k] * pml_q[pml_ent[k]][:]   (q_{l-1/2})
    const int32_t *__restrict__ pml_row;
    const int32_t *__restrict__ pml_ptr;
    const int32_t *__restrict__ pml_ent;
    const T *__restrict__ pml_coef;
    const T *__restrict__ pml_q;
    // packed per-node records (PK launches): beta, cols, coefficients
    const uint32_t *__restrict__ meta;
    // replayed launches (a captured run of steps): the per-step quantities are this
    // launch's offsets plus base = *step_base steps, read from device memory, which a
    // small kernel at the end of every replay advances; null for direct launches
    const int64_t *__restrict__ step_base;
    int64_t n_parts;              // parts row per step
    int64_t vel_stride;           // vel elements per step (negative: read backwards)
    int64_t vel_out_stride;       // vel_out elements per step
    // speculative gathers (SP launches): the operator's most common neighbour offsets
    // (column minus node, padded entries 0), used to issue the gathers before the record
    int32_t spec_off[8];
};

// Everything after the stencil sum: the PML load and nodal loads join the increment, then
// p_{l+1} = p_l + inc feeds the receiver taps, coarse-node histories, the adjoint
// correlation, the velocity output and the store.
template <typename T, int VEC, int LPN, bool NT>
__device__ __forceinline__ void step_tail(const StepArgs<T> &a, int64_t tile, int64_t node, int ln,
                                          int sub, int64_t off,
                                          const typename VecT<T, VEC>::type &pc,
                                          typename VecT<T, VEC>::type inc) {
    typedef typename VecT<T, VEC>::type V;
    constexpr int64_t BW = VEC * LPN;                 // row stride = batch width
    const int64_t sb = a.step_base ? a.step_base[0] : 0;
    if (a.pml_row) {
        const int32_t pr = a.pml_row[node];
        if (pr >= 0) {
            const int32_t k0 = a.pml_ptr[pr], k1 = a.pml_ptr[pr + 1];
            // unrolled so that several entry -> q gather chains are in flight
#pragma unroll 4
            for (int32_t k = k0; k < k1; ++k)
                inc += a.pml_coef[k] *
                       *reinterpret_cast<const V *>(a.pml_q + (int64_t)a.pml_ent[k] * BW + (int64_t)sub * VEC);
        }
    }

    // nodal loads of this tile (sources, adjoint residuals, impulses)
    if (a.inj_ptr) {
        const int e0 = a.inj_ptr[tile], e1 = a.inj_ptr[tile + 1];
        for (int e = e0; e < e1; ++e) {
            if (a.inj_loc[e] != ln) continue;
            const int q = a.inj_col[e] - sub * VEC;
            if (q < 0 || q >= VEC) continue;
            const T add = (T)(a.inj_w[e] * a.series[(int64_t)a.inj_sid[e] * a.series_len + a.series_t + sb]);
#pragma unroll
            for (int u = 0; u < VEC; ++u)
                if (u == q) inc[u] += add;
        }
    }
    const V out = pc + inc;
    // receiver taps
    if (a.parts) {
        const int e0 = a.rec_ptr[tile], e1 = a.rec_ptr[tile + 1];
        for (int e = e0; e < e1; ++e) {
            if (a.rec_loc[e] != ln) continue;
            const int q = a.rec_col[e] - sub * VEC;
            if (q < 0 || q >= VEC) continue;
            T val = out[0];
#pragma unroll
            for (int u = 1; u < VEC; ++u)
                if (u == q) val = out[u];
            a.parts[sb * a.n_parts + a.rec_dst[e]] = a.rec_w[e] * (double)val;
        }
    }
    // coarse-node histories
    if (a.hist) {
        const int e0 = a.hist_ptr[tile], e1 = a.hist_ptr[tile + 1];
        for (int e = e0; e < e1; ++e) {
            if (a.hist_loc[e] != ln) continue;
            const int64_t ho = (a.hist_t * a.hist_nh + a.hist_idx[e]) * BW + (int64_t)sub * VEC;
            const V vel = -inc * a.inv_dt;
            *reinterpret_cast<V *>(a.hist + ho) = a.hist_mode == 1 ? vel : out;
            if (a.hist_mode == 2) *reinterpret_cast<V *>(a.hist2 + ho) = vel;
        }
    }
    // zero-lag correlation with a stored forward field (adjoint sweep)
    if (a.acc) {
        const V vv = *reinterpret_cast<const V *>(a.vel + sb * a.vel_stride + off);
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < VEC; ++u) s += (double)out[u] * (double)vv[u];
#pragma unroll
        for (int o = LPN / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
        if (sub == 0) a.acc[node] += s;
    }
    if (a.vel_out) *reinterpret_cast<V *>(a.vel_out + sb * a.vel_out_stride + off) = -inc * a.inv_dt;
    if constexpr (NT) __builtin_nontemporal_store(out, reinterpret_cast<V *>(a.pm + off));
    else *reinterpret_cast<V *>(a.pm + off) = out;
}

// PK: the node's beta, coefficient and column ids come from one packed record of 32-bit
// words (FP64 values as two words); lane j of the node's lane group loads words j,
// j + LPN, j + 2 LPN, ... and the group shares them through cross-lane shuffles instead
// of every lane loading all of them.  The record holds one coefficient: on structured
// meshes every interior node's W off-diagonal coefficients are the same value (bit for
// bit in the working precision; the stiffness matrix does not depend on eps).  Nodes
// whose coefficients differ (boundary rows, unstructured meshes) carry the top bit of
// their first column id and read their W coefficients from the slice arrays instead.
template <typename T, int W>
struct PackedRecord {
    static constexpr int VW = sizeof(T) / 4;              // words per value
    static constexpr int words = 2 * VW + W;              // beta, coefficient, cols
};
constexpr uint32_t REC_GENERAL = 0x80000000u;             // flag on the first column id

// word K of a node's record from the lanes that loaded it (lane K % LPN of the node's
// group, slot K / LPN).  With DPP (FP32 records; measured slower for the longer FP64 ones)
// the broadcast stays in the VALU: quad_perm for groups of 2 or 4 lanes, a row broadcast
// for 16, two row broadcasts and a select for 8 (two nodes share a 16-lane row); else a
// cross-lane shuffle within the group.
template <int LPN, int NWL, int K, bool DPP>
__device__ __forceinline__ uint32_t record_word(const uint32_t (&wl)[NWL]) {
    constexpr int slot = K / LPN, src = K % LPN;
    if constexpr (LPN == 1) {
        return wl[K];
    } else if constexpr (DPP && LPN == 2) {
        constexpr int qp = src | (src << 2) | ((2 + src) << 4) | ((2 + src) << 6);
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)wl[slot], qp, 0xF, 0xF, false);
    } else if constexpr (DPP && LPN == 4) {
        constexpr int qp = src | (src << 2) | (src << 4) | (src << 6);
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)wl[slot], qp, 0xF, 0xF, false);
    } else if constexpr (DPP && LPN == 8) {
        const int lo = __builtin_amdgcn_update_dpp(0, (int)wl[slot], 0x150 + src, 0xF, 0xF, false);
        const int hi = __builtin_amdgcn_update_dpp(0, (int)wl[slot], 0x150 + 8 + src, 0xF, 0xF, false);
        return (uint32_t)((threadIdx.x & 8) ? hi : lo);
    } else if constexpr (DPP && LPN == 16) {
        return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)wl[slot], 0x150 + src, 0xF, 0xF, false);
    } else {
        return (uint32_t)__shfl((int)wl[slot], src, LPN);
    }
}

template <int K, int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (K < N) {
        f(std::integral_constant<int, K>{});
        static_for<K + 1, N>(f);
    }
}

template <typename T>
__device__ __forceinline__ T packed_value(uint32_t lo, uint32_t hi) {
    if constexpr (sizeof(T) == 4) {
        (void)hi;
        return __uint_as_float(lo);
    } else {
        return __hiloint2double((int)hi, (int)lo);
    }
}
template <typename T, int VEC, int LPN, int W, bool NT, bool PK = false, bool SP = false>
__global__ __launch_bounds__(256) void k_step(const StepArgs<T> a) {
    typedef typename VecT<T, VEC>::type V;
    constexpr int S = 256 / LPN;
    const int bid = blockIdx.x;
    // XCD-contiguous order (consecutive workgroup ids go to different XCDs) or linear
    const int64_t tile = a.xcd_map ? (int64_t)(bid & 7) * a.per_xcd + (bid >> 3) : (int64_t)bid;
    if (tile >= a.n_tiles) return;
    const int ln = threadIdx.x / LPN;
    const int sub = threadIdx.x % LPN;
    const int64_t node = tile * S + ln;
    if (node >= a.n) return;

    // the row stride is the batch width VEC * LPN (a power of two: shifts, not multiplies)
    constexpr int64_t BW = VEC * LPN;
    const int64_t off = node * BW + (int64_t)sub * VEC;
    // p_{l-1} is read once and p_{l+1} written once: optionally streamed past the caches
    auto load_state = [&](V &pc_, V &pv_) {
        pc_ = *reinterpret_cast<const V *>(a.p + off);
        if constexpr (NT) pv_ = __builtin_nontemporal_load(reinterpret_cast<const V *>(a.pm + off));
        else pv_ = *reinterpret_cast<const V *>(a.pm + off);
    };
    if constexpr (PK && W > 0) {
        constexpr int MW = PackedRecord<T, W>::words;
        constexpr int VW = PackedRecord<T, W>::VW;
        constexpr int NWL = (MW + LPN - 1) / LPN;                 // words per lane
        // the record first: the neighbour gathers wait for it alone while p_l and p_{l-1}
        // of the node are still in flight
        const uint32_t *rec = a.meta + node * MW;
        uint32_t wl[NWL];
#pragma unroll
        for (int j = 0; j < NWL; ++j) wl[j] = sub + j * LPN < MW ? rec[sub + j * LPN] : 0u;
        V pc, pv;
        load_state(pc, pv);
        V pj[W];
        if constexpr (SP) {
            // SP: gather at node + spec_off[k] (clamped into the array) right away; the
            // record's columns decide below whether these are the right rows
#pragma unroll
            for (int k = 0; k < W; ++k) {
                int64_t ck = node + a.spec_off[k];
                ck = ck < 0 ? 0 : (ck >= a.n ? a.n - 1 : ck);
                pj[k] = *reinterpret_cast<const V *>(a.p + ck * BW + (int64_t)sub * VEC);
            }
        }
        __builtin_amdgcn_sched_barrier(0);       // keep the state loads ahead of that wait
        // words K and K + 1 (the second only for FP64) as one value of type T
        auto value = [&](auto kc) -> T {
            constexpr int K = decltype(kc)::value;
            if constexpr (VW == 2)
                return packed_value<T>(record_word<LPN, NWL, K, false>(wl),
                                       record_word<LPN, NWL, K + 1, false>(wl));
            else
                return packed_value<T>(record_word<LPN, NWL, K, true>(wl), 0u);
        };
        const T be = value(std::integral_constant<int, 0>{});
        const T cu = value(std::integral_constant<int, VW>{});
        V inc = be * (pc - pv);
        int c[W];
        T v[W];
        static_for<0, W>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            c[k] = (int)record_word<LPN, NWL, 2 * VW + k, VW == 1>(wl);
        });
        const bool general = ((uint32_t)c[0] & REC_GENERAL) != 0;
        c[0] = (int)((uint32_t)c[0] & ~REC_GENERAL);
#pragma unroll
        for (int k = 0; k < W; ++k) v[k] = cu;
        if (general) {
            const int64_t sp = a.slice_ptr[tile] + ln;
#pragma unroll
            for (int k = 0; k < W; ++k) v[k] = a.vals[sp + (int64_t)k * S];
        }
        bool regather = true;
        if constexpr (SP) {
            regather = false;
#pragma unroll
            for (int k = 0; k < W; ++k) regather |= (int64_t)c[k] != node + a.spec_off[k];
        }
        if (regather) {
#pragma unroll
            for (int k = 0; k < W; ++k)
                pj[k] = *reinterpret_cast<const V *>(a.p + (int64_t)c[k] * BW + (int64_t)sub * VEC);
        }
#pragma unroll
        for (int k = 0; k < W; ++k) inc += v[k] * (pj[k] - pc);
        step_tail<T, VEC, LPN, NT>(a, tile, node, ln, sub, off, pc, inc);
        return;
    }
    V pc, pv;
    load_state(pc, pv);
    const int64_t sp = a.slice_ptr[tile] + ln;
    V inc = a.beta[node] * (pc - pv);
    if constexpr (W > 0) {
        // every slice is padded to exactly W entries (padding: own row, value 0), so the
        // gathers are branch-free and all of them are in flight together
        int c[W];
        T v[W];
        V pj[W];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            c[k] = a.cols[sp + (int64_t)k * S];
            v[k] = a.vals[sp + (int64_t)k * S];
        }
#pragma unroll
        for (int k = 0; k < W; ++k)
            pj[k] = *reinterpret_cast<const V *>(a.p + (int64_t)c[k] * BW + (int64_t)sub * VEC);
#pragma unroll
        for (int k = 0; k < W; ++k) inc += v[k] * (pj[k] - pc);
    } else {
        const int w = a.slice_w[tile];
        for (int k = 0; k < w; ++k) {
            const int cj = a.cols[sp + (int64_t)k * S];
            const T vk = a.vals[sp + (int64_t)k * S];
            const V pj = *reinterpret_cast<const V *>(a.p + (int64_t)cj * BW + (int64_t)sub * VEC);
            inc += vk * (pj - pc);
        }
    }
    step_tail<T, VEC, LPN, NT>(a, tile, node, ln, sub, off, pc, inc);
}

// One chunk of staged histories (count <= 64 steps, stage[s][series], series = c * B + col)
// to the time-contiguous series hist[series][t], t = t_base + s (hist_len - 1 - t when
// reverse), through a 64 x 64 LDS tile: reads coalesced over series, writes over time.
template <typename T>
__global__ __launch_bounds__(256) void k_hist_flush(const T *__restrict__ stage, int64_t nser, int count,
                                                    T *__restrict__ hist, int64_t hist_len, int64_t t_base,
                                                    int reverse, const int64_t *__restrict__ step_base) {
    __shared__ T tile[64][65];
    if (step_base) t_base += step_base[0];
    const int64_t ser0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int st = ty; st < count; st += 4)
        tile[tx][st] = ser0 + tx < nser ? stage[(int64_t)st * nser + ser0 + tx] : T(0);
    __syncthreads();
    if (tx >= count) return;
    const int64_t t = t_base + tx;
    const int64_t pos = reverse ? hist_len - 1 - t : t;
    for (int r = ty; r < 64; r += 4)
        if (ser0 + r < nser) hist[(ser0 + r) * hist_len + pos] = tile[r][tx];
}

// x[0 .. count) = 0 (a fill kernel: no memset node where callers capture the stream).
template <typename T>
__global__ void k_zero(T *__restrict__ x, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < count) x[i] = T(0);
}

// Step base of replayed launches: base = value (set) or base += value (advance).
__global__ void k_step_base(int64_t *__restrict__ base, int64_t value, int advance) {
    if (blockIdx.x == 0 && threadIdx.x == 0) base[0] = advance ? base[0] + value : value;
}

// Split-field PML: q_{l+1/2} = (1 - dt zeta) q_{l-1/2} + dt d_k p_l|_T for every listed
// element-direction; VEC columns per lane, LPN = B / VEC lanes per entry.  Each entry's
// record [its NV nodes, dt d_k phi_a|_T for the NV nodes, 1 - dt zeta] (values as 1 or 2
// 32-bit words) is contiguous, so a workgroup's records are one contiguous range: the
// lanes copy it to LDS one word each and read their entry's words from there.
template <typename T, int VEC, int NV>
__global__ __launch_bounds__(256) void k_pml_q(const uint32_t *__restrict__ ent_rec, int64_t n_ent,
                                               int64_t B, const T *__restrict__ p,
                                               const T *__restrict__ q, T *__restrict__ qn) {
    typedef typename VecT<T, VEC>::type V;
    constexpr int VW = sizeof(T) / 4;
    constexpr int MW = NV + (NV + 1) * VW;
    __shared__ uint32_t rec[256 * MW];
    const int lpn = (int)(B / VEC);
    const int per_block = 256 / lpn;
    const int64_t e0 = (int64_t)blockIdx.x * per_block;
    const int64_t words = std::min<int64_t>(per_block, n_ent - e0) * MW;
    for (int64_t w = threadIdx.x; w < words; w += 256) rec[w] = ent_rec[e0 * MW + w];
    __syncthreads();
    const int le = threadIdx.x / lpn;
    const int64_t e = e0 + le;
    if (e >= n_ent) return;
    const int64_t off = (int64_t)(threadIdx.x % lpn) * VEC;
    const uint32_t *r = rec + le * MW;
    auto value = [&](int k) -> T {
        if constexpr (VW == 1) return __uint_as_float(r[k]);
        else return __hiloint2double((int)r[k + 1], (int)r[k]);
    };
    V s = value(NV + NV * VW) * *reinterpret_cast<const V *>(q + e * B + off);
#pragma unroll
    for (int a = 0; a < NV; ++a)
        s += value(NV + a * VW) * *reinterpret_cast<const V *>(p + (int64_t)r[a] * B + off);
    // streamed out: the step reads q_{l+1/2} only in the next launch, and dirty lines left
    // in the XCDs' L2 caches would be written back at the kernel boundary
    __builtin_nontemporal_store(s, reinterpret_cast<V *>(qn + e * B + off));
}

// ------------------------------------------------------------------------------------
// Plain per-source FP64 CSR stepper: one thread per node, no batching, the recurrence
// written directly from M, r and K.  Reference point for the batched kernels.
struct PlainArgs {
    const double *__restrict__ p;
    double *__restrict__ pm;
    const int64_t *__restrict__ row;
    const int32_t *__restrict__ col;
    const double *__restrict__ val;
    const double *__restrict__ kdiag;
    const double *__restrict__ M;
    const double *__restrict__ r;
    double dt;
    int64_t n;
    int32_t src_node[4];
    double src_w[4];
    double g;                     // (w_l - w_{l-1}) / dt
    int32_t n_taps;
    int32_t tap_node[32];
    int32_t tap_dst[32];
    double tap_w[32];
    double *__restrict__ parts;
};

__global__ __launch_bounds__(256) void k_step_plain(const PlainArgs a) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    double kp = a.kdiag[i] * a.p[i];
    for (int64_t k = a.row[i]; k < a.row[i + 1]; ++k) kp += a.val[k] * a.p[a.col[k]];
    double f = 0.0;
    for (int q = 0; q < 4; ++q)
        if (a.src_node[q] == i) f += a.src_w[q];
    const double Mi = a.M[i], h = 0.5 * a.dt * a.r[i];
    const double pn = (2.0 * Mi * a.p[i] - (Mi - h) * a.pm[i] - a.dt * a.dt * kp + a.dt * a.dt * f * a.g) / (Mi + h);
    a.pm[i] = pn;
    for (int q = 0; q < a.n_taps; ++q)
        if (a.tap_node[q] == i) a.parts[a.tap_dst[q]] = a.tap_w[q] * pn;
}

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

// packed-record launch where it exists (FP32, record of at most two words per lane),
// else the plain one (identical results)
// pk: 0 = per-slice coefficient arrays, 1 = packed records, 2 = packed records with
// speculative gathers.  The packed launches exist for FP32 and FP64 records of at most
// eight words per lane; elsewhere the plain one runs (identical results).
template <typename T, int VEC, int LPN, int W, bool NT>
void launch_step_pk(const StepArgs<T> &a, int pk, int64_t grid, hipStream_t s) {
    if constexpr (PackedRecord<T, W>::words <= 8 * LPN) {
        if (pk == 2) {
            hipLaunchKernelGGL((k_step<T, VEC, LPN, W, NT, true, true>), dim3(grid), dim3(256), 0, s, a);
            return;
        }
        if (pk == 1) {
            hipLaunchKernelGGL((k_step<T, VEC, LPN, W, NT, true>), dim3(grid), dim3(256), 0, s, a);
            return;
        }
    }
    (void)pk;
    hipLaunchKernelGGL((k_step<T, VEC, LPN, W, NT, false>), dim3(grid), dim3(256), 0, s, a);
}

template <typename T, int VEC, int LPN, bool NT>
void launch_step_w(const StepArgs<T> &a, int W, int pk, int64_t grid, hipStream_t s) {
    switch (W) {
    case 4: launch_step_pk<T, VEC, LPN, 4, NT>(a, pk, grid, s); break;
    case 6: launch_step_pk<T, VEC, LPN, 6, NT>(a, pk, grid, s); break;
    case 8: hipLaunchKernelGGL((k_step<T, VEC, LPN, 8, NT>), dim3(grid), dim3(256), 0, s, a); break;
    case 12: hipLaunchKernelGGL((k_step<T, VEC, LPN, 12, NT>), dim3(grid), dim3(256), 0, s, a); break;
    case 16: hipLaunchKernelGGL((k_step<T, VEC, LPN, 16, NT>), dim3(grid), dim3(256), 0, s, a); break;
    default: hipLaunchKernelGGL((k_step<T, VEC, LPN, 0, NT>), dim3(grid), dim3(256), 0, s, a); break;
    }
}

template <typename T, int VEC, int LPN>
void launch_step_t(const StepArgs<T> &a, int W, bool nt, int pk, int64_t grid, hipStream_t s) {
    MGRT_REQUIRE(a.B == VEC * LPN, MGRT_E_ARG, "row stride must equal the batch width");
    if (nt) launch_step_w<T, VEC, LPN, true>(a, W, pk, grid, s);
    else launch_step_w<T, VEC, LPN, false>(a, W, pk, grid, s);
}

template <typename T, int VEC>
void launch_pml_q_v(int d, const PmlOp &P, int B, int64_t g, const T *p, const T *q, T *qn,
                    hipStream_t s) {
    if (d == 2)
        hipLaunchKernelGGL((k_pml_q<T, VEC, 3>), dim3(g), dim3(256), 0, s, P.ent_rec.as<uint32_t>(),
                           P.n_ent, (int64_t)B, p, q, qn);
    else
        hipLaunchKernelGGL((k_pml_q<T, VEC, 4>), dim3(g), dim3(256), 0, s, P.ent_rec.as<uint32_t>(),
                           P.n_ent, (int64_t)B, p, q, qn);
}

template <typename T>
void launch_pml_q(int d, int vec, const PmlOp &P, int B, int64_t g, const T *p, const T *q, T *qn,
                  hipStream_t s) {
    if (vec == 4) launch_pml_q_v<T, 4>(d, P, B, g, p, q, qn, s);
    else if (vec == 2) launch_pml_q_v<T, 2>(d, P, B, g, p, q, qn, s);
    else launch_pml_q_v<T, 1>(d, P, B, g, p, q, qn, s);
}

template <typename T>
void launch_step(const StepArgs<T> &a, int B, int W, bool nt, int pk, int64_t grid, hipStream_t s);

template <>
void launch_step<float>(const StepArgs<float> &a, int B, int W, bool nt, int pk, int64_t grid,
                        hipStream_t s) {
    switch (B) {
    case 1: launch_step_t<float, 1, 1>(a, W, nt, pk, grid, s); break;
    case 4: launch_step_t<float, 4, 1>(a, W, nt, pk, grid, s); break;
    case 8: launch_step_t<float, 4, 2>(a, W, nt, pk, grid, s); break;
    case 16: launch_step_t<float, 4, 4>(a, W, nt, pk, grid, s); break;
    case 32: launch_step_t<float, 4, 8>(a, W, nt, pk, grid, s); break;
    case 64: launch_step_t<float, 4, 16>(a, W, nt, pk, grid, s); break;
    case 128: launch_step_t<float, 4, 32>(a, W, nt, pk, grid, s); break;
    default: throw Error(MGRT_E_ARG, "unsupported FP32 batch width");
    }
}

template <>
void launch_step<double>(const StepArgs<double> &a, int B, int W, bool nt, int pk, int64_t grid,
                         hipStream_t s) {
    switch (B) {
    case 1: launch_step_t<double, 1, 1>(a, W, nt, pk, grid, s); break;
    case 2: launch_step_t<double, 2, 1>(a, W, nt, pk, grid, s); break;
    case 4: launch_step_t<double, 2, 2>(a, W, nt, pk, grid, s); break;
    case 8: launch_step_t<double, 2, 4>(a, W, nt, pk, grid, s); break;
    case 16: launch_step_t<double, 2, 8>(a, W, nt, pk, grid, s); break;
    case 32: launch_step_t<double, 2, 16>(a, W, nt, pk, grid, s); break;
    case 64: launch_step_t<double, 2, 32>(a, W, nt, pk, grid, s); break;
    case 128: launch_step_t<double, 2, 64>(a, W, nt, pk, grid, s); break;
    default: throw Error(MGRT_E_ARG, "unsupported FP64 batch width");
    }
}

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
    int best = rule;
    double best_est = 0;
    int k = 0;
    for (int b : cands) {
        StepOp &op = get_step_op(c, tile_nodes(prec, b), prec, dt);
        const double us = prec == 32 ? tuned_for<float>(c, op, b).best_us : tuned_for<double>(c, op, b).best_us;
        const double est = (double)((n_cols + b - 1) / b) * us;
        if (k < 6) {
            c.timing.tune_b[k] = b;
            c.timing.tune_b_us[k] = us;
            ++k;
        }
        if (best_est == 0 || est <= best_est) {
            best_est = est;
            best = b;
        }
    }
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
