// Device side of the leap-frog stepper: the kernels (the batched three-level step with
// its fused tail, the history flush, the PML update of the split-field layer, the plain
// per-source CSR step) and the mapping from batch width, slice width and record mode to
// their template instantiations.  Included by step.hip only, which holds the host side
// (operator build, tile lists, launch variants, tuning, graph replay).
#pragma once

#include <cstdint>
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

namespace {

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

}  // namespace

}  // namespace mgrt
