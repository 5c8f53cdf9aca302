// Internal declarations of libmgrt (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <algorithm>
#include <cstring>
#include <functional>
#include <tuple>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/mgrt.h"

namespace mgrt {

// Error carried through the C++ layer and turned into a return code at the ABI.
struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

#define MGRT_HIP(call)                                                                   \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            throw ::mgrt::Error(MGRT_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define MGRT_REQUIRE(cond, code, msg)                                                    \
    do {                                                                                  \
        if (!(cond)) throw ::mgrt::Error((code), (msg));                                  \
    } while (0)

// Owning device allocation.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    DevBuf() = default;
    explicit DevBuf(size_t b) { alloc(b); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t b) {
        release();
        if (b == 0) return;
        hipError_t e = hipMalloc(&p, b);
        if (e != hipSuccess) {
            p = nullptr;
            throw Error(MGRT_E_OOM_PLAN, "hipMalloc of " + std::to_string(b) + " bytes failed: " +
                                             hipGetErrorString(e));
        }
        bytes = b;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    template <typename T> T *as() const { return static_cast<T *>(p); }
};

// Bump allocation inside caller-provided device memory (the allocation-free entry
// point's scratch): 256-byte aligned pieces, MGRT_E_OOM_PLAN past the end.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    void *take(size_t bytes) {
        const size_t off = (used + 255) & ~(size_t)255;
        if (off + bytes > cap)
            throw Error(MGRT_E_OOM_PLAN, "the call needs more than the " + std::to_string(cap >> 20) +
                                             " MiB of the allocation-free scratch");
        used = off + bytes;
        return base + off;
    }
};

// Copy a host vector into an arena piece (blocking copy, like upload()).
template <typename T>
inline T *put(Arena &ar, const std::vector<T> &v) {
    T *p = static_cast<T *>(ar.take(std::max<size_t>(1, v.size()) * sizeof(T)));
    if (!v.empty()) MGRT_HIP(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
}

template <typename T>
inline DevBuf upload(const std::vector<T> &v, hipStream_t s) {
    // blocking copy: the host vector may be freed as soon as this returns
    (void)s;
    DevBuf b(v.size() * sizeof(T));
    if (!v.empty()) MGRT_HIP(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return b;
}

// P1 point stencil: the d+1 nodes of the containing simplex and the barycentric weights.
struct Stencil {
    int32_t node[4] = {0, 0, 0, 0};
    double w[4] = {0, 0, 0, 0};
};

// Host copy of the mesh and everything derived from it that does not depend on eps.
struct HostMesh {
    int d = 0;
    int64_t n = 0, m = 0, nb = 0, nc = 0;
    std::vector<double> coords;          // n*d
    std::vector<int32_t> elems;          // m*(d+1)
    std::vector<double> vol;             // m
    std::vector<double> grad;            // m*(d+1)*d
    std::vector<int64_t> n2e_ptr;        // node -> incident (element*(d+1)+local)
    std::vector<int64_t> n2e_idx;
    // stiffness K: diagonal + off-diagonal CSR, node-ordered
    std::vector<double> kdiag;           // n
    std::vector<int64_t> krow;           // n+1
    std::vector<int32_t> kcol;
    std::vector<double> kval;
    std::vector<double> rbound;          // n, absorbing-boundary damping
    // stepping order of the nodes: perm[internal] = external id, iperm[external] = internal
    std::vector<int32_t> perm, iperm;
    bool reordered = false;
    // coarse level
    std::vector<int32_t> coarse_of_elem; // m
    std::vector<int32_t> coarse_verts;   // nc*(d+1)
    std::vector<double> cvol;            // nc
    std::vector<int32_t> cnodes;         // unique coarse vertices (fine node ids), sorted
    std::vector<int32_t> cvert_idx;      // nc*(d+1) -> index into cnodes
    std::vector<int64_t> c2f_ptr;        // coarse element -> fine elements
    std::vector<int32_t> c2f_idx;
    // uniform bucket grid of the nodes (about one node per cell) for point location
    double grid_lo[3] = {0, 0, 0}, grid_h = 1.0;
    int64_t grid_dim[3] = {1, 1, 1};
    std::vector<int64_t> grid_ptr;       // cells + 1
    std::vector<int32_t> grid_idx;       // node ids by cell
};

// Device copies of eps-independent mesh data.
struct DevMesh {
    DevBuf krow, kcol, kval, kdiag;   // CSR (FP64) of the off-diagonal stiffness + diagonal
    DevBuf rbound;
    DevBuf elems, vol;                // for element-level restriction of gradients
    DevBuf c2f_ptr, c2f_idx, cvol;
    DevBuf cnodes, cvert_idx;
    DevBuf iperm;                     // external node id -> stepping order
};

// Stepping operator in a working precision for one (slice height, precision, dt).
// Three-level recurrence per node i and column b, as an increment of p (K_ii = -sum_j K_ij):
//   p+ = p + beta_i (p - p-) + sum_{j != i} c_ij (p_j - p_i) + gamma_i g_l(b)
// beta = (M - dt r/2)/D, c_ij = -dt^2 K_ij / D, gamma = dt^2/D, D = M + dt r/2.
// Split-field PML terms of a step operator (App. A, S and T^(k) = zeta^(k) A).  With q
// eliminated where zeta = 0, the three-level recurrence gains the load
//   gamma_i sum_{(T,k): zeta^(k)_T > 0} zeta^(k)_T |T| d_k phi_i|_T q^(k)_{T,l-1/2}
// and only the listed element-directions carry q: q <- (1 - dt zeta) q + dt d_k p|_T.
struct PmlOp {
    int64_t n_ent = 0;         // element-directions with zeta > 0
    int64_t n_rows = 0;        // nodes that receive the load
    int64_t nnz = 0;
    // per entry, 32-bit words: its d+1 nodes (stepping order), dt d_k phi_a|_T for them and
    // 1 - dt zeta (values as 1 (FP32) or 2 (FP64) words)
    DevBuf ent_rec;
    DevBuf row_ptr;            // int32 n_rows+1
    DevBuf row_ent;            // int32 nnz
    DevBuf row_coef;           // T nnz: gamma_i zeta |T| d_k phi_i|_T
    DevBuf node_row;           // int32 n (stepping order): load row or -1
};

struct StepOp {
    int prec = 0;
    int S = 0;                 // nodes per tile (= SELL slice height)
    double dt = 0;
    uint64_t eps_version = 0;
    int64_t n_tiles = 0;
    int wmax = 0;              // widest slice
    double wmean = 0;
    DevBuf slice_ptr;          // int64 n_tiles+1
    DevBuf slice_w;            // int32 n_tiles
    DevBuf cols;               // int32
    DevBuf vals;               // T
    DevBuf beta;               // T, n
    // packed per-node record, stepping order: beta, the node's shared off-diagonal
    // coefficient and W column ids (padded slices as above), values as 1 (FP32) or 2 (FP64)
    // 32-bit words; rows whose coefficients differ flag their first column id and read the
    // slice values
    DevBuf meta;
    int meta_words = 0;
    int64_t uniform_rows = 0;  // nodes whose record carries the shared coefficient
    double oper_bytes = 0;     // operator bytes one step reads (beta, ids, coefficients)
    // dominant neighbour-offset pattern of the records (speculative-gather launches)
    bool spec_ok = false;
    int32_t spec_off[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    std::vector<double> gamma; // host, n (injection weights)
    PmlOp pml;
    // several-steps-per-launch tables for small meshes (multistep.hip), built on first use
    // and dropped whenever the values are refilled
    std::shared_ptr<void> multi;
};

// Launch-variant timing of one stepping configuration (best of two rounds per variant on
// scratch state, microseconds per launch).
struct Tuned {
    int variant = 2;
    double us[16] = {};
    double best_us = 0;
};

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    std::string last_error;
    bool have_mesh = false, have_eps = false;
    HostMesh hm;
    DevMesh dm;
    std::vector<double> Mlump;   // n, lumped eps-mass (host)
    std::vector<double> rdamp;   // n, total damping (host): rsig + rxi
    std::vector<double> rsig;    // n, boundary + conductivity damping
    std::vector<double> rxi;     // n, lumped PML mass S (empty without a PML)
    std::vector<double> pml_zeta;  // m*d, PML zeta^(k)_T (empty without a PML)
    bool have_pml = false;
    DevBuf dM, dR;               // device copies (FP64)
    double gersh = 0;            // max_i sum_j |K_ij| / M_i
    uint64_t eps_version = 0;
    std::map<std::tuple<int, int>, std::unique_ptr<StepOp>> ops;   // key (S, prec)
    std::map<std::tuple<int, int, int, int>, Tuned> tuned;         // (prec, B, S, W) -> variant
    std::map<std::tuple<int, int64_t>, int> batch_tuned;           // (prec, columns) -> B
    std::shared_ptr<void> fft_plans;   // deconv.hip: FFT plans kept per (length, batch, precision)
    mgrt_timing timing{};
};

// mesh_ops.hip
void build_host_mesh(HostMesh &hm, int d, int64_t n, const double *coords, int64_t m,
                     const int32_t *elems, int64_t nb, const int32_t *bfacets,
                     const double *admittance, int64_t nc, const int32_t *coarse_of_elem,
                     const int32_t *coarse_verts);
std::vector<Stencil> locate_points(const HostMesh &hm, int64_t npts, const double *pts);
void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn,
                  int64_t grain = 4096);
void choose_node_order(HostMesh &hm);
void build_node_grid(HostMesh &hm);

// step.hip
StepOp &get_step_op(Ctx &c, int S, int prec, double dt);
int choose_batch(int prec, int64_t n_src, int requested);
int pick_batch(Ctx &c, int prec, int64_t n_cols, int requested, double dt, int flags);
int tile_nodes(int prec, int B);

struct Injection {       // one nodal load entry: p+[node][col] += weight * series[sid][l]
    int64_t node;
    int32_t col;
    int32_t sid;
    double weight;       // includes gamma_i
};
struct Record {          // parts[l][dst] = weight * p+[node][col]
    int64_t node;
    int32_t col;
    int32_t dst;
    double weight;
};

// Batched run of the three-level recurrence on B columns for n_steps steps.
struct BatchRun {
    int prec = 32;
    int B = 64;
    int flags = 0;
    int launch = 0;                    // 0 = tuned launch variant, v + 1 = variant v
    int64_t n_steps = 0;
    int64_t step0 = 0;                 // global index of the first step (series offset)
    std::vector<Injection> inj;
    const double *d_series = nullptr;  // device, [n_series][series_len]
    int64_t series_len = 0;
    std::vector<Record> rec;
    double *d_parts = nullptr;         // device, [n_steps][n_parts]
    int64_t n_parts = 0;
    // coarse-node history: hist[c][col][l] (time contiguous), mode 0 = p+, 1 = -(p+ - p)/dt,
    // 2 = both (p+ to d_hist, -(p+ - p)/dt to d_hist2, same layout)
    bool hist = false;
    int hist_mode = 0;
    void *d_hist = nullptr;
    void *d_hist2 = nullptr;
    int64_t hist_len = 0;              // time extent of each (c, col) series
    int64_t hist_off = 0;              // time offset of step 0 within the series
    bool reverse_hist = false;         // store at hist_len-1-(step) instead
    std::vector<int64_t> hist_nodes;   // fine node ids; index = coarse-node index
    // state buffers (device, n*B each); caller-provided so runs can be resumed
    void *d_p = nullptr, *d_pm = nullptr;
    // adjoint correlation: acc[i] += sum_b p+[i][b] * vel[l][i][b]
    const void *d_vel = nullptr;       // device [n_steps][n][B] in T, indexed by local step
    bool vel_reverse = false;          // local step l reads vel[n_steps-1-l]
    double *d_acc = nullptr;           // device [n] FP64
    void *d_vel_out = nullptr;         // device [n_steps][n][B] in T: -(p+ - p)/dt, all nodes
    // split-field PML state q^(k) of the listed element-directions, [n_ent][B] in T: in/out
    // (resumable runs); null = a zero state local to this call
    void *d_q = nullptr;
    // allocation-free runs: every device buffer of the run comes from this arena, the steps
    // are launched directly (no graph, no tuning, no per-launch events)
    Arena *arena = nullptr;
};
int64_t pml_entries(const Ctx &c);
// multistep.hip: several steps per launch where the run and mesh allow it (false: the
// caller steps one launch per step)
bool run_multistep(Ctx &c, StepOp &op, BatchRun &run);

// deconv.hip: in-place Tikhonov deconvolution of n_series contiguous series of length N
// (FP32 or FP64) by the source function f (N samples), relative regularisation delta,
// scratch memory bounded by scratch_cap bytes
void deconvolve_series(Ctx &c, void *x, int prec, int64_t n_series, int64_t N,
                       const std::vector<double> &f, double delta, size_t scratch_cap);
// deconv.hip: in place, every series x[s] <- the first N samples of x[s] * h (causal
// convolution with one kernel h of N samples), FP64 transforms, scratch bounded likewise
void convolve_series(Ctx &c, void *x, int prec, int64_t n_series, int64_t N,
                     const std::vector<double> &h, size_t scratch_cap);
void run_batch(Ctx &c, StepOp &op, BatchRun &run);
void run_plain(Ctx &c, double dt, int64_t n_steps, const Stencil &src, const double *h_g,
               const std::vector<Record> &rec, double *d_parts, int64_t n_parts, int flags);

// api.hip helpers shared with the Jacobian / gradient / TV code
struct Acquisition {
    int64_t n_src = 0;
    int32_t n_rec = 0;
    std::vector<Stencil> src;   // n_src
    std::vector<Stencil> rec;   // n_src * n_rec
};
Acquisition make_acquisition(Ctx &c, int64_t n_src, const double *src_xyz, int32_t n_rec,
                             const double *rec_xyz);
std::vector<double> load_series(const double *w, int64_t n_steps, double dt);
void check_stability(Ctx &c, double dt, int flags);
int run_precision(const mgrt_run_opts *o);

}  // namespace mgrt

struct mgrt_ctx {
    mgrt::Ctx c;
};

// Run f on the context's device; turn exceptions into MGRT_E_* return codes.
template <typename F>
static inline int mgrt_guarded(mgrt_ctx *ctx, F &&f) {
    if (!ctx) return MGRT_E_ARG;
    try {
        MGRT_HIP(hipSetDevice(ctx->c.device));
        f(ctx->c);
        ctx->c.last_error.clear();
        return MGRT_OK;
    } catch (const mgrt::Error &e) {
        ctx->c.last_error = e.what();
        return e.code;
    } catch (const std::bad_alloc &) {
        ctx->c.last_error = "host allocation failed";
        return MGRT_E_OOM_PLAN;
    } catch (const std::exception &e) {
        ctx->c.last_error = e.what();
        return MGRT_E_ARG;
    }
}
