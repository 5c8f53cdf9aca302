/*
 * mgrt: leap-frog FE wave stepping and its coarse-level linearisation on MI355X.
 *
 * C ABI of libmgrt.so.  Method: Takala, Us, Pursiainen, "Multigrid-based inversion
 * for volumetric radar imaging with asteroid interior reconstruction as a potential
 * application", IEEE TCI 2018 (arXiv 1707.04605).
 *
 * Physics (Sec. II-A, eqs. pde1 / first-order_system / weak_form): the scalar wave
 * equation eps_r u_tt + sigma u_t - Lap u = d/dt f with a point source
 * f = delta_p(x) w(t), discretised with P1 nodal potentials and P0 element gradients
 * (Sec. II-B) and stepped by leap-frog (Appendix A, eqs. leap-frog1/2) with row-sum
 * lumped mass, a first-order absorbing boundary on the listed facets and midpoint
 * damping.  Eliminating the element field gives the equivalent nodal recurrence
 *
 *   (M + dt r/2) p_{l+1} = 2 M p_l - (M - dt r/2) p_{l-1} - dt^2 K p_l
 *                          + dt (f_l - f_{l-1}),          p_0 = p_{-1} = 0,
 *
 * with K = sum_k B^(k)T A^-1 B^(k) (the P1 stiffness matrix), M_i = sum_T eps_T |T|/(d+1),
 * r = lumped conductivity mass + sum over boundary facets of Y_F |F| / d, f_l = w_l phi(x_s)
 * (P1 weights of the source point), and trace[l] = phi(x_r) . p_{l+1}.
 *
 * Conventions for every call:
 *   - Return 0 on success, a negative MGRT_E_* code on failure; mgrt_last_error()
 *     then gives a message.  No C++ exception crosses the ABI.
 *   - Array arguments are host pointers owned by the caller unless the argument
 *     says "device" or opts->flags has MGRT_F_DEVICE_OUT for outputs.  The library
 *     copies what it keeps into device memory it owns and frees in mgrt_destroy().
 *   - Calls are synchronous with respect to the host: on return, outputs are written.
 *   - A context is not thread-safe; separate contexts are independent.
 *   - All floating-point inputs are FP64; "precision" selects the arithmetic of the
 *     wave fields (32 or 64).  Traces, Jacobians and gradients are accumulated and
 *     returned in FP64 unless stated otherwise.
 */
#ifndef MGRT_H
#define MGRT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define MGRT_OK 0
#define MGRT_E_ARG (-1)        /* bad argument (null pointer, size, range)               */
#define MGRT_E_UNSTABLE (-2)   /* dt above the leap-frog stability bound                 */
#define MGRT_E_OOM_PLAN (-3)   /* memory plan does not fit the device (or the budget)    */
#define MGRT_E_HIP (-4)        /* HIP runtime error                                      */
#define MGRT_E_NONFINITE (-5)  /* non-finite value in an input or an output              */
#define MGRT_E_MESH (-6)       /* degenerate, inconsistent or non-nested mesh            */
#define MGRT_E_STATE (-7)      /* call out of order (e.g. no mesh / permittivity yet)    */

/* flags for mgrt_run_opts.flags */
#define MGRT_F_DEVICE_OUT 1    /* output pointers are device pointers                    */
#define MGRT_F_TIMING 2        /* time every stepping launch with HIP events             */
#define MGRT_F_SKIP_STABILITY 8 /* do not reject dt above the Gershgorin bound           */
#define MGRT_F_NO_TUNE 16      /* skip the one-off timing of launch variants            */
#define MGRT_F_JAC_SPLIT 32    /* MG Jacobian: split the wavelet between the source and  */
                               /* receiver runs (default for FP32 fields where the     */
                               /* wavelet's band lies well below the grid scale)        */
#define MGRT_F_JAC_DIRECT 64   /* MG Jacobian: pair the physical source runs with unit   */
                               /* impulses (default for FP64 fields)                     */
#define MGRT_F_NO_GRAPH 128    /* launch every step directly instead of replaying a      */
                               /* captured graph of 64 (or one history chunk of) steps  */
#define MGRT_F_JAC_PAIRED 256  /* MG Jacobian: keep one source run and one receiver run */
                               /* per pair even when every receiver coincides with its  */
                               /* source (default there: one run, see jacobian_coarse)  */
#define MGRT_F_ONE_STEP 512    /* one launch per leap-frog step also where a small mesh  */
                               /* would take several steps per launch (one-column     */
                               /* forward runs on meshes of at most 256 tiles)          */

/* stepping variants */
#define MGRT_STEP_BATCHED 0    /* multi-source node-major ELL launch (default)           */
#define MGRT_STEP_PLAIN 1      /* one source per sweep, FP64 CSR, one launch per step    */

/* Jacobian modes (Sec. II-B) */
#define MGRT_JAC_MG 0          /* eq. approx_2: coarse-node (multigrid) Jacobian J2      */
#define MGRT_JAC_EXACT 1       /* eq. approx_1: exact restricted Jacobian J1 (columns)   */
#define MGRT_JAC_DECONV 2      /* eq. approx_2 by the paper's regularised deconvolution  */

typedef struct mgrt_ctx mgrt_ctx;

typedef struct {
    int precision;             /* 32 or 64 (wave-field arithmetic); 0 = 32              */
    int variant;               /* MGRT_STEP_*                                            */
    int batch;                 /* sources per launch (1..128, power of two), 0 = auto   */
                               /* (timed by the batch tuner on large meshes)           */
    int flags;                 /* MGRT_F_*                                               */
    double mem_budget_gb;      /* device memory the call may plan for; 0 = free memory  */
    double deconv_delta;       /* MGRT_JAC_DECONV: Tikhonov parameter, relative to the   */
                               /* peak power max|F|^2 of the source function (>= 0)      */
    int launch;                /* batched stepping launch variant: 0 = the tuned one    */
                               /* (untuned: packed records, speculative gathers, linear) */
                               /* 1..16 = variant launch-1 (bit 0 non-temporal state,   */
                               /* bit 1 XCD-contiguous tile order, bit 2 packed        */
                               /* per-node records, bit 3 with bit 2 speculative        */
                               /* neighbour gathers); identical results                 */
} mgrt_run_opts;

typedef struct {
    int64_t step_launches;     /* stepping kernel launches in the last call             */
    double step_ms_total;      /* summed event time of those launches (MGRT_F_TIMING)   */
    double call_ms;            /* wall time of the whole call on the device stream      */
    int64_t node_updates;      /* nodes x steps x live sources advanced                  */
    int64_t nodes;             /* mesh nodes                                             */
    int batch;                 /* batch width (columns per launch) used                  */
    int precision;             /* 32 or 64                                               */
    int ell_width;             /* widest off-diagonal row of the stiffness operator     */
    double ell_mean_width;     /* mean off-diagonal row length                          */
    int variant;               /* launch variant of the last stepping run (0..15, as in */
                               /* mgrt_run_opts.launch - 1)                              */
    double step_bytes;         /* algorithmic HBM bytes of those launches: per node and  */
                               /* column 3 state words (+1 velocity out, +1 velocity in */
                               /* in adjoint sweeps); per node beta, the stiffness row's */
                               /* column ids, its coefficients (one where all are equal) */
                               /* and (adjoint) the FP64 accumulator                     */
    double tune_us[16];        /* per-launch microseconds of launch variants 0..15 when */
                               /* this call ran the one-off tuning (best of two rounds */
                               /* on scratch state; 0 for variants not timed), else 0    */
    int jac_split;             /* 1 if the last MG Jacobian split the wavelet            */
    int64_t graph_steps;       /* stepping launches issued by replaying captured graphs */
    int tune_b[6];             /* batch widths timed by the batch tuner in this call     */
                               /* (0 = unused slot; none when the width was requested, */
                               /* the problem was small or the choice was cached)       */
    double tune_b_us[6];       /* their per-launch microseconds (fastest launch variant) */
    int jac_runs;              /* stepping runs per source batch of the last MG Jacobian */
                               /* (1: one run per monostatic pair, 2: source and receiver */
                               /* runs), 0 when the last call formed none               */
    int jac_sets;              /* history sets of the one-run pairing: 2 when a batch    */
                               /* steps while the previous batch is filtered and summed */
                               /* on a second stream, 1 when it waits for them; 0       */
                               /* otherwise                                             */
    int steps_per_launch;      /* leap-frog steps per stepping launch of the last run:  */
                               /* 1, or k when each workgroup advanced its tile and the */
                               /* tile's k-ring k steps in LDS (small one-column runs)  */
} mgrt_timing;

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t to launch
 * on (the caller keeps it alive) or NULL for a stream the context owns. */
int mgrt_create(int device, void *hip_stream, mgrt_ctx **out);
int mgrt_destroy(mgrt_ctx *ctx);
/* Message of the last failing call on ctx (static storage of the context). */
const char *mgrt_last_error(const mgrt_ctx *ctx);

/* Upload the fine simplex mesh T and its nesting into the coarse inversion mesh T'
 * (Sec. II-B; Fig. 2 nesting).
 *   dim          2 or 3
 *   coords       n_nodes x dim, node coordinates
 *   elems        n_elems x (dim+1), node ids of each fine simplex
 *   bfacets      n_bfacets x dim, node ids of absorbing-boundary facets (may be 0 / NULL)
 *   admittance   n_bfacets boundary admittances Y_F (NULL = 1, a vacuum boundary)
 *   coarse_of_elem  n_elems, coarse element containing each fine element (0..n_coarse-1)
 *   coarse_verts n_coarse x (dim+1), fine-node ids of the coarse vertices
 * Builds the stiffness matrix K (eps-independent), the boundary damping and the
 * restriction maps on the device.  Checks positive volumes and that every fine
 * element lies inside its coarse element (MGRT_E_MESH otherwise). */
int mgrt_upload_mesh(mgrt_ctx *ctx, int dim, int64_t n_nodes, const double *coords,
                     int64_t n_elems, const int32_t *elems, int64_t n_bfacets,
                     const int32_t *bfacets, const double *admittance, int64_t n_coarse,
                     const int32_t *coarse_of_elem, const int32_t *coarse_verts);

/* Set eps_r (n_elems, > 0, finite) and sigma (n_elems, >= 0, or NULL = 0) per fine
 * element (Sec. II-A).  Rebuilds only the lumped mass and damping diagonals. */
int mgrt_upload_permittivity(mgrt_ctx *ctx, const double *eps, const double *sigma);

/* Split-field perfectly matched layer (App. A: the xi-weighted mass S in the p-equation
 * and T^(k) = zeta^(k) A in the q-equations of eqs. system1/2, leap-frog1/2).
 *   xi    n_elems, >= 0: S weight per fine element (lumped, taken at the midpoint with
 *         the other damping)
 *   zeta  n_elems x dim, >= 0: zeta^(k) per fine element and direction
 * Both NULL removes the layer.  Only element-directions with zeta > 0 carry the field
 * q^(k) (their load enters the three-level step of every node they touch); elsewhere q is
 * eliminated as without a layer.  Applies to every later forward, Jacobian and gradient
 * run (the gradient checkpoints q with p); the plain reference stepper rejects it
 * (MGRT_E_ARG).  Call after mgrt_upload_mesh, which removes any layer; the order with
 * respect to mgrt_upload_permittivity does not matter. */
int mgrt_upload_pml(mgrt_ctx *ctx, const double *xi, const double *zeta);

/* Largest dt accepted by the stability guard: 2 / sqrt(max_i sum_j |K_ij| / M_i), a
 * Gershgorin bound below the leap-frog limit 2 / sqrt(lambda_max(M^-1 K)). */
int mgrt_stability_bound(mgrt_ctx *ctx, double *dt_max);

/* Forward traces (Sec. II-A point source; App. A leap-frog).  n_src independent runs;
 * run s injects w_l phi(src_s) and records n_rec receivers rec[s][r].
 *   src_xyz   n_src x dim          rec_xyz  n_src x n_rec x dim
 *   wavelet   n_steps, w_l = w(l dt), shared by all sources
 *   traces    out, n_src x n_rec x n_steps (FP64), trace[l] = phi(rec) . p_{l+1}
 * MGRT_E_ARG if n_src, n_rec or n_steps is below 1, a pointer is NULL or a point lies
 * outside the mesh; MGRT_E_UNSTABLE if dt exceeds mgrt_stability_bound (unless
 * MGRT_F_SKIP_STABILITY), MGRT_E_NONFINITE if a coordinate, a wavelet sample or a trace
 * is not finite.  Runs of one source without a PML on meshes of at most 256 tiles
 * (65,536 nodes) whose tiles' k-rings fit in LDS for some k >= 2 advance k steps per
 * launch, each workgroup stepping its tile and the tile's k-ring in the stiffness graph
 * (the same node updates; MGRT_F_ONE_STEP keeps one launch per step;
 * mgrt_timing.steps_per_launch reports which ran). */
int mgrt_forward_traces(mgrt_ctx *ctx, int64_t n_src, const double *src_xyz, int32_t n_rec,
                        const double *rec_xyz, const double *wavelet, double dt,
                        int64_t n_steps, const mgrt_run_opts *opts, double *traces);

/* Forward traces exactly as mgrt_forward_traces (batched stepper only), for callers that
 * cannot allocate device memory (code under stream capture, serving loops, harnesses
 * that forbid hipMalloc): the call allocates no device memory and frees none.  Its device
 * buffers (state, wavelet, tile lists, receiver parts, staging) come from one fixed
 * 64 MiB array per GPU that the library holds until the process ends; MGRT_E_OOM_PLAN
 * when a call needs more (about 2 n B s + 8 n_steps B n_rec (d + 2) bytes, s = 4 or 8).
 * Every call on a GPU shares that array: calls that overlap on one GPU (two threads, two
 * contexts on the same device) race and must be serialised by the caller.  The step
 * operator is not built here: an earlier mgrt_forward_traces on this context with the
 * same precision, batch width (requested, or the one the batch tuner picked for this
 * source count), dt and permittivity must have built it, else MGRT_E_STATE.  Steps are
 * launched directly (no graph replay, no tuning, no per-launch events); the launch variant
 * is the tuned one if this context tuned it, else the default.  Traces are the same values
 * as mgrt_forward_traces' (same kernels, same summation order); MGRT_F_DEVICE_OUT
 * writes them to device memory. */
int mgrt_forward_traces_noalloc(mgrt_ctx *ctx, int64_t n_src, const double *src_xyz,
                                int32_t n_rec, const double *rec_xyz, const double *wavelet,
                                double dt, int64_t n_steps, const mgrt_run_opts *opts,
                                double *traces);

/* Jacobian of sampled traces w.r.t. the coarse permittivity coordinates c_j,
 * eps = eps_0 + sum_j c_j chi'_j (Sec. II-B), at the uploaded eps_0.
 *   sample_steps  n_samples increasing step indices l (rows record trace[l])
 *   mode          MGRT_JAC_MG: eq. approx_2 -- the auxiliary source of App. A-3 with the
 *                 coarse mass derivative lumped to the d+1 coarse vertices, all n_coarse
 *                 columns (cols must be NULL);
 *                 MGRT_JAC_EXACT: eq. approx_1 with the exact auxiliary source, for the
 *                 n_cols columns listed in cols;
 *                 MGRT_JAC_DECONV: eq. approx_2 by the regularised deconvolution of
 *                 App. A-2: the source function is placed at each receiver, the field
 *                 recorded at the coarse nodes is deconvolved by it,
 *                 G = conj(F) P / (|F|^2 + delta max|F|^2) on the window zero-padded to
 *                 a power of two >= 2 n_steps (delta = opts->deconv_delta), and the result
 *                 replaces the exact impulse response in the MG correlation; all
 *                 columns.  Equals MG where delta = 0 and the responses die out inside
 *                 the window; the source spectrum must not vanish when delta = 0.
 *   J             out, FP64, (n_src*n_rec*n_samples) x n_out row-major, row
 *                 (s*n_rec + r)*n_samples + k, n_out = n_coarse (MG, DECONV) or n_cols
 *                 (EXACT).
 * The auxiliary source uses the exact nodal velocity b_l = -(p_{l+1} - p_l)/dt.  MG mode
 * pairs one run per source (b at the coarse nodes) with one impulse run per receiver
 * (discrete reciprocity), the wavelet split exactly between them by default for FP32
 * fields (MGRT_F_JAC_SPLIT / MGRT_F_JAC_DIRECT); with the split, when every source has
 * one receiver at its own point (the same P1 stencil), a single run per source gives both
 * factors (mgrt_timing.jac_runs = 1; MGRT_F_JAC_PAIRED keeps two runs); the filter and
 * the lagged sums of one batch then overlap the run of the next (mgrt_timing.jac_sets). */
int mgrt_jacobian_coarse(mgrt_ctx *ctx, int64_t n_src, const double *src_xyz, int32_t n_rec,
                         const double *rec_xyz, const double *wavelet, double dt,
                         int64_t n_steps, int32_t n_samples, const int64_t *sample_steps,
                         int mode, int64_t n_cols, const int64_t *cols,
                         const mgrt_run_opts *opts, double *J);

/* Misfit gradient g = J1^T rho: the exact derivative of sum_{s,r,l} rho[s][r][l] *
 * trace[s][r][l] w.r.t. eps, by a reverse-time adjoint run with checkpointed forward
 * recomputation.  residual: n_src x n_rec x n_steps.  level 0: grad has n_coarse
 * entries (d/dc_j); level 1: grad has n_elems entries (d/d eps_T of each fine element).
 * MGRT_E_OOM_PLAN if even one source does not fit the memory budget. */
int mgrt_misfit_gradient(mgrt_ctx *ctx, int64_t n_src, const double *src_xyz, int32_t n_rec,
                         const double *rec_xyz, const double *wavelet, double dt,
                         int64_t n_steps, const double *residual, int level,
                         const mgrt_run_opts *opts, double *grad);

/* TV-regularised linearised inversion on one level (Sec. II-C, eq. tv_iteration):
 *   z_{l+1} = (L^T L + alpha D^T Gamma_l D)^{-1} L^T r,  z = x - x0,  r = y - y0,
 *   Gamma_0 = I,  Gamma_l = diag(1 / max(|D z_l|, tau)),  tau = 1e-8 max |D z_l|
 *   (Gamma_l = I when D z_l vanishes),
 * each system A z = L^T r solved in FP64, by solver:
 *   MGRT_TV_AUTO  where the library forms the normal matrix G = L^T L (when it is smaller
 *                 than two passes over L and fits the free memory), directly: dense
 *                 Cholesky A = U^T U and two triangular solves (the step reports 0
 *                 iterations); otherwise, or if A is not numerically positive definite
 *                 or its factor does not fit the free device memory, as MGRT_TV_CG
 *   MGRT_TV_CG    preconditioned conjugate gradients (Jacobi, or for rows <= 512 < M the
 *                 exact inverse of alpha diag(D^T Gamma D) + L^T L by the Woodbury
 *                 identity; warm start from the previous iterate) to relative residual
 *                 ||L^T r - A z|| <= cg_rtol ||L^T r||, at most cg_maxit iterations per
 *                 outer step (the residual is checked every 8 iterations)
 *   L          rows x M row-major, FP32 (L_precision 32) or FP64 (64); host pointer, or
 *              a device pointer when L_on_device != 0
 *   r          rows (FP64)
 *   D          CSR with M rows: D_rowptr (M+1), D_col (nnz), D_val (nnz)
 *   solver     MGRT_TV_AUTO or MGRT_TV_CG (else MGRT_E_ARG)
 *   z_out      iters x M (FP64): every iterate z_1 .. z_iters
 *   cg_iters   optional out (iters): CG iterations used per outer step (0: direct) */
#define MGRT_TV_AUTO 0
#define MGRT_TV_CG 1
int mgrt_tv_invert_level(mgrt_ctx *ctx, int64_t rows, int64_t M, const void *L,
                         int L_precision, int L_on_device, const double *r,
                         const int64_t *D_rowptr, const int32_t *D_col, const double *D_val,
                         double alpha, int iters, double cg_rtol, int cg_maxit, int solver,
                         double *z_out, int32_t *cg_iters);

/* Coarse-to-fine TV inversion over two nested levels T' (M elements, the columns of L)
 * and T'' (M2 elements) (Sec. II-D, eqs. decomposition, tv_iteration_0, tv_iteration_2;
 * Sec. II-E, compression).  With z = x - x0 = 0 initially and r = y - y0, each of the
 * iters steps does
 *   (2) z_c = (L_c^T L_c + alpha D_c^T Gamma_c D_c)^{-1} L_c^T r,  L_c = L R_c;
 *   compression: keep the fine basis of the n_keep parents with the largest |z_c|
 *       (ties to the lower id; n_keep >= M2 keeps all, 0 none);
 *   (3) z_f = (L_f^T L_f + alpha (D_f R_f)^T Gamma_f (D_f R_f))^{-1} L_f^T (r - L_c z_c),
 *       L_f = L R_f;
 *   (4) x - x0 = R_c z_c + R_f z_f.
 * R_c: each T' element takes its parent's value.  R_f: per parent, +1/-1 on pairs of
 * children sharing a facet (the edges of a spanning tree of the children's facet
 * adjacency; in 2D the three corner/middle pairs).  Gamma of each level is built as in
 * mgrt_tv_invert_level from that level's previous iterate (Gamma_f from D_f applied to
 * the previous fine field on T'); Gamma = I on the first step.  The results (x, z_c) do
 * not depend on which spanning tree is used.  Each system is solved as in
 * mgrt_tv_invert_level by solver (CG: coarse warm-started, fine from zero).
 *   L, L_precision, L_on_device, r   as for mgrt_tv_invert_level
 *   dim         2 or 3
 *   elem_verts  M x (dim+1) vertex ids of the T' elements (any numbering; two elements
 *               are adjacent when they share dim ids)
 *   parent      M, the T'' element containing each T' element (every T'' element needs
 *               at least one child; children of one parent must be facet-connected, else
 *               MGRT_E_MESH)
 *   D_c         CSR, M2 x M2 (eq. d_mat on T'');  D_f  CSR, M x M (eq. d_mat on T')
 *   x_out       iters x M: x_l - x0 on T'
 *   zc_out      optional, iters x M2: z_c per step
 *   kept_out    optional, iters x min(n_keep, M2): kept parents, ascending
 *   cg_iters    optional, iters x 2: CG iterations of the coarse and the fine solve
 *               (0: direct) */
int mgrt_tv_invert_two_level(mgrt_ctx *ctx, int64_t rows, int64_t M, const void *L,
                             int L_precision, int L_on_device, const double *r, int dim,
                             const int32_t *elem_verts, int64_t M2, const int32_t *parent,
                             const int64_t *Dc_rowptr, const int32_t *Dc_col,
                             const double *Dc_val, const int64_t *Df_rowptr,
                             const int32_t *Df_col, const double *Df_val, double alpha,
                             int iters, int64_t n_keep, double cg_rtol, int cg_maxit,
                             int solver, double *x_out, double *zc_out, int32_t *kept_out,
                             int32_t *cg_iters);

/* Quadrature weights of the time-weighted inner products of Sec. II-F on a sample grid,
 *   <a, b>_1 = int_0^T a b dt,   <a, b>_2 = (1/T) int_0^T t a b dt,   T = n_steps dt,
 * for mgrt_project_rows: sample k holds the field at t_k = (sample_steps[k] + 1) dt (the
 * trace after step sample_steps[k]), integrated by the rectangle rule with widths
 * w_k = t_k - t_{k-1}, t_{-1} = 0:
 *   q[0][k] = w_k,   q[1][k] = (t_k / T) w_k          (q: 2 x n_samples, caller-owned)
 * so that <a, b>_j = sum_k q[j][k] a_k b_k.  Host arithmetic only; needs no context.
 * MGRT_E_ARG for null pointers, n_samples < 1, n_steps < 1, dt not positive and finite,
 * or sample steps outside 0..n_steps-1 or not increasing. */
int mgrt_projection_weights(const int64_t *sample_steps, int32_t n_samples, double dt,
                            int64_t n_steps, double *q);

/* Projection of sampled rows onto time-weighted inner products (Sec. II-F):
 *   P[i][j][c] = sum_k q[j][k] u[i][k] J[i*n_samples + k][c],
 * i.e. <u_i, J_i[:, c]>_j with <a, b>_j = sum_k q[j][k] a_k b_k.  With J the Jacobian
 * (rows (trace, sample), as written by mgrt_jacobian_coarse) and u the measured traces
 * this gives the projected Jacobian rows d<u, u0>_j/dc; with J a trace array (M = 1) it
 * gives the projected data <u, u0>_j or <u, u>_j.  The quadrature q is an input: the
 * paper's <a, b>_1 and <a, b>_2 come from mgrt_projection_weights.  Sums in FP64, in
 * sample order.
 *   J        n_traces*n_samples x M row-major, FP32 (J_precision 32) or FP64 (64); host
 *            pointer, or device pointer when J_on_device != 0
 *   u        n_traces x n_samples (FP64, host);  q  n_proj x n_samples (FP64, host)
 *   n_proj   1..8;  n_traces <= 65535
 *   P        out, n_traces x n_proj x M (FP64, host, caller-owned)
 * mgrt_last_timing reports the device time of the reduction in call_ms. */
int mgrt_project_rows(mgrt_ctx *ctx, int64_t n_traces, int32_t n_samples, int64_t M,
                      const void *J, int J_precision, int J_on_device, const double *u,
                      int32_t n_proj, const double *q, double *P);

/* Counters and event timings of the last stepping call on ctx.  Launch variants of the
 * stepping kernel (bit 0: non-temporal p_{l-1}/p_{l+1} accesses, bit 1: XCD-contiguous
 * tile order, bit 2: packed per-node records, bit 3: speculative neighbour gathers at the
 * operator's most common offsets) all compute identical results; the fastest is picked by
 * timing a few steps the first time a configuration runs on a context. */
int mgrt_last_timing(const mgrt_ctx *ctx, mgrt_timing *out);

/* sizeof(mgrt_run_opts) and sizeof(mgrt_timing) as this library was built, for bindings
 * that mirror the two structs (needs no device).  Either pointer may be NULL.  Returns
 * MGRT_OK. */
int mgrt_struct_sizes(size_t *run_opts_bytes, size_t *timing_bytes);

#ifdef __cplusplus
}
#endif

#endif /* MGRT_H */
