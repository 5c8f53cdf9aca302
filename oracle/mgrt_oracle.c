/*
 * FP64 CPU oracle for the leap-frog FE wave solver and its linearisation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code with the GPU library.
 *
 * It steps the paper's mixed form (Appendix A, eqs. system1/system2 and leap-frog1/2)
 * literally: a nodal P1 potential p and an elementwise P0 gradient field q^(k),
 *
 *   q_{l+1/2}|_T = q_{l-1/2}|_T + dt * grad(p_l)|_T                     (A^-1 B^(k) p)
 *   (M + dt r/2) p_{l+1} = (M - dt r/2) p_l + dt (f_l - sum_k B^(k)T q^(k)_{l+1/2})
 *
 * with A_TT = |T|, B^(k)_{T,j} = |T| d_k phi_j|_T, M the row-sum lumped eps-weighted mass
 * matrix C, and r the lumped damping (conductivity mass R plus a first-order absorbing
 * boundary term); the damping is taken at the midpoint (p_{l+1} + p_l)/2.  The
 * stiffness matrix is never assembled.
 *
 * Linearisation (Sec. II-B eqs. approx_1 / approx_2, Appendix A-1 and A-3):
 *   - tangent-linear recurrence in (dp, dq) with source h_l = -dM (p_{l+1} - p_l)/dt;
 *   - complex-step forward (eps + i delta dEps) as an independent derivative;
 *   - per-node response runs used to build the multigrid Jacobian.
 *
 * Conventions: zero initial state unless given; source f_l = w_l * phi(x_s) at
 * t_l = l dt, l = 0..N-1; trace[l] = phi(x_r) . p_{l+1}.
 *
 * Error behaviour: functions return 0 on success and a negative code on bad input
 * (-1 argument, -2 point outside the mesh, -3 out of memory).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef int64_t i64;
typedef int32_t i32;

/* ---------------------------------------------------------------------------------
 * Geometry (Sec. II-B): simplex volume |T| and gradients of the P1 basis on T.
 * grad layout: (m, d+1, d).
 * ------------------------------------------------------------------------------- */
static double simplex_geometry(int d, const double *x[4], double g[4][3])
{
    double E[3][3] = {{0}};
    for (int k = 0; k < d; ++k)
        for (int a = 0; a < d; ++a)
            E[a][k] = x[k + 1][a] - x[0][a];          /* column k = x_{k+1} - x_0 */
    double det, inv[3][3];
    if (d == 2) {
        det = E[0][0] * E[1][1] - E[0][1] * E[1][0];
        inv[0][0] = E[1][1] / det;  inv[0][1] = -E[0][1] / det;
        inv[1][0] = -E[1][0] / det; inv[1][1] = E[0][0] / det;
    } else {
        double c00 = E[1][1] * E[2][2] - E[1][2] * E[2][1];
        double c01 = E[1][2] * E[2][0] - E[1][0] * E[2][2];
        double c02 = E[1][0] * E[2][1] - E[1][1] * E[2][0];
        det = E[0][0] * c00 + E[0][1] * c01 + E[0][2] * c02;
        inv[0][0] = c00 / det;
        inv[1][0] = c01 / det;
        inv[2][0] = c02 / det;
        inv[0][1] = (E[0][2] * E[2][1] - E[0][1] * E[2][2]) / det;
        inv[1][1] = (E[0][0] * E[2][2] - E[0][2] * E[2][0]) / det;
        inv[2][1] = (E[0][1] * E[2][0] - E[0][0] * E[2][1]) / det;
        inv[0][2] = (E[0][1] * E[1][2] - E[0][2] * E[1][1]) / det;
        inv[1][2] = (E[0][2] * E[1][0] - E[0][0] * E[1][2]) / det;
        inv[2][2] = (E[0][0] * E[1][1] - E[0][1] * E[1][0]) / det;
    }
    /* barycentric lambda_k (k>=1) = row k-1 of E^-1 applied to (x - x0) */
    for (int a = 0; a < d; ++a) g[0][a] = 0.0;
    for (int k = 1; k <= d; ++k)
        for (int a = 0; a < d; ++a) {
            g[k][a] = inv[k - 1][a];
            g[0][a] -= inv[k - 1][a];
        }
    double fact = (d == 2) ? 2.0 : 6.0;
    return fabs(det) / fact;
}

int orc_geometry(int d, i64 m, const double *coords, const i32 *elems, double *vol, double *grad)
{
    if (d != 2 && d != 3) return -1;
#pragma omp parallel for schedule(static)
    for (i64 t = 0; t < m; ++t) {
        const double *x[4];
        double g[4][3];
        for (int a = 0; a <= d; ++a) x[a] = coords + (i64)elems[t * (d + 1) + a] * d;
        vol[t] = simplex_geometry(d, x, g);
        for (int a = 0; a <= d; ++a)
            for (int k = 0; k < d; ++k) grad[(t * (d + 1) + a) * d + k] = g[a][k];
    }
    return 0;
}

/* Row-sum lumped weighted mass: out_i = sum_{T containing i} w_T |T| / (d+1). */
int orc_lumped_mass(int d, i64 n, i64 m, const i32 *elems, const double *vol, const double *w,
                    double *out)
{
    memset(out, 0, sizeof(double) * n);
    for (i64 t = 0; t < m; ++t) {
        double c = (w ? w[t] : 1.0) * vol[t] / (d + 1);
        for (int a = 0; a <= d; ++a) out[elems[t * (d + 1) + a]] += c;
    }
    return 0;
}

/* First-order absorbing boundary du/dn = -Y du/dt on facets F: the boundary integral
 * of Y u_t v over F, row-sum lumped: adds Y_F |F| / d to each facet node. */
int orc_boundary_damping(int d, i64 n, const double *coords, i64 nb, const i32 *bfacets,
                         const double *adm, double *r)
{
    for (i64 f = 0; f < nb; ++f) {
        const i32 *v = bfacets + f * d;
        double meas;
        if (d == 2) {
            double dx = coords[v[1] * 2] - coords[v[0] * 2];
            double dy = coords[v[1] * 2 + 1] - coords[v[0] * 2 + 1];
            meas = sqrt(dx * dx + dy * dy);
        } else {
            double a[3], b[3];
            for (int k = 0; k < 3; ++k) {
                a[k] = coords[(i64)v[1] * 3 + k] - coords[(i64)v[0] * 3 + k];
                b[k] = coords[(i64)v[2] * 3 + k] - coords[(i64)v[0] * 3 + k];
            }
            double cx = a[1] * b[2] - a[2] * b[1];
            double cy = a[2] * b[0] - a[0] * b[2];
            double cz = a[0] * b[1] - a[1] * b[0];
            meas = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
        }
        double c = (adm ? adm[f] : 1.0) * meas / d;
        for (int a = 0; a < d; ++a) r[v[a]] += c;
    }
    (void)n;
    return 0;
}

/* Point location (Sec. II-A point source; P1 weights phi_i(x)): the lowest-numbered
 * element whose barycentric coordinates are all >= -1e-12; nodes and weights out. */
int orc_locate(int d, const double *coords, i64 m, const i32 *elems, i64 npts, const double *pts,
               i32 *out_nodes, double *out_w)
{
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (i64 p = 0; p < npts; ++p) {
        const double *y = pts + p * d;
        int found = 0;
        for (i64 t = 0; t < m && !found; ++t) {
            const double *x[4];
            double g[4][3];
            for (int a = 0; a <= d; ++a) x[a] = coords + (i64)elems[t * (d + 1) + a] * d;
            simplex_geometry(d, x, g);
            double lam[4], mn = 1e300;
            for (int a = 0; a <= d; ++a) {
                /* lambda_a(y) = 1[a==0] + grad_a . (y - x0) */
                double s = (a == 0) ? 1.0 : 0.0;
                for (int k = 0; k < d; ++k) s += g[a][k] * (y[k] - x[0][k]);
                lam[a] = s;
                if (s < mn) mn = s;
            }
            if (mn >= -1e-12) {
                for (int a = 0; a <= d; ++a) {
                    out_nodes[p * (d + 1) + a] = elems[t * (d + 1) + a];
                    out_w[p * (d + 1) + a] = lam[a];
                }
                found = 1;
            }
        }
        if (!found) {
#pragma omp atomic write
            bad = 1;
        }
    }
    return bad ? -2 : 0;
}

/* ---------------------------------------------------------------------------------
 * The mixed-form operator pieces.
 * ------------------------------------------------------------------------------- */
typedef struct {
    int d;
    i64 n, m;
    const i32 *elems;
    const double *vol;
    const double *grad;
    const double *zeta;   /* m x d split-field PML coefficients zeta^(k)_T, or NULL */
    i64 *adj_ptr;   /* node -> incident (element, local vertex) */
    i64 *adj_idx;   /* value = t*(d+1) + a */
} mesh_t;

static int mesh_init(mesh_t *ms, int d, i64 n, i64 m, const i32 *elems, const double *vol,
                     const double *grad, const double *zeta)
{
    ms->d = d; ms->n = n; ms->m = m; ms->elems = elems; ms->vol = vol; ms->grad = grad;
    ms->zeta = zeta;
    ms->adj_ptr = calloc(n + 1, sizeof(i64));
    ms->adj_idx = malloc(sizeof(i64) * m * (d + 1));
    if (!ms->adj_ptr || !ms->adj_idx) return -3;
    for (i64 k = 0; k < m * (d + 1); ++k) ms->adj_ptr[elems[k] + 1]++;
    for (i64 i = 0; i < n; ++i) ms->adj_ptr[i + 1] += ms->adj_ptr[i];
    i64 *fill = malloc(sizeof(i64) * n);
    if (!fill) return -3;
    memcpy(fill, ms->adj_ptr, sizeof(i64) * n);
    for (i64 k = 0; k < m * (d + 1); ++k) ms->adj_idx[fill[elems[k]]++] = k;
    free(fill);
    return 0;
}

static void mesh_free(mesh_t *ms)
{
    free(ms->adj_ptr);
    free(ms->adj_idx);
}

/* leap-frog1: q^(k)_{l+1/2} = q^(k)_{l-1/2} + dt A^-1 (B^(k) p_l - T^(k) q^(k)_{l-1/2}),
 * with A^-1 B^(k) p = d_k p|_T and A^-1 T^(k) = zeta^(k)_T (the split-field PML; zero
 * outside the layer, or everywhere when no PML is given) */
static void update_q(const mesh_t *ms, double dt, const double *p, double *q, int par)
{
    const int d = ms->d;
    const double *zeta = ms->zeta;
#pragma omp parallel for schedule(static) if (par && ms->m > 50000)
    for (i64 t = 0; t < ms->m; ++t) {
        const i32 *e = ms->elems + t * (d + 1);
        const double *g = ms->grad + t * (d + 1) * d;
        for (int k = 0; k < d; ++k) {
            double s = 0.0;
            for (int a = 0; a <= d; ++a) s += p[e[a]] * g[a * d + k];
            if (zeta) s -= zeta[t * d + k] * q[t * d + k];
            q[t * d + k] += dt * s;
        }
    }
}

/* s_i = sum_k (B^(k)T q^(k))_i = sum_{T containing i} |T| grad(phi_i)|_T . q_T */
static double btq_node(const mesh_t *ms, const double *q, i64 i)
{
    const int d = ms->d;
    double s = 0.0;
    for (i64 k = ms->adj_ptr[i]; k < ms->adj_ptr[i + 1]; ++k) {
        i64 v = ms->adj_idx[k];
        i64 t = v / (d + 1);
        int a = (int)(v % (d + 1));
        const double *g = ms->grad + (t * (d + 1) + a) * d;
        double dot = 0.0;
        for (int c = 0; c < d; ++c) dot += g[c] * q[t * d + c];
        s += ms->vol[t] * dot;
    }
    return s;
}

/* p_{l+1} from p_l, q_{l+1/2} and the nodal load f (dense) */
static void update_p(const mesh_t *ms, double dt, const double *M, const double *r,
                     const double *q, const double *f, double *p, int par)
{
#pragma omp parallel for schedule(static) if (par && ms->m > 50000)
    for (i64 i = 0; i < ms->n; ++i) {
        double s = btq_node(ms, q, i);
        double load = f ? f[i] : 0.0;
        double lo = M[i] - 0.5 * dt * r[i];
        double hi = M[i] + 0.5 * dt * r[i];
        p[i] = (lo * p[i] + dt * (load - s)) / hi;
    }
}

/* K p computed through the mixed form: B^T A^-1 B p (used by the tests and the CFL
 * power iteration). */
int orc_apply_stiffness(int d, i64 n, i64 m, const i32 *elems, const double *vol,
                        const double *grad, const double *p, double *out)
{
    mesh_t ms;
    if (mesh_init(&ms, d, n, m, elems, vol, grad, NULL)) return -3;
    double *q = calloc((size_t)m * d, sizeof(double));
    if (!q) return -3;
    update_q(&ms, 1.0, p, q, 1);
#pragma omp parallel for schedule(static)
    for (i64 i = 0; i < n; ++i) out[i] = btq_node(&ms, q, i);
    free(q);
    mesh_free(&ms);
    return 0;
}

/* lambda_max(M^-1 K) by power iteration from a seeded start (xorshift). */
int orc_lambda_max(int d, i64 n, i64 m, const i32 *elems, const double *vol, const double *grad,
                   const double *M, int iters, double *out)
{
    mesh_t ms;
    if (mesh_init(&ms, d, n, m, elems, vol, grad, NULL)) return -3;
    double *v = malloc(sizeof(double) * n), *w = malloc(sizeof(double) * n);
    double *q = malloc(sizeof(double) * m * d);
    uint64_t s = 0x9E3779B97F4A7C15ull;
    for (i64 i = 0; i < n; ++i) {
        s ^= s << 13; s ^= s >> 7; s ^= s << 17;
        v[i] = (double)(s >> 11) / 9007199254740992.0 - 0.5;
    }
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        /* w = M^-1 K v; Rayleigh quotient in the M inner product */
        memset(q, 0, sizeof(double) * m * d);
        update_q(&ms, 1.0, v, q, 1);
        double num = 0.0, den = 0.0;
        for (i64 i = 0; i < n; ++i) {
            double kv = btq_node(&ms, q, i);
            num += v[i] * kv;
            den += v[i] * M[i] * v[i];
            w[i] = kv / M[i];
        }
        lam = num / den;
        double nrm = 0.0;
        for (i64 i = 0; i < n; ++i) nrm += w[i] * M[i] * w[i];
        nrm = sqrt(nrm);
        for (i64 i = 0; i < n; ++i) v[i] = w[i] / nrm;
    }
    *out = lam;
    free(v); free(w); free(q);
    mesh_free(&ms);
    return 0;
}

/* ---------------------------------------------------------------------------------
 * Forward runs.
 *
 * One "simulation" = one source stencil (d+1 nodes, weights) driven by a wavelet,
 * observed by n_rec receiver stencils.  Simulations are independent and run in
 * parallel.  Optional initial state (p0, q0) and final state (p_N, p_{N-1}, q_{N-1/2})
 * are supported for a single simulation.
 * ------------------------------------------------------------------------------- */
static double stencil_dot(int d, const i32 *nodes, const double *w, const double *p)
{
    double s = 0.0;
    for (int a = 0; a <= d; ++a) s += w[a] * p[nodes[a]];
    return s;
}

int orc_forward(int d, i64 n, i64 m, const i32 *elems, const double *vol, const double *grad,
                const double *zeta,
                const double *M, const double *r, double dt, i64 nsteps,
                i64 nsim, const i32 *src_nodes, const double *src_w,
                const double *wavelet, i64 wav_stride,
                i64 nrec, const i32 *rec_nodes, const double *rec_w,
                double *traces,
                const double *p0, const double *q0,
                double *p_last, double *p_prev, double *q_last)
{
    mesh_t ms;
    if (mesh_init(&ms, d, n, m, elems, vol, grad, zeta)) return -3;
    int inner = nsim == 1;
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) if (!inner)
    for (i64 s = 0; s < nsim; ++s) {
        double *p = calloc(n, sizeof(double));
        double *pold = calloc(n, sizeof(double));
        double *q = calloc((size_t)m * d, sizeof(double));
        double *f = calloc(n, sizeof(double));
        if (!p || !q || !f || !pold) { err = -3; continue; }
        if (p0) memcpy(p, p0, sizeof(double) * n);
        if (q0) memcpy(q, q0, sizeof(double) * m * d);
        const i32 *sn = src_nodes ? src_nodes + s * (d + 1) : NULL;
        const double *sw = src_w ? src_w + s * (d + 1) : NULL;
        const double *wav = wavelet ? wavelet + s * wav_stride : NULL;
        for (i64 l = 0; l < nsteps; ++l) {
            if (sn && wav)
                for (int a = 0; a <= d; ++a) f[sn[a]] = 0.0;
            if (sn && wav)
                for (int a = 0; a <= d; ++a) f[sn[a]] += wav[l] * sw[a];
            memcpy(pold, p, sizeof(double) * n);
            update_q(&ms, dt, p, q, inner);
            update_p(&ms, dt, M, r, q, (sn && wav) ? f : NULL, p, inner);
            for (i64 k = 0; k < nrec; ++k) {
                const i32 *rn = rec_nodes + (s * nrec + k) * (d + 1);
                const double *rw = rec_w + (s * nrec + k) * (d + 1);
                traces[(s * nrec + k) * nsteps + l] = stencil_dot(d, rn, rw, p);
            }
        }
        if (nsim == 1) {
            if (p_last) memcpy(p_last, p, sizeof(double) * n);
            if (p_prev) memcpy(p_prev, pold, sizeof(double) * n);
            if (q_last) memcpy(q_last, q, sizeof(double) * m * d);
        }
        free(p); free(pold); free(q); free(f);
    }
    mesh_free(&ms);
    return err;
}

/* Tangent-linear (exact restricted Jacobian, eq. approx_1 with the exact source).
 * For each (simulation s, direction c): the forward run together with
 *   (M + dt r/2) dp_{l+1} = (M - dt r/2) dp_l + dt (h_l - B^T dq_{l+1/2}),
 *   dq_{l+1/2} = dq_{l-1/2} + dt grad(dp_l),   h_l = -dM_c (p_{l+1} - p_l) / dt,
 * where dM_c is the derivative of the lumped mass along the direction c.
 * Output dtraces (nsim, ndir, nrec, nsteps). */
int orc_tangent(int d, i64 n, i64 m, const i32 *elems, const double *vol, const double *grad,
                const double *zeta,
                const double *M, const double *r, double dt, i64 nsteps,
                i64 nsim, const i32 *src_nodes, const double *src_w,
                const double *wavelet, i64 wav_stride,
                i64 nrec, const i32 *rec_nodes, const double *rec_w,
                i64 ndir, const double *dM, double *dtraces)
{
    mesh_t ms;
    if (mesh_init(&ms, d, n, m, elems, vol, grad, zeta)) return -3;
    int err = 0;
    i64 njobs = nsim * ndir;
    int inner = njobs == 1;
#pragma omp parallel for schedule(dynamic, 1) if (!inner)
    for (i64 job = 0; job < njobs; ++job) {
        i64 s = job / ndir, c = job % ndir;
        double *p = calloc(n, sizeof(double)), *pold = calloc(n, sizeof(double));
        double *q = calloc((size_t)m * d, sizeof(double));
        double *dp = calloc(n, sizeof(double)), *dq = calloc((size_t)m * d, sizeof(double));
        double *f = calloc(n, sizeof(double)), *hh = calloc(n, sizeof(double));
        if (!p || !pold || !q || !dp || !dq || !f || !hh) { err = -3; continue; }
        const i32 *sn = src_nodes + s * (d + 1);
        const double *sw = src_w + s * (d + 1);
        const double *wav = wavelet + s * wav_stride;
        const double *dm = dM + c * n;
        for (i64 l = 0; l < nsteps; ++l) {
            for (int a = 0; a <= d; ++a) f[sn[a]] = 0.0;
            for (int a = 0; a <= d; ++a) f[sn[a]] += wav[l] * sw[a];
            memcpy(pold, p, sizeof(double) * n);
            update_q(&ms, dt, p, q, inner);
            update_p(&ms, dt, M, r, q, f, p, inner);
            for (i64 i = 0; i < n; ++i) hh[i] = -dm[i] * (p[i] - pold[i]) / dt;
            update_q(&ms, dt, dp, dq, inner);
            update_p(&ms, dt, M, r, dq, hh, dp, inner);
            for (i64 k = 0; k < nrec; ++k) {
                const i32 *rn = rec_nodes + (s * nrec + k) * (d + 1);
                const double *rw = rec_w + (s * nrec + k) * (d + 1);
                dtraces[((s * ndir + c) * nrec + k) * nsteps + l] = stencil_dot(d, rn, rw, dp);
            }
        }
        free(p); free(pold); free(q); free(dp); free(dq); free(f); free(hh);
    }
    mesh_free(&ms);
    return err;
}

/* Complex-step forward: the same recurrence in complex arithmetic with
 * M = M_re + i * delta * dM (the lumped mass of eps + i delta dEps).  Returns
 * Im(trace) / delta, an independent route to the tangent-linear traces. */
int orc_complex_step(int d, i64 n, i64 m, const i32 *elems, const double *vol, const double *grad,
                const double *zeta,
                     const double *M, const double *r, double dt, i64 nsteps,
                     const i32 *src_nodes, const double *src_w, const double *wavelet,
                     i64 nrec, const i32 *rec_nodes, const double *rec_w,
                     const double *dM, double delta, double *out)
{
    mesh_t ms;
    if (mesh_init(&ms, d, n, m, elems, vol, grad, zeta)) return -3;
    double complex *p = calloc(n, sizeof(double complex));
    double complex *q = calloc((size_t)m * d, sizeof(double complex));
    double *f = calloc(n, sizeof(double));
    if (!p || !q || !f) return -3;
    for (i64 l = 0; l < nsteps; ++l) {
        for (int a = 0; a <= d; ++a) f[src_nodes[a]] = 0.0;
        for (int a = 0; a <= d; ++a) f[src_nodes[a]] += wavelet[l] * src_w[a];
#pragma omp parallel for schedule(static)
        for (i64 t = 0; t < m; ++t) {
            const i32 *e = elems + t * (d + 1);
            const double *g = grad + t * (d + 1) * d;
            for (int k = 0; k < d; ++k) {
                double complex s = 0.0;
                for (int a = 0; a <= d; ++a) s += p[e[a]] * g[a * d + k];
                if (zeta) s -= zeta[t * d + k] * q[t * d + k];
                q[t * d + k] += dt * s;
            }
        }
#pragma omp parallel for schedule(static)
        for (i64 i = 0; i < n; ++i) {
            double complex s = 0.0;
            for (i64 k = ms.adj_ptr[i]; k < ms.adj_ptr[i + 1]; ++k) {
                i64 v = ms.adj_idx[k];
                i64 t = v / (d + 1);
                int a = (int)(v % (d + 1));
                const double *g = grad + (t * (d + 1) + a) * d;
                double complex dot = 0.0;
                for (int c = 0; c < d; ++c) dot += g[c] * q[t * d + c];
                s += vol[t] * dot;
            }
            double complex Mi = M[i] + I * delta * dM[i];
            double complex lo = Mi - 0.5 * dt * r[i];
            double complex hi = Mi + 0.5 * dt * r[i];
            p[i] = (lo * p[i] + dt * (f[i] - s)) / hi;
        }
        for (i64 k = 0; k < nrec; ++k) {
            double complex s = 0.0;
            for (int a = 0; a <= d; ++a) s += rec_w[k * (d + 1) + a] * p[rec_nodes[k * (d + 1) + a]];
            out[k * nsteps + l] = cimag(s) / delta;
        }
    }
    free(p); free(q); free(f);
    mesh_free(&ms);
    return 0;
}

/* Forward run recording the nodal velocity b_i(l) = -(p_{l+1,i} - p_{l,i}) / dt at the
 * listed nodes (the auxiliary source of App. A-1 in its exact form), out (nsteps, nnodes). */
int orc_record_velocity(int d, i64 n, i64 m, const i32 *elems, const double *vol,
                        const double *grad, const double *zeta, const double *M,
                        const double *r, double dt,
                        i64 nsteps, const i32 *src_nodes, const double *src_w,
                        const double *wavelet, i64 nnodes, const i32 *nodes, double *out)
{
    mesh_t ms;
    if (mesh_init(&ms, d, n, m, elems, vol, grad, zeta)) return -3;
    double *p = calloc(n, sizeof(double)), *pold = calloc(n, sizeof(double));
    double *q = calloc((size_t)m * d, sizeof(double)), *f = calloc(n, sizeof(double));
    if (!p || !pold || !q || !f) return -3;
    for (i64 l = 0; l < nsteps; ++l) {
        for (int a = 0; a <= d; ++a) f[src_nodes[a]] = 0.0;
        for (int a = 0; a <= d; ++a) f[src_nodes[a]] += wavelet[l] * src_w[a];
        memcpy(pold, p, sizeof(double) * n);
        update_q(&ms, dt, p, q, 1);
        update_p(&ms, dt, M, r, q, f, p, 1);
        for (i64 k = 0; k < nnodes; ++k)
            out[l * nnodes + k] = -(p[nodes[k]] - pold[nodes[k]]) / dt;
    }
    free(p); free(pold); free(q); free(f);
    mesh_free(&ms);
    return 0;
}

/* Forward run recording the field p_{l+1,i} at the listed nodes (step (2) of the
 * regularised-deconvolution route of App. A-2 stores the response at a node to a source
 * placed at the receiver), out (nsteps, nnodes). */
int orc_record_field(int d, i64 n, i64 m, const i32 *elems, const double *vol,
                     const double *grad, const double *zeta, const double *M,
                     const double *r, double dt, i64 nsteps, const i32 *src_nodes,
                     const double *src_w, const double *wavelet, i64 nnodes, const i32 *nodes,
                     double *out)
{
    mesh_t ms;
    if (mesh_init(&ms, d, n, m, elems, vol, grad, zeta)) return -3;
    double *p = calloc(n, sizeof(double));
    double *q = calloc((size_t)m * d, sizeof(double)), *f = calloc(n, sizeof(double));
    if (!p || !q || !f) return -3;
    for (i64 l = 0; l < nsteps; ++l) {
        for (int a = 0; a <= d; ++a) f[src_nodes[a]] = 0.0;
        for (int a = 0; a <= d; ++a) f[src_nodes[a]] += wavelet[l] * src_w[a];
        update_q(&ms, dt, p, q, 1);
        update_p(&ms, dt, M, r, q, f, p, 1);
        for (i64 k = 0; k < nnodes; ++k) out[l * nnodes + k] = p[nodes[k]];
    }
    free(p); free(q); free(f);
    mesh_free(&ms);
    return 0;
}

/* Responses to single-node sources: for each listed node c, a run from rest with the
 * nodal load f_l = e_{node_c} * series_c(l) (series (nnodes, nsteps)), recording the
 * receivers at every step.  out (nnodes, nrec, nsteps).  This is the auxiliary system
 * (linearized1/2) of App. A-1 driven by one node's source term. */
int orc_node_responses(int d, i64 n, i64 m, const i32 *elems, const double *vol,
                       const double *grad, const double *zeta, const double *M,
                       const double *r, double dt,
                       i64 nsteps, i64 nnodes, const i32 *nodes, const double *series,
                       i64 nrec, const i32 *rec_nodes, const double *rec_w, double *out)
{
    mesh_t ms;
    if (mesh_init(&ms, d, n, m, elems, vol, grad, zeta)) return -3;
    int err = 0;
#ifdef _OPENMP
    int inner = nnodes < omp_get_max_threads();
#else
    int inner = 0;
#endif
#pragma omp parallel for schedule(dynamic, 1) if (!inner)
    for (i64 c = 0; c < nnodes; ++c) {
        double *p = calloc(n, sizeof(double)), *q = calloc((size_t)m * d, sizeof(double));
        double *f = calloc(n, sizeof(double));
        if (!p || !q || !f) { err = -3; continue; }
        for (i64 l = 0; l < nsteps; ++l) {
            f[nodes[c]] = series[c * nsteps + l];
            update_q(&ms, dt, p, q, inner);
            update_p(&ms, dt, M, r, q, f, p, inner);
            for (i64 k = 0; k < nrec; ++k)
                out[(c * nrec + k) * nsteps + l] =
                    stencil_dot(d, rec_nodes + k * (d + 1), rec_w + k * (d + 1), p);
        }
        free(p); free(q); free(f);
    }
    mesh_free(&ms);
    return err;
}

/* Thread count of the following calls (n < 1: leave it unchanged). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
