// Host-side operator build (run once per mesh): simplex geometry, the P1 stiffness
// matrix K in node-ordered CSR, the absorbing-boundary damping, the coarse-level maps
// and P1 point stencils.  Sec. II-B (mesh, basis, nesting) and App. A (matrices).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <numeric>
#include <thread>

#include "mgrt_internal.hpp"

namespace mgrt {

void parallel_for(int64_t n, const std::function<void(int64_t, int64_t)> &fn, int64_t grain) {
    if (n <= 0) return;
    unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    int64_t nt = std::min<int64_t>(std::min<int64_t>(hw, 32), std::max<int64_t>(1, n / grain));
    if (nt <= 1) {
        fn(0, n);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (int64_t t = 0; t < nt; ++t) {
        int64_t a = t * chunk, b = std::min(n, a + chunk);
        if (a >= b) break;
        th.emplace_back([&fn, a, b] { fn(a, b); });
    }
    for (auto &x : th) x.join();
}

namespace {

// Gradient of the barycentric coordinate of vertex a: the normal n of the opposite
// facet, scaled so that grad . (x_a - x_b) = 1 for any other vertex b.  |T| follows
// from the same triple (double) product: |n . (x_a - x_b)| / d!.
double simplex_grads(int d, const double *x[4], double g[4][3]) {
    double vol = 0;
    for (int a = 0; a <= d; ++a) {
        int o[3], k = 0;
        for (int b = 0; b <= d; ++b)
            if (b != a) o[k++] = b;
        double nrm[3] = {0, 0, 0};
        if (d == 2) {
            double ex = x[o[1]][0] - x[o[0]][0], ey = x[o[1]][1] - x[o[0]][1];
            nrm[0] = -ey;
            nrm[1] = ex;
        } else {
            double u[3], v[3];
            for (int c = 0; c < 3; ++c) {
                u[c] = x[o[1]][c] - x[o[0]][c];
                v[c] = x[o[2]][c] - x[o[0]][c];
            }
            nrm[0] = u[1] * v[2] - u[2] * v[1];
            nrm[1] = u[2] * v[0] - u[0] * v[2];
            nrm[2] = u[0] * v[1] - u[1] * v[0];
        }
        double h = 0;
        for (int c = 0; c < d; ++c) h += nrm[c] * (x[a][c] - x[o[0]][c]);
        if (h == 0.0) return 0.0;
        for (int c = 0; c < d; ++c) g[a][c] = nrm[c] / h;
        if (a == 0) vol = std::fabs(h) / (d == 2 ? 2.0 : 6.0);
    }
    return vol;
}

// Barycentric coordinates of y in the simplex with vertices x (via the gradients).
void barycentric(int d, const double *x[4], const double g[4][3], const double *y, double *lam) {
    // lambda_a(y) = 1 - grad_a . (x_a - y)   (lambda_a(x_a) = 1, linear)
    for (int a = 0; a <= d; ++a) {
        double s = 1.0;
        for (int c = 0; c < d; ++c) s -= g[a][c] * (x[a][c] - y[c]);
        lam[a] = s;
    }
}

}  // namespace

void build_host_mesh(HostMesh &hm, int d, int64_t n, const double *coords, int64_t m,
                     const int32_t *elems, int64_t nb, const int32_t *bfacets,
                     const double *admittance, int64_t nc, const int32_t *coarse_of_elem,
                     const int32_t *coarse_verts) {
    hm = HostMesh();
    hm.d = d;
    hm.n = n;
    hm.m = m;
    hm.nb = nb;
    hm.nc = nc;
    const int V = d + 1;
    hm.coords.assign(coords, coords + n * d);
    hm.elems.assign(elems, elems + m * V);
    for (int64_t k = 0; k < m * V; ++k)
        MGRT_REQUIRE(elems[k] >= 0 && elems[k] < n, MGRT_E_MESH, "element node id out of range");

    // geometry
    hm.vol.resize(m);
    hm.grad.resize(m * V * d);
    std::atomic<int> bad{0};
    parallel_for(m, [&](int64_t a0, int64_t a1) {
        for (int64_t t = a0; t < a1; ++t) {
            const double *x[4];
            double g[4][3];
            for (int a = 0; a < V; ++a) x[a] = coords + (int64_t)elems[t * V + a] * d;
            double v = simplex_grads(d, x, g);
            if (!(v > 0.0) || !std::isfinite(v)) bad = 1;
            hm.vol[t] = v;
            for (int a = 0; a < V; ++a)
                for (int c = 0; c < d; ++c) hm.grad[(t * V + a) * d + c] = g[a][c];
        }
    });
    MGRT_REQUIRE(!bad, MGRT_E_MESH, "degenerate (zero-volume) element");

    // node -> element adjacency
    hm.n2e_ptr.assign(n + 1, 0);
    for (int64_t k = 0; k < m * V; ++k) hm.n2e_ptr[elems[k] + 1]++;
    for (int64_t i = 0; i < n; ++i) hm.n2e_ptr[i + 1] += hm.n2e_ptr[i];
    hm.n2e_idx.resize(m * V);
    {
        std::vector<int64_t> fill(hm.n2e_ptr.begin(), hm.n2e_ptr.end() - 1);
        for (int64_t k = 0; k < m * V; ++k) hm.n2e_idx[fill[elems[k]]++] = k;
    }

    // stiffness K_ij = sum_T |T| grad phi_i . grad phi_j, assembled row by row
    hm.kdiag.assign(n, 0.0);
    std::vector<int32_t> rowlen(n, 0);
    const int nthreads_rows = 64;   // row blocks, assembled independently then concatenated
    std::vector<std::vector<int32_t>> blk_col(nthreads_rows);
    std::vector<std::vector<double>> blk_val(nthreads_rows);
    int64_t rb = (n + nthreads_rows - 1) / nthreads_rows;
    parallel_for(nthreads_rows, [&](int64_t b0, int64_t b1) {
        std::vector<std::pair<int32_t, double>> ent;
        for (int64_t blk = b0; blk < b1; ++blk) {
            int64_t i0 = blk * rb, i1 = std::min(n, i0 + rb);
            for (int64_t i = i0; i < i1; ++i) {
                ent.clear();
                double diag = 0.0;
                for (int64_t k = hm.n2e_ptr[i]; k < hm.n2e_ptr[i + 1]; ++k) {
                    int64_t t = hm.n2e_idx[k] / V;
                    int a = (int)(hm.n2e_idx[k] % V);
                    const double *ga = &hm.grad[(t * V + a) * d];
                    for (int b = 0; b < V; ++b) {
                        const double *gb = &hm.grad[(t * V + b) * d];
                        double s = 0;
                        for (int c = 0; c < d; ++c) s += ga[c] * gb[c];
                        s *= hm.vol[t];
                        if (b == a) diag += s;
                        else ent.emplace_back(elems[t * V + b], s);
                    }
                }
                std::sort(ent.begin(), ent.end(),
                          [](const auto &u, const auto &v) { return u.first < v.first; });
                hm.kdiag[i] = diag;
                int32_t len = 0;
                for (size_t q = 0; q < ent.size();) {
                    int32_t j = ent[q].first;
                    double s = 0;
                    while (q < ent.size() && ent[q].first == j) s += ent[q++].second;
                    // entries that vanish up to rounding (e.g. the hypotenuse edges of right
                    // simplices) are structural zeros of K and are dropped
                    if (std::fabs(s) > 1e-14 * std::fabs(diag)) {
                        blk_col[blk].push_back(j);
                        blk_val[blk].push_back(s);
                        ++len;
                    }
                }
                rowlen[i] = len;
            }
        }
    }, 1);
    hm.krow.assign(n + 1, 0);
    for (int64_t i = 0; i < n; ++i) hm.krow[i + 1] = hm.krow[i] + rowlen[i];
    hm.kcol.resize(hm.krow[n]);
    hm.kval.resize(hm.krow[n]);
    for (int blk = 0; blk < nthreads_rows; ++blk) {
        int64_t i0 = blk * rb;
        if (i0 >= n) break;
        std::copy(blk_col[blk].begin(), blk_col[blk].end(), hm.kcol.begin() + hm.krow[i0]);
        std::copy(blk_val[blk].begin(), blk_val[blk].end(), hm.kval.begin() + hm.krow[i0]);
    }

    // absorbing boundary: Y_F |F| / d per facet node (row-sum lumped facet mass)
    hm.rbound.assign(n, 0.0);
    for (int64_t f = 0; f < nb; ++f) {
        const int32_t *v = bfacets + f * d;
        for (int a = 0; a < d; ++a)
            MGRT_REQUIRE(v[a] >= 0 && v[a] < n, MGRT_E_MESH, "boundary facet node out of range");
        double meas;
        const double *x0 = coords + (int64_t)v[0] * d, *x1 = coords + (int64_t)v[1] * d;
        if (d == 2) {
            meas = std::hypot(x1[0] - x0[0], x1[1] - x0[1]);
        } else {
            const double *x2 = coords + (int64_t)v[2] * d;
            double u[3], w[3];
            for (int c = 0; c < 3; ++c) { u[c] = x1[c] - x0[c]; w[c] = x2[c] - x0[c]; }
            double cx = u[1] * w[2] - u[2] * w[1], cy = u[2] * w[0] - u[0] * w[2],
                   cz = u[0] * w[1] - u[1] * w[0];
            meas = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
        }
        double y = admittance ? admittance[f] : 1.0;
        MGRT_REQUIRE(std::isfinite(y) && y >= 0, MGRT_E_ARG, "admittance must be finite and >= 0");
        for (int a = 0; a < d; ++a) hm.rbound[v[a]] += y * meas / d;
    }

    // coarse level (T' of Sec. II-B)
    if (nc > 0) {
        MGRT_REQUIRE(coarse_of_elem && coarse_verts, MGRT_E_ARG, "coarse maps missing");
        hm.coarse_of_elem.assign(coarse_of_elem, coarse_of_elem + m);
        hm.coarse_verts.assign(coarse_verts, coarse_verts + nc * V);
        for (int64_t k = 0; k < nc * V; ++k)
            MGRT_REQUIRE(coarse_verts[k] >= 0 && coarse_verts[k] < n, MGRT_E_MESH,
                         "coarse vertex id out of range");
        hm.cvol.resize(nc);
        std::vector<double> cg(nc * V * d);
        std::atomic<int> cbad{0};
        parallel_for(nc, [&](int64_t a0, int64_t a1) {
            for (int64_t j = a0; j < a1; ++j) {
                const double *x[4];
                double g[4][3];
                for (int a = 0; a < V; ++a) x[a] = coords + (int64_t)coarse_verts[j * V + a] * d;
                double v = simplex_grads(d, x, g);
                if (!(v > 0.0)) cbad = 1;
                hm.cvol[j] = v;
                for (int a = 0; a < V; ++a)
                    for (int c = 0; c < d; ++c) cg[(j * V + a) * d + c] = g[a][c];
            }
        });
        MGRT_REQUIRE(!cbad, MGRT_E_MESH, "degenerate coarse element");
        // nesting: every vertex of a fine element lies in its coarse element
        std::atomic<int> nest_bad{0}, range_bad{0};
        parallel_for(m, [&](int64_t a0, int64_t a1) {
            for (int64_t t = a0; t < a1; ++t) {
                int32_t j = coarse_of_elem[t];
                if (j < 0 || j >= nc) { range_bad = 1; continue; }
                const double *x[4];
                double g[4][3];
                for (int a = 0; a < V; ++a) {
                    x[a] = coords + (int64_t)coarse_verts[(int64_t)j * V + a] * d;
                    for (int c = 0; c < d; ++c) g[a][c] = cg[((int64_t)j * V + a) * d + c];
                }
                for (int a = 0; a < V; ++a) {
                    double lam[4];
                    barycentric(d, x, g, coords + (int64_t)elems[t * V + a] * d, lam);
                    for (int b = 0; b < V; ++b)
                        if (lam[b] < -1e-9) nest_bad = 1;
                }
            }
        });
        MGRT_REQUIRE(!range_bad, MGRT_E_MESH, "coarse element id out of range");
        MGRT_REQUIRE(!nest_bad, MGRT_E_MESH, "fine element not inside its coarse element");
        hm.cnodes.assign(coarse_verts, coarse_verts + nc * V);
        std::sort(hm.cnodes.begin(), hm.cnodes.end());
        hm.cnodes.erase(std::unique(hm.cnodes.begin(), hm.cnodes.end()), hm.cnodes.end());
        hm.cvert_idx.resize(nc * V);
        for (int64_t k = 0; k < nc * V; ++k)
            hm.cvert_idx[k] = (int32_t)(std::lower_bound(hm.cnodes.begin(), hm.cnodes.end(),
                                                         coarse_verts[k]) - hm.cnodes.begin());
        hm.c2f_ptr.assign(nc + 1, 0);
        for (int64_t t = 0; t < m; ++t) hm.c2f_ptr[coarse_of_elem[t] + 1]++;
        for (int64_t j = 0; j < nc; ++j) hm.c2f_ptr[j + 1] += hm.c2f_ptr[j];
        hm.c2f_idx.resize(m);
        std::vector<int64_t> fill(hm.c2f_ptr.begin(), hm.c2f_ptr.end() - 1);
        for (int64_t t = 0; t < m; ++t) hm.c2f_idx[fill[coarse_of_elem[t]]++] = (int32_t)t;
    }
}

// Stepping order of the nodes.  Each step gathers p at the stiffness neighbours of every
// node; the gathers hit in L2 when the neighbour's row was touched recently, i.e. when
// neighbours are close in the order.  Candidates: the caller's numbering, reverse
// Cuthill-McKee and a Morton (Z-order) curve over the node coordinates.  The score is the
// fraction of stiffness references whose two nodes lie more than FAR rows apart (beyond
// what one XCD's L2 holds of recently read rows at the usual batch widths), then the mean
// distance |i - j|.  The caller's numbering is kept unless a candidate halves its score;
// all inputs and outputs keep the caller's numbering.
static constexpr int64_t FAR = 4096;

static void order_scores(const HostMesh &hm, const std::vector<int32_t> &pos, double &far_frac,
                         double &mean) {
    double s = 0;
    int64_t nfar = 0;
    for (int64_t i = 0; i < hm.n; ++i)
        for (int64_t k = hm.krow[i]; k < hm.krow[i + 1]; ++k) {
            const double dd = std::fabs((double)pos[i] - (double)pos[hm.kcol[k]]);
            s += dd;
            nfar += dd > (double)FAR;
        }
    const double nref = (double)std::max<int64_t>(1, hm.krow[hm.n]);
    mean = s / nref;
    far_frac = (double)nfar / nref;
}

static std::vector<int32_t> rcm_order(const HostMesh &hm) {
    const int64_t n = hm.n;
    std::vector<int32_t> deg(n), order;
    order.reserve(n);
    for (int64_t i = 0; i < n; ++i) deg[i] = (int32_t)(hm.krow[i + 1] - hm.krow[i]);
    std::vector<char> seen(n, 0);
    std::vector<int32_t> byDeg(n);
    std::iota(byDeg.begin(), byDeg.end(), 0);
    std::stable_sort(byDeg.begin(), byDeg.end(), [&](int32_t a, int32_t b) { return deg[a] < deg[b]; });
    std::vector<int32_t> nb;
    for (int32_t start : byDeg) {
        if (seen[start]) continue;
        size_t head = order.size();
        order.push_back(start);
        seen[start] = 1;
        while (head < order.size()) {
            const int32_t v = order[head++];
            nb.clear();
            for (int64_t k = hm.krow[v]; k < hm.krow[v + 1]; ++k)
                if (!seen[hm.kcol[k]]) { nb.push_back(hm.kcol[k]); seen[hm.kcol[k]] = 1; }
            std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
                return deg[a] != deg[b] ? deg[a] < deg[b] : a < b;
            });
            order.insert(order.end(), nb.begin(), nb.end());
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

// bits of x spread to every third (d = 3) or every second (d = 2) position of a 64-bit key
static uint64_t spread_bits(uint64_t x, int d) {
    uint64_t r = 0;
    for (int b = 0; b < (d == 3 ? 21 : 32); ++b) r |= ((x >> b) & 1ull) << (b * d);
    return r;
}

// Morton order: node coordinates quantised to 2^bits cells per axis over the bounding
// box (bits from the node count, 21 at most in 3D), keys interleaved, ties by node id.
static std::vector<int32_t> morton_order(const HostMesh &hm) {
    const int d = hm.d;
    const int64_t n = hm.n;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int c = 0; c < d; ++c) { lo[c] = 1e300; hi[c] = -1e300; }
    for (int64_t i = 0; i < n; ++i)
        for (int c = 0; c < d; ++c) {
            lo[c] = std::min(lo[c], hm.coords[i * d + c]);
            hi[c] = std::max(hi[c], hm.coords[i * d + c]);
        }
    double ext = 0;
    for (int c = 0; c < d; ++c) ext = std::max(ext, hi[c] - lo[c]);
    ext = std::max(ext, 1e-300);
    const double side = std::pow((double)std::max<int64_t>(n, 2), 1.0 / d);
    int bits = 1;
    while ((double)(1ull << bits) < 4.0 * side && bits < (d == 3 ? 21 : 31)) ++bits;
    const double scale = (double)((1ull << bits) - 1) / ext;
    std::vector<std::pair<uint64_t, int32_t>> key(n);
    parallel_for(n, [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) {
            uint64_t k = 0;
            for (int c = 0; c < d; ++c) {
                const uint64_t q = (uint64_t)std::llround((hm.coords[i * d + c] - lo[c]) * scale);
                k |= spread_bits(q, d) << c;
            }
            key[i] = {k, (int32_t)i};
        }
    });
    std::sort(key.begin(), key.end());
    std::vector<int32_t> order(n);
    for (int64_t i = 0; i < n; ++i) order[i] = key[i].second;
    return order;
}

void choose_node_order(HostMesh &hm) {
    const int64_t n = hm.n;
    std::vector<int32_t> ident(n);
    std::iota(ident.begin(), ident.end(), 0);
    double f_best, d_best;
    order_scores(hm, ident, f_best, d_best);
    const double f_in = f_best, d_in = d_best;
    hm.perm = ident;
    hm.iperm = ident;
    hm.reordered = false;
    if (hm.d < 2 || hm.d > 3) return;
    for (int cand = 0; cand < 2; ++cand) {
        std::vector<int32_t> ord = cand == 0 ? rcm_order(hm) : morton_order(hm);
        std::vector<int32_t> pos(n);
        for (int64_t k = 0; k < n; ++k) pos[ord[k]] = (int32_t)k;
        double f, dm;
        order_scores(hm, pos, f, dm);
        // must beat the caller's numbering clearly (half its far fraction, or with a far
        // fraction no worse, half its mean distance) and the best candidate so far
        const bool beats_input = f < 0.5 * f_in || (f <= f_in && dm < 0.5 * d_in);
        const bool beats_best = f < f_best || (f == f_best && dm < d_best);
        if (beats_input && beats_best) {
            f_best = f;
            d_best = dm;
            hm.perm = std::move(ord);
            hm.iperm = std::move(pos);
            hm.reordered = true;
        }
    }
}


// P1 stencil of each point (Sec. II-A point source): the lowest-numbered element whose
// barycentric coordinates are all >= -1e-12.  Candidates are the elements around the
// nearest node and its neighbours (which contain every element holding the point); a
// full scan is the fallback.
// Bucket grid of the nodes: cubic cells of side h over the bounding box, h chosen for
// about one node per cell.
void build_node_grid(HostMesh &hm) {
    const int d = hm.d;
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (int c = 0; c < d; ++c) { lo[c] = 1e300; hi[c] = -1e300; }
    for (int64_t i = 0; i < hm.n; ++i)
        for (int c = 0; c < d; ++c) {
            lo[c] = std::min(lo[c], hm.coords[i * d + c]);
            hi[c] = std::max(hi[c], hm.coords[i * d + c]);
        }
    double vol = 1.0, ext_max = 0.0;
    for (int c = 0; c < d; ++c) {
        vol *= std::max(hi[c] - lo[c], 1e-300);
        ext_max = std::max(ext_max, hi[c] - lo[c]);
    }
    double h = std::pow(vol / (double)hm.n, 1.0 / d);
    if (!(h > 0) || !std::isfinite(h)) h = ext_max > 0 ? ext_max : 1.0;
    int64_t cells = 1;
    for (int c = 0; c < 3; ++c) {
        hm.grid_lo[c] = c < d ? lo[c] : 0.0;
        hm.grid_dim[c] = c < d ? std::max<int64_t>(1, (int64_t)std::ceil((hi[c] - lo[c]) / h) + 1) : 1;
        cells *= hm.grid_dim[c];
    }
    hm.grid_h = h;
    auto cell_of = [&](int64_t i) {
        int64_t lin = 0, stride = 1;
        for (int c = 0; c < d; ++c) {
            int64_t k = (int64_t)std::floor((hm.coords[i * d + c] - hm.grid_lo[c]) / h);
            k = std::min(std::max<int64_t>(k, 0), hm.grid_dim[c] - 1);
            lin += k * stride;
            stride *= hm.grid_dim[c];
        }
        return lin;
    };
    hm.grid_ptr.assign(cells + 1, 0);
    for (int64_t i = 0; i < hm.n; ++i) hm.grid_ptr[cell_of(i) + 1]++;
    for (int64_t k = 0; k < cells; ++k) hm.grid_ptr[k + 1] += hm.grid_ptr[k];
    hm.grid_idx.resize(hm.n);
    std::vector<int64_t> fill(hm.grid_ptr.begin(), hm.grid_ptr.end() - 1);
    for (int64_t i = 0; i < hm.n; ++i) hm.grid_idx[fill[cell_of(i)]++] = (int32_t)i;
}

// Nearest node to y: search the grid cells in shells of growing Chebyshev radius around
// y's cell; nodes in shells beyond r are at least r*h away, which ends the search.
static int64_t nearest_node(const HostMesh &hm, const double *y) {
    const int d = hm.d;
    int64_t ci[3] = {0, 0, 0};
    for (int c = 0; c < d; ++c) {
        int64_t k = (int64_t)std::floor((y[c] - hm.grid_lo[c]) / hm.grid_h);
        ci[c] = std::min(std::max<int64_t>(k, 0), hm.grid_dim[c] - 1);
    }
    int64_t best = -1;
    double bd = 1e300;
    const int64_t rmax = std::max(hm.grid_dim[0], std::max(hm.grid_dim[1], hm.grid_dim[2]));
    for (int64_t r = 0; r <= rmax; ++r) {
        const int64_t zr = d == 3 ? r : 0, yr = d >= 2 ? r : 0;
        for (int64_t dz = -zr; dz <= zr; ++dz)
            for (int64_t dy = -yr; dy <= yr; ++dy)
                for (int64_t dx = -r; dx <= r; ++dx) {
                    if (std::max(std::llabs(dx), std::max(std::llabs(dy), std::llabs(dz))) != r) continue;
                    const int64_t x = ci[0] + dx, yy = ci[1] + dy, z = ci[2] + dz;
                    if (x < 0 || x >= hm.grid_dim[0] || yy < 0 || yy >= hm.grid_dim[1] || z < 0 ||
                        z >= hm.grid_dim[2])
                        continue;
                    const int64_t cell = (z * hm.grid_dim[1] + yy) * hm.grid_dim[0] + x;
                    for (int64_t k = hm.grid_ptr[cell]; k < hm.grid_ptr[cell + 1]; ++k) {
                        const int64_t i = hm.grid_idx[k];
                        double s2 = 0;
                        for (int c = 0; c < d; ++c) {
                            const double e = hm.coords[i * d + c] - y[c];
                            s2 += e * e;
                        }
                        if (s2 < bd || (s2 == bd && i < best)) { bd = s2; best = i; }
                    }
                }
        const double reach = (double)r * hm.grid_h;
        if (best >= 0 && bd < reach * reach) break;   // strict: no tie can lie further out
    }
    return best;
}

std::vector<Stencil> locate_points(const HostMesh &hm, int64_t npts, const double *pts) {
    const int d = hm.d, V = d + 1;
    std::vector<Stencil> out(npts);
    std::vector<int> ok(npts, 0);
    auto test_elem = [&](int64_t t, const double *y, double *lam) {
        const double *x[4];
        double g[4][3];
        for (int a = 0; a < V; ++a) {
            x[a] = &hm.coords[(int64_t)hm.elems[t * V + a] * d];
            for (int c = 0; c < d; ++c) g[a][c] = hm.grad[(t * V + a) * d + c];
        }
        barycentric(d, x, g, y, lam);
        for (int a = 0; a < V; ++a)
            if (lam[a] < -1e-12) return false;
        return true;
    };
    parallel_for(npts, [&](int64_t p0, int64_t p1) {
        for (int64_t p = p0; p < p1; ++p) {
            const double *y = pts + p * d;
            const int64_t best = nearest_node(hm, y);
            std::vector<int64_t> cand;
            std::vector<int64_t> ring{best};
            for (int64_t k = hm.n2e_ptr[best]; k < hm.n2e_ptr[best + 1]; ++k) {
                int64_t t = hm.n2e_idx[k] / V;
                for (int a = 0; a < V; ++a) ring.push_back(hm.elems[t * V + a]);
            }
            for (int64_t v : ring)
                for (int64_t k = hm.n2e_ptr[v]; k < hm.n2e_ptr[v + 1]; ++k) cand.push_back(hm.n2e_idx[k] / V);
            std::sort(cand.begin(), cand.end());
            cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
            double lam[4];
            int64_t found = -1;
            for (int64_t t : cand)
                if (test_elem(t, y, lam)) { found = t; break; }
            if (found < 0)
                for (int64_t t = 0; t < hm.m; ++t)
                    if (test_elem(t, y, lam)) { found = t; break; }
            if (found < 0) continue;
            test_elem(found, y, lam);
            for (int a = 0; a < V; ++a) {
                out[p].node[a] = hm.elems[found * V + a];
                out[p].w[a] = lam[a];
            }
            ok[p] = 1;
        }
    });
    for (int64_t p = 0; p < npts; ++p)
        MGRT_REQUIRE(ok[p], MGRT_E_ARG, "point " + std::to_string(p) + " lies outside the mesh");
    return out;
}

}  // namespace mgrt
