// Host-side PolyDG setup: modal basis, quadrature, geometry and SIPG assembly.
//
// Section 3 of the paper defines the broken space P^p(T_h), the penalty of
// eq. (2) and the SIPG form of eq. (3); the system matrix is
// K = (chi_m C_m / dt) M + 1/2 A (the paper's K_h divided by dt).
// This file is an independent C++ implementation of those definitions; it is
// setup work (run once per mesh), not part of the per-step hot path.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

#include "pdg_internal.h"

namespace pdg {

int n_basis(int dim, int p) {
    return dim == 2 ? (p + 1) * (p + 2) / 2 : (p + 1) * (p + 2) * (p + 3) / 6;
}

// Total degree ascending; inside a degree alpha_1 descending, then alpha_2.
void multi_indices(int dim, int p, std::vector<int> &alpha) {
    alpha.clear();
    for (int deg = 0; deg <= p; ++deg) {
        for (int a1 = deg; a1 >= 0; --a1) {
            if (dim == 2) {
                alpha.insert(alpha.end(), {a1, deg - a1, 0});
            } else {
                for (int a2 = deg - a1; a2 >= 0; --a2) alpha.insert(alpha.end(), {a1, a2, deg - a1 - a2});
            }
        }
    }
}

// Gauss-Legendre nodes/weights on [0, 1] by Newton iteration on P_n.
void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0; }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        // recompute derivative at the converged node
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        if (n == 1) { p1 = z; p0 = 1.0; }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        // node on [-1,1] is z; map to [0,1] (ascending order)
        x[n - 1 - i] = 0.5 * (z + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);  // = 0.5 * 2/((1-z^2) P'^2)
    }
}

static void legendre(int p, double t, double *L, double *dL) {
    L[0] = 1.0;
    dL[0] = 0.0;
    if (p >= 1) { L[1] = t; dL[1] = 1.0; }
    for (int k = 1; k < p; ++k) {
        L[k + 1] = ((2.0 * k + 1.0) * t * L[k] - k * L[k - 1]) / (k + 1.0);
        dL[k + 1] = dL[k - 1] + (2.0 * k + 1.0) * L[k];
    }
}

void basis_eval(int dim, int p, const int *alpha, int nd, const double *xi, const double *ext,
                double *phi, double *dphi) {
    double L[3][8], dL[3][8], s[3][8];
    for (int j = 0; j < dim; ++j) {
        legendre(p, xi[j], L[j], dL[j]);
        for (int k = 0; k <= p; ++k) s[j][k] = std::sqrt((2.0 * k + 1.0) / ext[j]);
    }
    for (int b = 0; b < nd; ++b) {
        const int *a = alpha + 3 * b;
        double v = 1.0;
        for (int j = 0; j < dim; ++j) v *= s[j][a[j]] * L[j][a[j]];
        phi[b] = v;
        if (dphi) {
            for (int g = 0; g < dim; ++g) {
                double d = 1.0;
                for (int j = 0; j < dim; ++j)
                    d *= (j == g) ? s[j][a[j]] * dL[j][a[j]] * (2.0 / ext[j]) : s[j][a[j]] * L[j][a[j]];
                dphi[b * dim + g] = d;
            }
        }
    }
}

// Largest eigenvalue of a symmetric 2x2 (closed form) or 3x3 (cyclic Jacobi).
double lambda_max_sym(int dim, const double *S) {
    if (dim == 2) {
        double a = S[0], b = 0.5 * (S[1] + S[2]), d = S[3];
        return 0.5 * (a + d) + std::sqrt(0.25 * (a - d) * (a - d) + b * b);
    }
    double A[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[i][j] = 0.5 * (S[3 * i + j] + S[3 * j + i]);
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        if (off < 1e-30) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (std::fabs(A[p][q]) < 1e-300) continue;
                double th = 0.5 * (A[q][q] - A[p][p]) / A[p][q];
                double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
                double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < 3; ++k) {  // A <- A J
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - sn * akq;
                    A[k][q] = sn * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {  // A <- J^T A
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - sn * aqk;
                    A[q][k] = sn * apk + c * aqk;
                }
            }
    }
    return std::max(A[0][0], std::max(A[1][1], A[2][2]));
}

template <class F>
static void parallel_for(int64_t n, F f, int n_threads = 0) {
    if (n_threads <= 0) n_threads = (int)std::max(1u, std::thread::hardware_concurrency());
    n_threads = (int)std::min<int64_t>(n_threads, std::max<int64_t>(1, n));
    std::atomic<int64_t> next{0};
    auto worker = [&]() {
        for (;;) {
            int64_t i = next.fetch_add(1);
            if (i >= n) break;
            f(i);
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < n_threads; ++t) th.emplace_back(worker);
    worker();
    for (auto &t : th) t.join();
}

static void box_corners(const double *lo, const double *hi, std::vector<double> &pts) {
    for (int m = 0; m < 8; ++m)
        for (int d = 0; d < 3; ++d) pts.push_back(((m >> d) & 1) ? hi[d] : lo[d]);
}

void build_mesh(Mesh &m, const pdg_mesh *in, int p) {
    if (!in) throw Error(PDG_EINVAL, "mesh is NULL");
    if (in->dim != 2 && in->dim != 3) throw Error(PDG_EINVAL, "dim must be 2 or 3");
    if (p < 1 || p > 4) throw Error(PDG_EINVAL, "p must be in 1..4");
    if (in->n_elem <= 0 || !in->cell_ptr || !in->cell_geom || !in->sigma)
        throw Error(PDG_EINVAL, "empty mesh or NULL arrays");
    if (in->n_facet < 0 || (in->n_facet > 0 && (!in->facet_elem || !in->facet_geom || !in->facet_normal)))
        throw Error(PDG_EINVAL, "bad facet arrays");
    const int dim = in->dim;
    m.dim = dim;
    m.p = p;
    m.nd = n_basis(dim, p);
    m.n_elem = in->n_elem;
    m.n_facet = in->n_facet;
    multi_indices(dim, p, m.alpha);
    m.cell_ptr.assign(in->cell_ptr, in->cell_ptr + m.n_elem + 1);
    if (m.cell_ptr[0] != 0) throw Error(PDG_EINVAL, "cell_ptr[0] != 0");
    for (int64_t e = 0; e < m.n_elem; ++e)
        if (m.cell_ptr[e + 1] <= m.cell_ptr[e]) throw Error(PDG_EINVAL, "element without sub-cells");
    const int64_t n_cell = m.cell_ptr[m.n_elem];
    const int cg = dim == 2 ? 6 : 6;  // 3 vertices x 2 or 2 corners x 3
    m.cell_geom.assign(in->cell_geom, in->cell_geom + n_cell * cg);
    m.facet_elem.assign(in->facet_elem, in->facet_elem + 2 * m.n_facet);
    m.facet_geom.assign(in->facet_geom, in->facet_geom + (dim == 2 ? 4 : 6) * m.n_facet);
    m.facet_normal.assign(in->facet_normal, in->facet_normal + dim * m.n_facet);
    m.sigma.assign(in->sigma, in->sigma + m.n_elem * dim * dim);
    for (int64_t f = 0; f < m.n_facet; ++f) {
        int64_t a = m.facet_elem[2 * f], b = m.facet_elem[2 * f + 1];
        if (a < 0 || a >= m.n_elem || b < -1 || b >= m.n_elem || a == b)
            throw Error(PDG_EINVAL, "facet element index out of range");
        double nn = 0;
        for (int d = 0; d < dim; ++d) nn += m.facet_normal[dim * f + d] * m.facet_normal[dim * f + d];
        if (std::fabs(nn - 1.0) > 1e-10) throw Error(PDG_EINVAL, "facet normal is not a unit vector");
    }
    for (int64_t e = 0; e < m.n_elem; ++e) {
        const double *S = &m.sigma[e * dim * dim];
        // SPD check: leading principal minors
        double d1 = S[0];
        double d2 = S[0] * S[dim + 1] - S[1] * S[dim];
        double d3 = dim == 3 ? S[0] * (S[4] * S[8] - S[5] * S[7]) - S[1] * (S[3] * S[8] - S[5] * S[6]) +
                                   S[2] * (S[3] * S[7] - S[4] * S[6])
                             : 1.0;
        if (!(d1 > 0 && d2 > 0 && d3 > 0)) throw Error(PDG_EINVAL, "sigma is not SPD");
    }

    // bounding boxes and diameters
    m.lo.assign(m.n_elem * dim, 0.0);
    m.hi.assign(m.n_elem * dim, 0.0);
    m.hK.assign(m.n_elem, 0.0);
    parallel_for(m.n_elem, [&](int64_t e) {
        std::vector<double> pts;
        for (int64_t c = m.cell_ptr[e]; c < m.cell_ptr[e + 1]; ++c) {
            const double *g = &m.cell_geom[c * 6];
            if (dim == 2) pts.insert(pts.end(), g, g + 6);
            else box_corners(g, g + 3, pts);
        }
        const int64_t nv = (int64_t)pts.size() / dim;
        for (int d = 0; d < dim; ++d) {
            double a = 1e300, b = -1e300;
            for (int64_t v = 0; v < nv; ++v) { a = std::min(a, pts[v * dim + d]); b = std::max(b, pts[v * dim + d]); }
            m.lo[e * dim + d] = a;
            m.hi[e * dim + d] = b;
        }
        double best = 0.0;
        for (int64_t v = 0; v < nv; ++v)
            for (int64_t u = v + 1; u < nv; ++u) {
                double s = 0;
                for (int d = 0; d < dim; ++d) { double t = pts[v * dim + d] - pts[u * dim + d]; s += t * t; }
                best = std::max(best, s);
            }
        m.hK[e] = std::sqrt(best);
    });

    // element quadrature in reference (bbox) coordinates
    std::vector<double> gx, gw;
    const int nq1 = dim == 2 ? p + 2 : p + 1;
    gauss_legendre01(nq1, gx, gw);
    const int per_cell = dim == 2 ? nq1 * nq1 : nq1 * nq1 * nq1;
    m.qp_ptr.assign(m.n_elem + 1, 0);
    for (int64_t e = 0; e < m.n_elem; ++e)
        m.qp_ptr[e + 1] = m.qp_ptr[e] + (m.cell_ptr[e + 1] - m.cell_ptr[e]) * per_cell;
    const int64_t nq = m.qp_ptr[m.n_elem];
    m.qp_xi.assign(nq * dim, 0.0);
    m.qp_w.assign(nq, 0.0);
    m.norm.assign(m.n_elem * m.nd, 0.0);
    parallel_for(m.n_elem, [&](int64_t e) {
        const double *lo = &m.lo[e * dim], *hi = &m.hi[e * dim];
        int64_t q = m.qp_ptr[e];
        for (int64_t c = m.cell_ptr[e]; c < m.cell_ptr[e + 1]; ++c) {
            const double *g = &m.cell_geom[c * 6];
            if (dim == 2) {
                const double *v0 = g, *v1 = g + 2, *v2 = g + 4;
                double e1x = v1[0] - v0[0], e1y = v1[1] - v0[1], e2x = v2[0] - v1[0], e2y = v2[1] - v1[1];
                double det = std::fabs(e1x * e2y - e1y * e2x);
                for (int a = 0; a < nq1; ++a)
                    for (int b = 0; b < nq1; ++b, ++q) {
                        double s = gx[a], t = gx[b];
                        double x[2];
                        for (int d = 0; d < 2; ++d) x[d] = (1 - s) * v0[d] + s * ((1 - t) * v1[d] + t * v2[d]);
                        for (int d = 0; d < 2; ++d) m.qp_xi[q * 2 + d] = 2.0 * (x[d] - lo[d]) / (hi[d] - lo[d]) - 1.0;
                        m.qp_w[q] = gw[a] * gw[b] * s * det;
                    }
            } else {
                const double *blo = g, *bhi = g + 3;
                double vol = (bhi[0] - blo[0]) * (bhi[1] - blo[1]) * (bhi[2] - blo[2]);
                for (int a = 0; a < nq1; ++a)
                    for (int b = 0; b < nq1; ++b)
                        for (int cc = 0; cc < nq1; ++cc, ++q) {
                            const int ii[3] = {a, b, cc};
                            for (int d = 0; d < 3; ++d) {
                                double x = blo[d] + gx[ii[d]] * (bhi[d] - blo[d]);
                                m.qp_xi[q * 3 + d] = 2.0 * (x - lo[d]) / (hi[d] - lo[d]) - 1.0;
                            }
                            m.qp_w[q] = gw[a] * gw[b] * gw[cc] * vol;
                        }
            }
        }
        for (int b = 0; b < m.nd; ++b) {
            double v = 1.0;
            for (int j = 0; j < dim; ++j) v *= std::sqrt((2.0 * m.alpha[3 * b + j] + 1.0) / (hi[j] - lo[j]));
            m.norm[e * m.nd + b] = v;
        }
    });
}

// Facet quadrature (physical points and weights).
static void facet_points(const Mesh &m, int64_t f, std::vector<double> &x, std::vector<double> &w,
                         const std::vector<double> &gx, const std::vector<double> &gw) {
    const int dim = m.dim;
    x.clear();
    w.clear();
    const double *g = &m.facet_geom[f * (dim == 2 ? 4 : 6)];
    const int n = (int)gx.size();
    if (dim == 2) {
        double len = std::hypot(g[2] - g[0], g[3] - g[1]);
        for (int a = 0; a < n; ++a) {
            x.push_back(g[0] + gx[a] * (g[2] - g[0]));
            x.push_back(g[1] + gx[a] * (g[3] - g[1]));
            w.push_back(gw[a] * len);
        }
    } else {
        const double *lo = g, *hi = g + 3;
        int ax = -1;
        for (int d = 0; d < 3; ++d)
            if (hi[d] == lo[d]) { if (ax >= 0) throw Error(PDG_EINVAL, "degenerate 3-D facet"); ax = d; }
        if (ax < 0) throw Error(PDG_EINVAL, "3-D facet is not an axis-aligned rectangle");
        int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
        double e1 = hi[t1] - lo[t1], e2 = hi[t2] - lo[t2];
        for (int a = 0; a < n; ++a)
            for (int b = 0; b < n; ++b) {
                double pt[3];
                pt[ax] = lo[ax];
                pt[t1] = lo[t1] + gx[a] * e1;
                pt[t2] = lo[t2] + gx[b] * e2;
                x.insert(x.end(), pt, pt + 3);
                w.push_back(gw[a] * gw[b] * e1 * e2);
            }
    }
}

void element_inverse(int n, const double *A, double *Ainv) {
    std::vector<double> t(A, A + n * n);
    spd_inverse(n, t.data());
    std::copy(t.begin(), t.end(), Ainv);
}

void assemble(const Mesh &m, double c, double eta0, std::vector<double> &M, Bsr &K) {
    const int dim = m.dim, nd = m.nd, p = m.p;
    const int64_t n = m.n_elem;
    // facets per element and neighbour lists
    std::vector<std::vector<int64_t>> efacets(n);
    std::vector<std::vector<int32_t>> nbrs(n);
    for (int64_t f = 0; f < m.n_facet; ++f) {
        int64_t a = m.facet_elem[2 * f], b = m.facet_elem[2 * f + 1];
        if (b < 0) continue;
        efacets[a].push_back(f);
        efacets[b].push_back(f);
        nbrs[a].push_back((int32_t)b);
        nbrs[b].push_back((int32_t)a);
    }
    K.nd = nd;
    K.n_rows = n;
    K.row_ptr.assign(n + 1, 0);
    for (int64_t e = 0; e < n; ++e) {
        auto &v = nbrs[e];
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
        K.row_ptr[e + 1] = K.row_ptr[e] + 1 + (int64_t)v.size();
    }
    K.nnzb = K.row_ptr[n];
    K.col.assign(K.nnzb, 0);
    for (int64_t e = 0; e < n; ++e) {
        int64_t o = K.row_ptr[e];
        K.col[o] = (int32_t)e;
        for (size_t k = 0; k < nbrs[e].size(); ++k) K.col[o + 1 + k] = nbrs[e][k];
    }
    K.val.assign(K.nnzb * nd * nd, 0.0);
    M.assign(n * nd * nd, 0.0);

    std::vector<double> lam(n);
    for (int64_t e = 0; e < n; ++e) lam[e] = lambda_max_sym(dim, &m.sigma[e * dim * dim]);
    std::vector<double> gx, gw;
    gauss_legendre01(dim == 2 ? p + 2 : p + 1, gx, gw);

    parallel_for(n, [&](int64_t e) {
        const double *lo = &m.lo[e * dim], *hi = &m.hi[e * dim];
        double ext[3];
        for (int d = 0; d < dim; ++d) ext[d] = hi[d] - lo[d];
        const double *S = &m.sigma[e * dim * dim];
        std::vector<double> phi(nd), dphi(nd * dim), sg(nd * dim);
        double *Me = &M[e * nd * nd];
        double *Kd = &K.val[K.row_ptr[e] * nd * nd];  // diagonal block comes first
        std::vector<double> Avol(nd * nd, 0.0);
        for (int64_t q = m.qp_ptr[e]; q < m.qp_ptr[e + 1]; ++q) {
            basis_eval(dim, p, m.alpha.data(), nd, &m.qp_xi[q * dim], ext, phi.data(), dphi.data());
            const double w = m.qp_w[q];
            for (int j = 0; j < nd; ++j)
                for (int a = 0; a < dim; ++a) {
                    double s = 0;
                    for (int b = 0; b < dim; ++b) s += S[a * dim + b] * dphi[j * dim + b];
                    sg[j * dim + a] = s;
                }
            for (int i = 0; i < nd; ++i)
                for (int j = 0; j < nd; ++j) {
                    Me[i * nd + j] += w * phi[i] * phi[j];
                    double s = 0;
                    for (int a = 0; a < dim; ++a) s += dphi[i * dim + a] * sg[j * dim + a];
                    Avol[i * nd + j] += w * s;
                }
        }
        // interior facets touching e: this row's blocks only
        std::vector<double> xq, wq, pm(nd), pp(nd), dm(nd * dim), dp(nd * dim), gm(nd), gp(nd);
        std::vector<double> Aee(nd * nd, 0.0);
        for (int64_t f : efacets[e]) {
            const int64_t a = m.facet_elem[2 * f], b = m.facet_elem[2 * f + 1];
            const bool minus = (a == e);
            const int64_t o = minus ? b : a;
            const double *nrm = &m.facet_normal[f * dim];
            double exa[3], exb[3];
            for (int d = 0; d < dim; ++d) {
                exa[d] = m.hi[a * dim + d] - m.lo[a * dim + d];
                exb[d] = m.hi[b * dim + d] - m.lo[b * dim + d];
            }
            double Sna[3], Snb[3];  // Sigma n on each side (Sigma symmetric)
            for (int d = 0; d < dim; ++d) {
                Sna[d] = Snb[d] = 0;
                for (int k = 0; k < dim; ++k) {
                    Sna[d] += m.sigma[a * dim * dim + d * dim + k] * nrm[k];
                    Snb[d] += m.sigma[b * dim * dim + d * dim + k] * nrm[k];
                }
            }
            const double ha = m.hK[a], hb = m.hK[b];
            const double eta = eta0 * 0.5 * (lam[a] + lam[b]) * p * p / (2.0 * ha * hb / (ha + hb));
            // block position of (e, o) in row e
            int64_t pos = -1;
            for (int64_t k = K.row_ptr[e]; k < K.row_ptr[e + 1]; ++k)
                if (K.col[k] == (int32_t)o) { pos = k; break; }
            double *Keo = &K.val[pos * nd * nd];
            facet_points(m, f, xq, wq, gx, gw);
            for (size_t q = 0; q < wq.size(); ++q) {
                double xia[3], xib[3];
                for (int d = 0; d < dim; ++d) {
                    xia[d] = 2.0 * (xq[q * dim + d] - m.lo[a * dim + d]) / exa[d] - 1.0;
                    xib[d] = 2.0 * (xq[q * dim + d] - m.lo[b * dim + d]) / exb[d] - 1.0;
                }
                basis_eval(dim, p, m.alpha.data(), nd, xia, exa, pm.data(), dm.data());
                basis_eval(dim, p, m.alpha.data(), nd, xib, exb, pp.data(), dp.data());
                for (int j = 0; j < nd; ++j) {
                    double s1 = 0, s2 = 0;
                    for (int d = 0; d < dim; ++d) { s1 += dm[j * dim + d] * Sna[d]; s2 += dp[j * dim + d] * Snb[d]; }
                    gm[j] = s1;  // (Sigma^- grad phi^-_j) . n
                    gp[j] = s2;  // (Sigma^+ grad phi^+_j) . n
                }
                const double w = wq[q];
                // trial j, test i.  [v] = (v^- - v^+) n, {Sigma grad u} = (g^- + g^+)/2
                for (int i = 0; i < nd; ++i)
                    for (int j = 0; j < nd; ++j) {
                        double self, cross;
                        if (minus) {
                            self = -0.5 * gm[j] * pm[i] - 0.5 * pm[j] * gm[i] + eta * pm[j] * pm[i];
                            cross = -0.5 * gp[j] * pm[i] + 0.5 * pp[j] * gm[i] - eta * pp[j] * pm[i];
                        } else {
                            self = 0.5 * gp[j] * pp[i] + 0.5 * pp[j] * gp[i] + eta * pp[j] * pp[i];
                            cross = 0.5 * gm[j] * pp[i] - 0.5 * pm[j] * gp[i] - eta * pm[j] * pp[i];
                        }
                        Aee[i * nd + j] += w * self;
                        Keo[i * nd + j] += 0.5 * w * cross;
                    }
            }
        }
        for (int k = 0; k < nd * nd; ++k) Kd[k] = c * Me[k] + 0.5 * (Avol[k] + Aee[k]);
    });
}

}  // namespace pdg
