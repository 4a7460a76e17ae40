// Host-side setup of the two-level additive Schwarz preconditioner of
// Section 4, eq. (5):
//   local level:  K_i = principal submatrix of K on the dofs of subdomain i;
//   coarse level: P = exact L^2 injection of P^q on each coarse agglomerate
//                 (same modal basis on the agglomerate's bounding box),
//                 K_0 = P^T K P.
// Every K_i and K_0 is inverted densely in FP64 (Cholesky, then the inverse of
// the factor) and stored as packed lower-triangular 64 x 64 tiles, the layout
// the Schwarz-apply kernel streams.  Setup work, not part of the hot path.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "pdg_internal.h"

namespace pdg {

template <class F>
static void parallel_for(int64_t n, F f, int n_threads) {
    if (n_threads <= 0) n_threads = (int)std::max(1u, std::thread::hardware_concurrency());
    n_threads = (int)std::min<int64_t>(n_threads, std::max<int64_t>(1, n));
    std::atomic<int64_t> next{0};
    std::atomic<int> failed{0};
    Error first(PDG_OK, "");
    auto worker = [&]() {
        for (;;) {
            int64_t i = next.fetch_add(1);
            if (i >= n || failed.load()) break;
            try {
                f(i);
            } catch (Error &e) {
                if (failed.exchange(1) == 0) first = e;
            }
        }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < n_threads; ++t) th.emplace_back(worker);
    worker();
    for (auto &t : th) t.join();
    if (failed.load()) throw first;
}

static inline double dot(const double *a, const double *b, int64_t n) {
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    int64_t k = 0;
    for (; k + 4 <= n; k += 4) {
        s0 += a[k] * b[k];
        s1 += a[k + 1] * b[k + 1];
        s2 += a[k + 2] * b[k + 2];
        s3 += a[k + 3] * b[k + 3];
    }
    for (; k < n; ++k) s0 += a[k] * b[k];
    return (s0 + s1) + (s2 + s3);
}

// A (row-major, SPD) -> A^{-1}.  Cholesky A = L L^T column by column (the
// entries below each pivot are independent), then the rows of
// W^T = (L^{-1})^T by forward substitution (independent per row), then
// A^{-1} = W^T W (independent per row).  With n_threads > 1 the independent
// parts run on that many threads; every entry is formed by the same
// expression in the same order either way, so the result does not depend on
// the thread count.
void spd_inverse(int64_t n, double *A, int n_threads) {
    std::vector<double> L(n * n, 0.0);
    const bool par = n_threads > 1 && n >= 256;
    for (int64_t j = 0; j < n; ++j) {
        double *Lj = &L[j * n];
        const double s = A[j * n + j] - dot(Lj, Lj, j);
        if (!(s > 0.0) || !std::isfinite(s)) throw Error(PDG_ENOTSPD, "Cholesky pivot <= 0 (matrix not SPD)");
        Lj[j] = std::sqrt(s);
        auto below = [&](int64_t i) {
            double *Li = &L[i * n];
            Li[j] = (A[i * n + j] - dot(Li, Lj, j)) / Lj[j];
        };
        const int64_t rows = n - j - 1;
        if (par && rows * j >= (1 << 16)) {
            const int64_t blk = 16, nb = (rows + blk - 1) / blk;
            parallel_for(nb, [&](int64_t b) {
                for (int64_t i = j + 1 + b * blk; i < std::min(n, j + 1 + (b + 1) * blk); ++i) below(i);
            }, n_threads);
        } else {
            for (int64_t i = j + 1; i < n; ++i) below(i);
        }
    }
    // Wt[j][k] = (L^{-1})[k][j], k >= j: solve L w = e_j
    std::vector<double> Wt(n * n, 0.0);
    auto wrow = [&](int64_t j, std::vector<double> &w) {
        std::fill(w.begin(), w.end(), 0.0);
        w[j] = 1.0 / L[j * n + j];
        for (int64_t k = j + 1; k < n; ++k) {
            const double *Lk = &L[k * n];
            w[k] = -dot(Lk + j, &w[j], k - j) / Lk[k];
        }
        std::copy(w.begin() + j, w.end(), &Wt[j * n + j]);
    };
    // A^{-1}[i][j] = sum_{k >= max(i,j)} Wt[i][k] Wt[j][k]
    auto prow = [&](int64_t i) {
        for (int64_t j = 0; j <= i; ++j) {
            double s = dot(&Wt[i * n + i], &Wt[j * n + i], n - i);
            A[i * n + j] = s;
            A[j * n + i] = s;
        }
    };
    if (par) {
        parallel_for(n, [&](int64_t j) {
            thread_local std::vector<double> w;
            w.resize(n);
            wrow(j, w);
        }, n_threads);
        parallel_for(n, prow, n_threads);
    } else {
        std::vector<double> w(n);
        for (int64_t j = 0; j < n; ++j) wrow(j, w);
        for (int64_t i = 0; i < n; ++i) prow(i);
    }
}

// Cholesky factorisation of the SPD matrix A (row-major n x n) in its lower
// triangle, in place; false at the first pivot that is not positive.
static bool cholesky_in_place(int64_t n, double *A) {
    for (int64_t j = 0; j < n; ++j) {
        double *Aj = &A[j * n];
        const double s = Aj[j] - dot(Aj, Aj, j);
        if (!(s > 0.0) || !std::isfinite(s)) return false;
        Aj[j] = std::sqrt(s);
        for (int64_t i = j + 1; i < n; ++i) {
            double *Ai = &A[i * n];
            Ai[j] = (Ai[j] - dot(Ai, Aj, j)) / Aj[j];
        }
    }
    return true;
}

// BF16 form of the inverse D (row-major n x n, SPD) of a local system:
// d_j = sqrt(D_jj) (rounded to FP32) into ds, the packed tiles of
// C = diag(d)^{-1} D diag(d)^{-1} rounded to BF16 into tiles; true if the
// rounded C minus margin * I is positive definite.  Overwrites D.
static bool bf16_scaled_tiles(double *D, int64_t n, double margin, float *ds, uint16_t *tiles) {
    for (int64_t j = 0; j < n; ++j) ds[j] = (float)std::sqrt(D[j * n + j]);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j <= i; ++j) {
            const double v = bf16_value(bf16_bits(D[i * n + j] / ((double)ds[i] * (double)ds[j])));
            D[i * n + j] = v;
            D[j * n + i] = v;
        }
    const int64_t nt = (n + kTile - 1) / kTile;
    for (int64_t I = 0; I < nt; ++I)
        for (int64_t J = 0; J <= I; ++J) {
            uint16_t *t = tiles + (I * (I + 1) / 2 + J) * kTile * kTile;
            for (int r = 0; r < kTile; ++r)
                for (int c = 0; c < kTile; ++c) {
                    const int64_t gr = I * kTile + r, gc = J * kTile + c;
                    t[r * kTile + c] = (gr < n && gc < n) ? bf16_bits(D[gr * n + gc]) : (uint16_t)0;
                }
        }
    for (int64_t j = 0; j < n; ++j) D[j * n + j] -= margin;
    return cholesky_in_place(n, D);
}

static void store_tiles(const double *D, int64_t n, double *tiles) {
    const int64_t nt = (n + kTile - 1) / kTile;
    for (int64_t I = 0; I < nt; ++I)
        for (int64_t J = 0; J <= I; ++J) {
            double *t = tiles + (I * (I + 1) / 2 + J) * kTile * kTile;
            for (int r = 0; r < kTile; ++r)
                for (int c = 0; c < kTile; ++c) {
                    int64_t gr = I * kTile + r, gc = J * kTile + c;
                    t[r * kTile + c] = (gr < n && gc < n) ? D[gr * n + gc] : 0.0;
                }
        }
}

void dense_inverse_of_system(const Precond &pc, int s, std::vector<double> &out) {
    const DenseSys &S = pc.sys[s];
    out.assign(S.n * S.n, 0.0);
    for (int64_t I = 0; I < S.nt; ++I)
        for (int64_t J = 0; J <= I; ++J) {
            const double *t = &pc.inv64[(S.tile_off + I * (I + 1) / 2 + J) * kTile * kTile];
            for (int r = 0; r < kTile; ++r)
                for (int c = 0; c < kTile; ++c) {
                    int64_t gr = I * kTile + r, gc = J * kTile + c;
                    if (gr < S.n && gc < S.n) {
                        out[gr * S.n + gc] = t[r * kTile + c];
                        out[gc * S.n + gr] = t[r * kTile + c];
                    }
                }
        }
}

void setup_precond(const Mesh &m, const Bsr &K, const std::vector<double> &Mblk,
                   const pdg_precond_desc *d, const std::vector<int32_t> &elem_bsys, int n_bsys, Precond &pc,
                   int n_threads, double bf16_margin) {
    if (!d || d->n_sub < 1 || !d->elem_sub) throw Error(PDG_EINVAL, "bad preconditioner descriptor");
    const int64_t n = m.n_elem;
    const int nd = m.nd, dim = m.dim;
    for (int pr : {d->local_prec, d->coarse_prec})
        if (pr != PDG_F64 && pr != PDG_F32 && pr != PDG_BF16) throw Error(PDG_EINVAL, "bad precision");
    if (d->coarse_prec == PDG_BF16) throw Error(PDG_EINVAL, "coarse precision must be F64 or F32");
    if (d->coarse_q < 0 || d->coarse_q > m.p) throw Error(PDG_EINVAL, "coarse_q must be in 0..p");
    pc = Precond();
    pc.n_sub = d->n_sub;
    pc.local_prec = d->local_prec;
    pc.coarse_prec = d->coarse_prec;
    pc.q = d->coarse_q;
    pc.n_bsys = n_bsys;

    // subdomain CSR (elements in ascending order inside a subdomain)
    std::vector<int32_t> cnt(pc.n_sub, 0);
    for (int64_t e = 0; e < n; ++e) {
        int s = d->elem_sub[e];
        if (s < 0 || s >= pc.n_sub) throw Error(PDG_EINVAL, "elem_sub label out of range");
        cnt[s]++;
    }
    pc.sub_ptr.assign(pc.n_sub + 1, 0);
    for (int s = 0; s < pc.n_sub; ++s) {
        if (cnt[s] == 0) throw Error(PDG_EINVAL, "empty subdomain");
        if ((int64_t)cnt[s] * nd > kMaxLocalDofs) throw Error(PDG_EINVAL, "subdomain exceeds 6144 dofs");
        pc.sub_ptr[s + 1] = pc.sub_ptr[s] + cnt[s];
    }
    pc.sub_elems.assign(n, 0);
    std::vector<int32_t> fill(pc.sub_ptr.begin(), pc.sub_ptr.end() - 1);
    std::vector<int32_t> pos(n);
    for (int64_t e = 0; e < n; ++e) {
        int s = d->elem_sub[e];
        pos[e] = fill[s] - pc.sub_ptr[s];
        pc.sub_elems[fill[s]++] = (int32_t)e;
    }
    pc.sub_bsys.assign(pc.n_sub, 0);
    for (int s = 0; s < pc.n_sub; ++s) {
        const int b = elem_bsys[pc.sub_elems[pc.sub_ptr[s]]];
        for (int k = pc.sub_ptr[s]; k < pc.sub_ptr[s + 1]; ++k)
            if (elem_bsys[pc.sub_elems[k]] != b) throw Error(PDG_EINVAL, "a subdomain spans two systems");
        pc.sub_bsys[s] = b;
    }

    // system table: locals then (optionally) the coarse system
    const bool coarse = pc.q > 0;
    pc.sys.resize(pc.n_sub + (coarse ? n_bsys : 0));
    int64_t toff = 0;
    for (int s = 0; s < pc.n_sub; ++s) {
        DenseSys &S = pc.sys[s];
        S.n = (int64_t)cnt[s] * nd;
        S.nt = (S.n + kTile - 1) / kTile;
        S.tile_off = toff;
        toff += S.nt * (S.nt + 1) / 2;
    }

    // coarse space
    if (coarse) {
        const int32_t *ec = d->elem_coarse ? d->elem_coarse : d->elem_sub;
        pc.n_coarse = d->elem_coarse ? d->n_coarse : d->n_sub;
        if (pc.n_coarse < 1) throw Error(PDG_EINVAL, "n_coarse < 1");
        std::vector<int32_t> cc(pc.n_coarse, 0), cb(pc.n_coarse, -1);
        for (int64_t e = 0; e < n; ++e) {
            if (ec[e] < 0 || ec[e] >= pc.n_coarse) throw Error(PDG_EINVAL, "elem_coarse label out of range");
            cc[ec[e]]++;
            if (cb[ec[e]] < 0) cb[ec[e]] = elem_bsys[e];
            else if (cb[ec[e]] != elem_bsys[e]) throw Error(PDG_EINVAL, "a coarse element spans two systems");
        }
        for (int c = 0; c < pc.n_coarse; ++c)
            if (cc[c] == 0) throw Error(PDG_EINVAL, "empty coarse element");
        // internal numbering: coarse elements of one system are contiguous
        // (stable in the caller's label order)
        pc.coarse_orig.resize(pc.n_coarse);
        std::iota(pc.coarse_orig.begin(), pc.coarse_orig.end(), 0);
        std::stable_sort(pc.coarse_orig.begin(), pc.coarse_orig.end(),
                         [&](int32_t a, int32_t b) { return cb[a] < cb[b]; });
        pc.cnum.assign(pc.n_coarse, 0);
        for (int k = 0; k < pc.n_coarse; ++k) pc.cnum[pc.coarse_orig[k]] = k;
        pc.csys_ce0.assign(n_bsys + 1, 0);
        for (int c = 0; c < pc.n_coarse; ++c) pc.csys_ce0[cb[c] + 1]++;
        for (int b = 0; b < n_bsys; ++b) {
            if (pc.csys_ce0[b + 1] == 0) throw Error(PDG_EINVAL, "a system has no coarse element");
            pc.csys_ce0[b + 1] += pc.csys_ce0[b];
        }
        pc.elem_coarse.resize(n);
        for (int64_t e = 0; e < n; ++e) pc.elem_coarse[e] = pc.cnum[ec[e]];
        std::vector<int32_t> ccnt(pc.n_coarse, 0);
        for (int64_t e = 0; e < n; ++e) ccnt[pc.elem_coarse[e]]++;
        pc.coarse_ptr.assign(pc.n_coarse + 1, 0);
        for (int c = 0; c < pc.n_coarse; ++c) pc.coarse_ptr[c + 1] = pc.coarse_ptr[c] + ccnt[c];
        pc.coarse_elems.assign(n, 0);
        std::vector<int32_t> cf(pc.coarse_ptr.begin(), pc.coarse_ptr.end() - 1);
        for (int64_t e = 0; e < n; ++e) pc.coarse_elems[cf[pc.elem_coarse[e]]++] = (int32_t)e;
        // coarse bounding boxes
        std::vector<double> clo(pc.n_coarse * dim, 1e300), chi(pc.n_coarse * dim, -1e300);
        for (int64_t e = 0; e < n; ++e)
            for (int k = 0; k < dim; ++k) {
                clo[ec[e] * dim + k] = std::min(clo[ec[e] * dim + k], m.lo[e * dim + k]);
                chi[ec[e] * dim + k] = std::max(chi[ec[e] * dim + k], m.hi[e * dim + k]);
            }
        std::vector<int> alpha0;
        multi_indices(dim, pc.q, alpha0);
        pc.nq0 = n_basis(dim, pc.q);
        const int nq0 = pc.nq0;
        pc.P.assign(n * nd * nq0, 0.0);
        parallel_for(n, [&](int64_t e) {
            const double *lo = &m.lo[e * dim], *hi = &m.hi[e * dim];
            double ext[3], cext[3];
            const int c = ec[e];
            for (int k = 0; k < dim; ++k) { ext[k] = hi[k] - lo[k]; cext[k] = chi[c * dim + k] - clo[c * dim + k]; }
            std::vector<double> G(nd * nq0, 0.0), phi(nd), psi(nq0), Minv(nd * nd);
            for (int64_t q = m.qp_ptr[e]; q < m.qp_ptr[e + 1]; ++q) {
                const double *xi = &m.qp_xi[q * dim];
                double cxi[3];
                for (int k = 0; k < dim; ++k) {
                    double x = lo[k] + 0.5 * (xi[k] + 1.0) * ext[k];
                    cxi[k] = 2.0 * (x - clo[c * dim + k]) / cext[k] - 1.0;
                }
                basis_eval(dim, m.p, m.alpha.data(), nd, xi, ext, phi.data(), nullptr);
                basis_eval(dim, pc.q, alpha0.data(), nq0, cxi, cext, psi.data(), nullptr);
                for (int i = 0; i < nd; ++i)
                    for (int j = 0; j < nq0; ++j) G[i * nq0 + j] += m.qp_w[q] * phi[i] * psi[j];
            }
            element_inverse(nd, &Mblk[e * nd * nd], Minv.data());
            double *PK = &pc.P[e * nd * nq0];
            for (int i = 0; i < nd; ++i)
                for (int j = 0; j < nq0; ++j) {
                    double s = 0;
                    for (int k = 0; k < nd; ++k) s += Minv[i * nd + k] * G[k * nq0 + j];
                    PK[i * nq0 + j] = s;
                }
        }, n_threads);
        // K0 = P^T K P (one dense block per batch system), accumulated
        // row-block by row-block of K
        pc.N0 = (int64_t)pc.n_coarse * nq0;
        pc.K0blk.assign(n_bsys, {});
        for (int b = 0; b < n_bsys; ++b) {
            const int64_t n0 = (int64_t)(pc.csys_ce0[b + 1] - pc.csys_ce0[b]) * nq0;
            if (n0 > kMaxCoarseDofs) throw Error(PDG_EINVAL, "coarse system exceeds 16384 dofs");
            pc.K0blk[b].assign(n0 * n0, 0.0);
        }
        std::vector<double> KP(nd * nq0);
        for (int64_t e = 0; e < n; ++e) {
            const int b = elem_bsys[e];
            const int64_t n0 = (int64_t)(pc.csys_ce0[b + 1] - pc.csys_ce0[b]) * nq0;
            double *K0 = pc.K0blk[b].data();
            const double *Pe = &pc.P[e * nd * nq0];
            for (int64_t k = K.row_ptr[e]; k < K.row_ptr[e + 1]; ++k) {
                const int64_t o = K.col[k];
                const double *Kb = &K.val[k * nd * nd];
                const double *Po = &pc.P[o * nd * nq0];
                for (int i = 0; i < nd; ++i)
                    for (int j = 0; j < nq0; ++j) {
                        double s = 0;
                        for (int t = 0; t < nd; ++t) s += Kb[i * nd + t] * Po[t * nq0 + j];
                        KP[i * nq0 + j] = s;
                    }
                const int64_t r0 = (int64_t)(pc.elem_coarse[e] - pc.csys_ce0[b]) * nq0;
                const int64_t c0 = (int64_t)(pc.elem_coarse[o] - pc.csys_ce0[b]) * nq0;
                for (int a = 0; a < nq0; ++a)
                    for (int bb = 0; bb < nq0; ++bb) {
                        double s = 0;
                        for (int i = 0; i < nd; ++i) s += Pe[i * nq0 + a] * KP[i * nq0 + bb];
                        K0[(r0 + a) * n0 + c0 + bb] += s;
                    }
            }
        }
        for (int b = 0; b < n_bsys; ++b) {
            double *K0 = pc.K0blk[b].data();
            const int64_t n0 = (int64_t)(pc.csys_ce0[b + 1] - pc.csys_ce0[b]) * nq0;
            for (int64_t i = 0; i < n0; ++i)
                for (int64_t j = 0; j < i; ++j) {
                    double s = 0.5 * (K0[i * n0 + j] + K0[j * n0 + i]);
                    K0[i * n0 + j] = K0[j * n0 + i] = s;
                }
            DenseSys &S = pc.sys[pc.n_sub + b];
            S.n = n0;
            S.nt = (n0 + kTile - 1) / kTile;
            S.tile_off = toff;
            toff += S.nt * (S.nt + 1) / 2;
        }
    }
    pc.n_tiles = toff;
    pc.inv64.assign(pc.n_tiles * kTile * kTile, 0.0);
    const bool b16 = pc.local_prec == PDG_BF16;
    if (b16) {
        int64_t rows = 0, loc_tiles = 0;
        pc.rbase.assign(pc.n_sub, 0);
        for (int s = 0; s < pc.n_sub; ++s) {
            pc.rbase[s] = rows;
            rows += pc.sys[s].nt * kTile;
            loc_tiles += pc.sys[s].nt * (pc.sys[s].nt + 1) / 2;
        }
        pc.dscale.assign(rows, 0.0f);
        pc.tiles_b16.assign(loc_tiles * kTile * kTile, 0);
        pc.fallback.assign(pc.n_sub, 0);
    }

    // local inverses (parallel over subdomains)
    parallel_for(pc.n_sub, [&](int64_t s) {
        const int64_t ni = pc.sys[s].n;
        std::vector<double> D(ni * ni, 0.0);
        for (int32_t le = 0; le < cnt[s]; ++le) {
            const int32_t e = pc.sub_elems[pc.sub_ptr[s] + le];
            for (int64_t k = K.row_ptr[e]; k < K.row_ptr[e + 1]; ++k) {
                const int32_t o = K.col[k];
                if (d->elem_sub[o] != s) continue;
                const int32_t lo = pos[o];
                const double *Kb = &K.val[k * nd * nd];
                for (int i = 0; i < nd; ++i)
                    for (int j = 0; j < nd; ++j) D[(int64_t)(le * nd + i) * ni + lo * nd + j] = Kb[i * nd + j];
            }
        }
        spd_inverse(ni, D.data());
        store_tiles(D.data(), ni, &pc.inv64[pc.sys[s].tile_off * kTile * kTile]);
        if (b16)  // local tiles come first, so tile_off is also the offset in the local store
            pc.fallback[s] = bf16_scaled_tiles(D.data(), ni, bf16_margin, &pc.dscale[pc.rbase[s]],
                                               &pc.tiles_b16[pc.sys[s].tile_off * kTile * kTile])
                                 ? 0
                                 : 1;
    }, n_threads);
    if (b16) pc.n_fallback = (int)std::count(pc.fallback.begin(), pc.fallback.end(), 1);
    if (coarse) {
        // few coarse systems: threads inside each inverse; many: one each
        const int nt = n_threads <= 0 ? (int)std::max(1u, std::thread::hardware_concurrency()) : n_threads;
        const bool inner = n_bsys < nt;
        auto one = [&](int64_t b) {
            std::vector<double> D = pc.K0blk[b];
            const DenseSys &S = pc.sys[pc.n_sub + b];
            spd_inverse(S.n, D.data(), inner ? nt : 1);
            store_tiles(D.data(), S.n, &pc.inv64[S.tile_off * kTile * kTile]);
        };
        if (inner)
            for (int b = 0; b < n_bsys; ++b) one(b);
        else
            parallel_for(n_bsys, one, n_threads);
    }
}

}  // namespace pdg
