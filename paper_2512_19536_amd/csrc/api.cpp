// C-ABI entry points of libpdg: context, workspace layout, device upload and
// the per-step / per-solve orchestration of the HIP kernels.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "kernels.h"
#include "pdg_internal.h"

using namespace pdg;

namespace {

enum State { S_CREATED = 0, S_MESH = 1, S_ASSEMBLED = 2, S_PRECOND = 3, S_BOUND = 4 };

#define HIPCHK(expr)                                                                           \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess)                                                                  \
            throw Error(PDG_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));         \
    } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    struct Item { size_t off = 0, bytes = 0; };
    std::vector<Item> items;
    size_t total = 0;
    int add(size_t bytes) {
        Item it;
        it.off = total;
        it.bytes = bytes;
        total = align256(total + std::max<size_t>(bytes, 1));
        items.push_back(it);
        return (int)items.size() - 1;
    }
};

// Workspace slots (indices into Layout::items).
struct Ws {
    int grows, gslot, gcol, gval, mass, minv, qpptr, qpxi, qpw, norm, prm, subptr, subel;
    int rtit0, itdot, rowpart;
    int rtk, rtnt, rtcb, colp, tloc, tcoa, P, ecoa, elsys;
    int grpptr, grpel, upsys, cchunk, csys0, rspmv, rupd, ritem, rowner;
    int chunk0, lanc, cbase;
    int x, r, z, p, q, I, t, b, r0p, sc, sca, part, rrpart;
    int tfb, dsc;                 // BF16 local store: FP32 fallback tiles, scales
    int idesc;                    // Schwarz item descriptors
    int updesc;                   // update workgroup records
    int pblk, dsrc, bcsrc;        // p-update block records, fine and coarse value sources
    int spdesc;                   // SpMV workgroup records
};

// State of the PCG run in progress (between pcg_begin and pcg_end).
struct PcgRun {
    double *x = nullptr;        // caller's iterate (written at the end)
    const double *b = nullptr;  // right-hand side kept for the true residual
    bool step = false;
    int maxit = 0;
    int j = 1;                  // next iteration to launch
    int next = 1;               // iterations to launch before the next poll
    bool active = false;
};

}  // namespace

struct pdg_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    int state = S_CREATED;
    std::string err;
    int n_threads = 0;
    // options
    int true_resid = 0, chunk = 4, timing = 0, item_kb = 128, use_graph = 0, spmv_wpg = 4;
    int coarse_split = 3;        // coarse-system items are cut to 1/coarse_split of the item size
                                 // (set at preconditioner setup, changed by the autotuner)
    int prev_iters = 0;
    // host data
    Mesh mesh;
    Bsr K;
    std::vector<double> M, Minv;
    double chi = 1, cm = 1, dt = 1, eta0 = 10, c = 1;
    std::vector<double> ionic;
    bool has_ionic = false;
    Precond pc;
    // batch of independent systems: system s owns elements [sys_elem_ptr[s], sys_elem_ptr[s+1])
    int n_sys = 1;
    std::vector<int64_t> sys_elem_ptr;
    std::vector<int32_t> elem_sys;
    // per-system ranges of units (groups, chunks, items) and of the producer
    // workgroups that own runs of them (one partial per workgroup)
    std::vector<int32_t> r_grp, r_chunk, r_itm;
    std::vector<int32_t> r_spmv, r_upd, r_item, r_owner;
    std::vector<int32_t> spmv_wg_g0, upd_wg_c0;
    // update chunks (element runs inside one coarse element)
    std::vector<int32_t> grp_ptr, grp_elems, upd_sys, cchunk_ptr;
    // Schwarz work items and tile rows
    std::vector<int32_t> it_sys, it_row, it_j0, it_nj, it_own, rt_item0, rt_k, rt_nt, dof_rt, coarse_rt0;
    std::vector<int64_t> rt_cbase;
    // per dense system, as the Schwarz items need them (set at bind)
    std::vector<int32_t> ds_n, ds_f32;
    std::vector<int64_t> ds_toff, ds_cbase, ds_dof0, ds_rbase;
    int max_nj = 1;
    int64_t items_reserved = 0;
    int pre_pq = 0, pre_rz = 0;  // dot products pre-summed by the reduction kernel
    int pre_rr = 0;              // same for (r, r) when no preconditioner is applied
    bool no_precond = false;     // B = I: plain CG
    int lcap = 2048;             // PCG coefficients kept per system (Lanczos estimate)
    int ion_endpoint = 1;        // ion term at 2u^k - u^(k-1) (eq. (4)); 0: at (3u^k - u^(k-1))/2
    int force_presum = 0;        // 1: the reduction kernel pre-sums the dot products at any size
    int bf16_margin_log2 = 10;   // BF16 local store: the rounded scaled inverse must keep
                                 // its eigenvalues above 2^-bf16_margin_log2
    bool lanczos_ok = false;     // device scalars still hold the last solve
    // group-ELL matrix (host staging)
    int G = 1;
    int64_t n_groups = 0, n_slots = 0;
    std::vector<int32_t> grp_rows, grp_col, grp_sys;
    std::vector<int64_t> grp_slot_off;
    std::vector<double> grp_val;
    // device
    Layout lay;
    Ws w{};
    char *ws = nullptr;
    size_t ws_bytes = 0;
    DevMatrix dA{};
    DevScalars *sc = nullptr, *sc_apply = nullptr, *sc_host = nullptr;
    int64_t schwarz_bytes = 0;
    PcgRun run;
    std::vector<DevScalars> last;       // per-system scalars of the last solve
    std::vector<double> last_true;      // per-system true relative residual (-1 if not computed)
    // graph of one chunk of PCG iterations
    hipGraphExec_t gexec = nullptr;
    int gexec_chunk = 0;
    // kernel timing
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
    size_t ev_used = 0;
    std::vector<int64_t> ev_idx;  // launch index (within the solve) of each used pool pair
    int64_t t_seq = 0;            // Schwarz launches of the current solve so far
    int64_t t_launches = 0;
    double t_ms = 0.0;
};

namespace {

void require(const pdg_ctx *c, int st, const char *what) {
    if (!c) throw Error(PDG_EINVAL, "ctx is NULL");
    if (c->state < st) throw Error(PDG_ESTATE, std::string(what) + ": call out of order");
}
void require_gpu(const pdg_ctx *c) {
    require(c, S_BOUND, "compute call");
    if (c->device < 0) throw Error(PDG_ESTATE, "host-only context");
}

template <class F>
pdg_status guard(pdg_ctx *c, F f) {
    try {
        f();
        if (c) c->err.clear();
        return PDG_OK;
    } catch (Error &e) {
        if (c) c->err = e.what();
        return e.code;
    } catch (std::bad_alloc &) {
        if (c) c->err = "host allocation failed";
        return PDG_ENOMEM;
    } catch (std::exception &e) {
        if (c) c->err = e.what();
        return PDG_EINVAL;
    }
}

void drop_graph(pdg_ctx *c) {
    if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
    c->gexec = nullptr;
    c->gexec_chunk = 0;
}

// Workgroups of the update kernel per system (about 8 per CU); the SpMV and
// Schwarz kernels keep one group / item per workgroup (the most loads in flight).
constexpr int kUpdateTarget = 2048;
constexpr int kOnePerWorkgroup = 1 << 30;
// Above this many (consumer workgroup x partial) reads per system, a
// dedicated reduction kernel sums the partials once instead.
constexpr int64_t kRedundantReads = 1 << 22;

// Splits each system's unit range [r_unit[s], r_unit[s+1]) into workgroups
// of per_s = ceil(n_s / target) consecutive units; wg0 receives the first unit
// of every workgroup (+ end), r_wg the workgroup range of each system.  The
// split of a system depends on that system alone, so its partial sums (and
// results) are the same alone or inside a batch.
void split_units(const std::vector<int32_t> &r_unit, int target, std::vector<int32_t> &wg0,
                 std::vector<int32_t> &r_wg) {
    const int n_sys = (int)r_unit.size() - 1;
    wg0.clear();
    r_wg.assign(n_sys + 1, 0);
    for (int b = 0; b < n_sys; ++b) {
        const int64_t n_b = r_unit[b + 1] - r_unit[b];
        const int64_t per = std::max<int64_t>(1, (n_b + target - 1) / target);
        for (int64_t u = r_unit[b]; u < r_unit[b + 1]; u += per) wg0.push_back((int32_t)u);
        r_wg[b + 1] = (int32_t)wg0.size();
    }
    wg0.push_back(r_unit[n_sys]);
}

// Group-ELL form of K: element rows sorted by (system, neighbour count
// descending), cut into groups of G rows that never straddle two systems.
void build_group_ell(pdg_ctx *c) {
    const int nd = c->mesh.nd;
    const int64_t n = c->K.n_rows;
    c->G = nd <= 64 ? 64 / nd : 1;
    const int G = c->G;
    std::vector<int32_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    auto nb = [&](int32_t r) { return c->K.row_ptr[r + 1] - c->K.row_ptr[r]; };
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) {
        if (c->elem_sys[a] != c->elem_sys[b]) return c->elem_sys[a] < c->elem_sys[b];
        return nb(a) > nb(b);
    });
    c->grp_rows.clear();
    c->grp_sys.clear();
    c->r_grp.assign(c->n_sys + 1, 0);
    for (int b = 0; b < c->n_sys; ++b) {
        const int64_t r0 = c->sys_elem_ptr[b], r1 = c->sys_elem_ptr[b + 1];  // rows of b are contiguous in perm
        for (int64_t k = r0; k < r1; k += G) {
            for (int r = 0; r < G; ++r) c->grp_rows.push_back(k + r < r1 ? perm[k + r] : -1);
            c->grp_sys.push_back(b);
        }
        c->r_grp[b + 1] = (int32_t)c->grp_sys.size();
    }
    c->n_groups = (int64_t)c->grp_sys.size();
    split_units(c->r_grp, kOnePerWorkgroup, c->spmv_wg_g0, c->r_spmv);
    c->grp_slot_off.assign(c->n_groups + 1, 0);
    for (int64_t g = 0; g < c->n_groups; ++g) {
        int64_t smax = 0;
        for (int r = 0; r < G; ++r) {
            const int32_t row = c->grp_rows[g * G + r];
            if (row >= 0) smax = std::max<int64_t>(smax, nb(row));
        }
        c->grp_slot_off[g + 1] = c->grp_slot_off[g] + smax;
    }
    c->n_slots = c->grp_slot_off[c->n_groups];
    c->grp_col.assign(c->n_slots * G, 0);
    c->grp_val.assign(c->n_slots * G * nd * nd, 0.0);
    for (int64_t g = 0; g < c->n_groups; ++g) {
        const int64_t s0 = c->grp_slot_off[g], ns = c->grp_slot_off[g + 1] - s0;
        for (int r = 0; r < G; ++r) {
            const int32_t row = c->grp_rows[g * G + r];
            for (int64_t s = 0; s < ns; ++s) {
                int32_t col = row >= 0 ? row : 0;
                const double *blk = nullptr;
                if (row >= 0 && s < nb(row)) {
                    const int64_t k = c->K.row_ptr[row] + s;
                    col = c->K.col[k];
                    blk = &c->K.val[k * nd * nd];
                }
                c->grp_col[(s0 + s) * G + r] = col;
                if (!blk) continue;
                if (nd >= kWideMinNd) {  // G = 1, chunked trial-index-major (kernels.h)
                    const int64_t c0 = s - s % kWideChunk, sl = s - c0;
                    const int64_t nch = std::min<int64_t>(kWideChunk, ns - c0);
                    for (int j = 0; j < nd; ++j)
                        for (int i = 0; i < nd; ++i)
                            c->grp_val[(s0 + c0) * nd * nd + j * nch * nd + sl * nd + i] = blk[i * nd + j];
                } else {
                    for (int j = 0; j < nd; ++j)
                        for (int i = 0; i < nd; ++i)
                            c->grp_val[(s0 + s) * G * nd * nd + (j * G + r) * nd + i] = blk[i * nd + j];
                }
            }
        }
    }
}

// Update chunks: runs of at most 32 elements inside one coarse element (or
// inside one system without a coarse level), in system order.
void plan_chunks(pdg_ctx *c) {
    const int kChunk = std::max(1, 128 / c->mesh.nd);  // about one dof per thread of the update kernel
    const Precond &pc = c->pc;
    c->grp_ptr.assign(1, 0);
    c->grp_elems.clear();
    c->upd_sys.clear();
    c->cchunk_ptr.assign(1, 0);
    auto add_run = [&](const int32_t *el, int64_t cnt, int b) {
        for (int64_t e = 0; e < cnt; e += kChunk) {
            for (int64_t k = e; k < std::min<int64_t>(cnt, e + kChunk); ++k) c->grp_elems.push_back(el[k]);
            c->grp_ptr.push_back((int32_t)c->grp_elems.size());
            c->upd_sys.push_back(b);
        }
    };
    if (pc.q > 0) {
        for (int cc = 0; cc < pc.n_coarse; ++cc) {
            const int a0 = pc.coarse_ptr[cc], a1 = pc.coarse_ptr[cc + 1];
            add_run(&pc.coarse_elems[a0], a1 - a0, c->elem_sys[pc.coarse_elems[a0]]);
            c->cchunk_ptr.push_back((int32_t)c->grp_ptr.size() - 1);
        }
    } else {
        std::vector<int32_t> el(c->mesh.n_elem);
        std::iota(el.begin(), el.end(), 0);
        for (int b = 0; b < c->n_sys; ++b)
            add_run(&el[c->sys_elem_ptr[b]], c->sys_elem_ptr[b + 1] - c->sys_elem_ptr[b], b);
    }
    c->r_chunk.assign(c->n_sys + 1, 0);
    for (int32_t b : c->upd_sys) c->r_chunk[b + 1]++;
    for (int b = 0; b < c->n_sys; ++b) c->r_chunk[b + 1] += c->r_chunk[b];
    split_units(c->r_chunk, kUpdateTarget, c->upd_wg_c0, c->r_upd);
}

// Per system: the update kernel's workgroups each sum the system's SpMV
// partials, the p-update kernel's workgroups its Schwarz shares; where that
// is many reads, the reduction kernel does it once.
void choose_reductions(pdg_ctx *c) {
    int64_t upd = 0, pup = 0, pur = 0;
    const int nd = c->mesh.nd;
    for (int b = 0; b < c->n_sys; ++b) {
        const int64_t n_up = c->r_upd[b + 1] - c->r_upd[b], n_sp = c->r_spmv[b + 1] - c->r_spmv[b];
        const int64_t dofs = (c->sys_elem_ptr[b + 1] - c->sys_elem_ptr[b]) * nd;
        const int64_t n_pu = (dofs + 255) / 256 + 1, n_sw = c->r_item[b + 1] - c->r_item[b];
        upd = std::max(upd, n_up * n_sp);
        pup = std::max(pup, n_pu * n_sw);
        pur = std::max(pur, n_pu * n_up);
    }
    c->pre_pq = c->force_presum || upd > kRedundantReads;
    c->pre_rz = c->force_presum || pup > kRedundantReads;
    c->pre_rr = c->force_presum || pur > kRedundantReads;
}

size_t tile_elem_bytes(int prec) { return prec == PDG_F64 ? 8 : (prec == PDG_F32 ? 4 : 2); }
int store_kind(int prec) { return prec == PDG_F64 ? STORE_F64 : (prec == PDG_F32 ? STORE_F32 : STORE_BF16); }

// Storage precision of dense system sidx (local systems of a BF16 store that
// failed the positive-definiteness check of their rounded form are FP32).
int sys_prec(const Precond &pc, size_t sidx) {
    if ((int)sidx >= pc.n_sub) return pc.coarse_prec;
    if (pc.local_prec == PDG_BF16 && pc.fallback[sidx]) return PDG_F32;
    return pc.local_prec;
}

// Schwarz work items for a target of `kb` KiB of tiles per item: the stored
// tiles (I, J <= I) of each packed tile row, split into even runs.  Order: per
// batch system its coarse system, then its subdomains (ascending), so each
// system's items (and tile rows) are one contiguous range.  Coarse items gather
// their input from the restriction shares, which makes them slower to start;
// launched first and split for a third of the size, they no longer form the
// tail of the grid.  With count_only set, returns the item count and changes
// nothing.
// LDS one Schwarz workgroup may use; items are cut to fit it whatever the
// requested size.
constexpr size_t kSchwarzLdsMax = 65536;
constexpr int kMaxCoarseSplit = 4;

// Largest tile count per item whose LDS fits kSchwarzLdsMax.
int64_t max_tiles_per_item(const pdg_ctx *c) {
    const int ls = store_kind(c->pc.local_prec), cs = store_kind(c->pc.coarse_prec);
    int64_t nj = 1;
    while (schwarz_lds_bytes(ls, cs, (int)nj + 1) <= kSchwarzLdsMax) ++nj;
    return nj;
}

// Coarse items are cut smaller only where the coarse tiles are a small share
// (at most an eighth) of the apply's bytes: there they would otherwise form
// the grid's tail.  Where the coarse system dominates, small items would only
// add per-item latency.
int default_coarse_split(const pdg_ctx *c) {
    const Precond &pc = c->pc;
    double coarse = 0.0, all = 0.0;
    for (size_t s = 0; s < pc.sys.size(); ++s) {
        const double nt = (double)pc.sys[s].nt;
        const double b = nt * (nt + 1.0) / 2.0 * tile_elem_bytes(sys_prec(pc, s));
        all += b;
        if ((int)s >= pc.n_sub) coarse += b;
    }
    return coarse * 8.0 <= all ? 3 : 1;
}

int64_t plan_items(pdg_ctx *c, int kb, bool count_only) {
    const Precond &pc = c->pc;
    const int nd = c->mesh.nd;
    const int64_t nj_cap = max_tiles_per_item(c);
    std::vector<std::vector<int>> subs(c->n_sys);
    for (int s = 0; s < pc.n_sub; ++s) subs[pc.sub_bsys[s]].push_back(s);
    int64_t count = 0;
    if (!count_only) {
        c->it_sys.clear(); c->it_row.clear(); c->it_j0.clear(); c->it_nj.clear(); c->it_own.clear();
        c->rt_item0.assign(1, 0);
        c->rt_k.clear(); c->rt_nt.clear(); c->rt_cbase.clear();
        c->coarse_rt0.assign(c->n_sys, 0);
        c->r_itm.assign(c->n_sys + 1, 0);
        c->max_nj = 1;
    }
    std::vector<int32_t> rt0_of_sub(pc.n_sub, 0);
    int32_t n_rt = 0;
    auto add_sys = [&](int sidx, int b) {
        const int64_t nt = pc.sys[sidx].nt;
        const int prec = sys_prec(pc, sidx);
        int64_t jc = std::max<int64_t>(1, ((int64_t)kb * 1024) / (kTile * kTile * (int64_t)tile_elem_bytes(prec)));
        if (sidx >= pc.n_sub) jc = std::max<int64_t>(1, jc / c->coarse_split);
        jc = std::min(jc, nj_cap);
        for (int64_t I = 0; I < nt; ++I) {
            const int64_t ntile = I + 1, nc = (ntile + jc - 1) / jc;
            count += nc;
            ++n_rt;
            if (count_only) continue;
            for (int64_t k = 0; k < nc; ++k) {
                const int64_t j0 = k * ntile / nc, j1 = (k + 1) * ntile / nc;
                c->it_sys.push_back(sidx);
                c->it_row.push_back((int32_t)I);
                c->it_j0.push_back((int32_t)j0);
                c->it_nj.push_back((int32_t)(j1 - j0));
                c->it_own.push_back(b);
                c->max_nj = std::max<int>(c->max_nj, (int)(j1 - j0));
            }
            c->rt_item0.push_back((int32_t)c->it_sys.size());
            c->rt_k.push_back((int32_t)I);
            c->rt_nt.push_back((int32_t)nt);
            c->rt_cbase.push_back(pc.sys[sidx].tile_off);
        }
    };
    for (int b = 0; b < c->n_sys; ++b) {
        if (pc.q > 0) {
            if (!count_only) c->coarse_rt0[b] = n_rt;
            add_sys(pc.n_sub + b, b);
        }
        for (int s : subs[b]) {
            rt0_of_sub[s] = n_rt;
            add_sys(s, b);
        }
        if (!count_only) c->r_itm[b + 1] = (int32_t)c->it_sys.size();
    }
    if (count_only) return count;
    c->r_item = c->r_itm;  // one Schwarz workgroup (and share of (r, z)) per item
    // tile row (and row inside it) of every fine dof, for assembling z
    c->dof_rt.assign(c->mesh.n_elem * nd, 0);
    for (int s = 0; s < pc.n_sub; ++s) {
        const int a0 = pc.sub_ptr[s], a1 = pc.sub_ptr[s + 1];
        for (int le = 0; le < a1 - a0; ++le)
            for (int i = 0; i < nd; ++i) {
                const int pos = le * nd + i;
                c->dof_rt[(int64_t)pc.sub_elems[a0 + le] * nd + i] = (rt0_of_sub[s] + pos / kTile) * kTile + pos % kTile;
            }
    }
    return count;
}

void plan_layout(pdg_ctx *c) {
    const int64_t n = c->mesh.n_elem, nd = c->mesh.nd, N = n * nd, nq = c->mesh.qp_ptr[n];
    const Precond &pc = c->pc;
    const int64_t n_dsys = (int64_t)pc.sys.size(), n_rt = (int64_t)c->rt_item0.size() - 1;
    const int64_t n_items = c->items_reserved, n_sys = c->n_sys;
    int64_t local_tiles = 0, coarse_tiles = 0;
    for (int64_t s = 0; s < n_dsys; ++s) (s < pc.n_sub ? local_tiles : coarse_tiles) += pc.sys[s].nt * (pc.sys[s].nt + 1) / 2;
    const int64_t n_chunks = (int64_t)c->grp_ptr.size() - 1;
    Layout &L = c->lay;
    L = Layout();
    Ws &w = c->w;
    w.grows = L.add(c->grp_rows.size() * 4);
    w.gslot = L.add(c->grp_slot_off.size() * 8);
    w.gcol = L.add(c->grp_col.size() * 4);
    w.gval = L.add(c->grp_val.size() * 8);
    w.mass = L.add(N * nd * 8);
    w.minv = L.add(N * nd * 8);
    w.qpptr = L.add((n + 1) * 8);
    w.qpxi = L.add(nq * c->mesh.dim * 8);
    w.qpw = L.add(nq * 8);
    w.norm = L.add(N * 8);
    w.prm = L.add(kIonicParams * 8);
    w.subptr = L.add(pc.sub_ptr.size() * 4);
    w.subel = L.add(pc.sub_elems.size() * 4);
    w.idesc = L.add(n_items * sizeof(ItemDesc));
    w.updesc = L.add(std::max<size_t>(1, c->upd_wg_c0.size()) * sizeof(UpdDesc));
    const int64_t n_pblk = (N + 255) / 256;
    w.pblk = L.add(std::max<int64_t>(1, n_pblk) * sizeof(PuBlk));
    w.dsrc = L.add(std::max<int64_t>(1, N) * sizeof(ZSrc));
    w.bcsrc = L.add(std::max<int64_t>(1, n_pblk * kPupdateKmax * std::max(pc.nq0, 1)) * sizeof(ZSrc));
    w.rtit0 = L.add((n_rt + 1) * 4);
    w.itdot = L.add(n_items * 8);  // one share per Schwarz workgroup (at most one per item)
    w.rowpart = L.add(n_items * kTile * 8);
    w.rtk = L.add(n_rt * 4);
    w.rtnt = L.add(n_rt * 4);
    w.rtcb = L.add(n_rt * 8);
    w.colp = L.add((local_tiles + coarse_tiles) * kTile * 8);
    w.tloc = L.add(local_tiles * kTile * kTile * tile_elem_bytes(pc.local_prec));
    w.tcoa = L.add(coarse_tiles * kTile * kTile * tile_elem_bytes(pc.coarse_prec));
    int64_t fb_tiles = 0;
    if (pc.local_prec == PDG_BF16)
        for (int s = 0; s < pc.n_sub; ++s)
            if (pc.fallback[s]) fb_tiles += pc.sys[s].nt * (pc.sys[s].nt + 1) / 2;
    w.tfb = L.add(fb_tiles * kTile * kTile * 4);
    w.dsc = L.add(pc.dscale.size() * 4);
    w.P = L.add(pc.P.size() * 8);
    w.ecoa = L.add(pc.elem_coarse.size() * 4);
    w.elsys = L.add(n * 4);
    w.grpptr = L.add(c->grp_ptr.size() * 4);
    w.grpel = L.add(c->grp_elems.size() * 4);
    w.upsys = L.add(c->upd_sys.size() * 4);
    w.cchunk = L.add(c->cchunk_ptr.size() * 4);
    w.csys0 = L.add((n_sys + 1) * 4);
    w.rspmv = L.add((n_sys + 1) * 4);
    w.rupd = L.add((n_sys + 1) * 4);
    w.ritem = L.add((n_sys + 1) * 4);
    w.rowner = L.add(n_sys * 4);
    w.spdesc = L.add(std::max<size_t>(1, c->spmv_wg_g0.size()) * sizeof(SpDesc));
    w.chunk0 = L.add(n_sys * 4);
    w.x = L.add(N * 8);
    w.r = L.add(N * 8);
    w.z = L.add(N * 8);
    w.p = L.add(N * 8);
    w.q = L.add(N * 8);
    w.I = L.add(N * 8);
    w.t = L.add(N * 8);
    w.b = L.add(N * 8);
    w.r0p = L.add(std::max<int64_t>(1, n_chunks * std::max(pc.nq0, 1)) * 8);
    w.sc = L.add(n_sys * sizeof(DevScalars));
    w.sca = L.add(n_sys * sizeof(DevScalars));
    w.part = L.add(std::max<int64_t>(1, (int64_t)c->spmv_wg_g0.size()) * 2 * 8);  // SpMV partials
    w.rrpart = L.add(std::max<int64_t>(1, (int64_t)c->upd_wg_c0.size()) * 8);     // update partials
    w.lanc = L.add((size_t)n_sys * c->lcap * 16);                                 // PCG coefficients
    w.cbase = L.add(std::max(pc.n_coarse, 1) * 4);   // coarse values: tile-row position of each coarse element
}

// For coarse element c of batch system b: 64 * (b's first coarse tile row) +
// (c's first dof in b's coarse system), so that value j of c sits in tile row
// (base + j) / 64 at row (base + j) % 64.
std::vector<int32_t> coarse_value_base(const pdg_ctx *c) {
    const Precond &pc = c->pc;
    std::vector<int32_t> out(std::max(pc.n_coarse, 1), 0);
    if (pc.q <= 0) return out;
    for (int b = 0; b < c->n_sys; ++b)
        for (int ce = pc.csys_ce0[b]; ce < pc.csys_ce0[b + 1]; ++ce)
            out[ce] = 64 * c->coarse_rt0[b] + (ce - pc.csys_ce0[b]) * pc.nq0;
    return out;
}

// Per block of 256 dofs of the p-update: the first coarse element its dofs
// touch and how many (elements are numbered so that these are few); more than
// kPupdateKmax marks a block that reads coarse values per dof instead.
std::vector<int32_t> pupdate_coarse_ranges(const pdg_ctx *c) {
    const int64_t nd = c->mesh.nd, N = c->mesh.n_elem * nd, nb = (N + 255) / 256;
    std::vector<int32_t> out(nb * 2, 0);
    if (c->pc.q <= 0) return out;
    for (int64_t blk = 0; blk < nb; ++blk) {
        const int64_t e0 = blk * 256 / nd, e1 = (std::min(N, blk * 256 + 256) - 1) / nd;
        int32_t lo = c->pc.elem_coarse[e0], hi = lo;
        for (int64_t e = e0; e <= e1; ++e) {
            lo = std::min(lo, c->pc.elem_coarse[e]);
            hi = std::max(hi, c->pc.elem_coarse[e]);
        }
        out[2 * blk] = lo;
        out[2 * blk + 1] = hi - lo + 1 <= kPupdateKmax ? hi - lo + 1 : kPupdateKmax + 1;
    }
    return out;
}

template <class T>
T *wptr(pdg_ctx *c, int item) { return reinterpret_cast<T *>(c->ws + c->lay.items[item].off); }

template <class T>
void upload(pdg_ctx *c, int item, const std::vector<T> &v) {
    if (v.empty()) return;
    if (v.size() * sizeof(T) > c->lay.items[item].bytes) throw Error(PDG_EINVAL, "internal: upload exceeds its slot");
    HIPCHK(hipMemcpyAsync(c->ws + c->lay.items[item].off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice,
                          c->stream));
}

void upload_items(pdg_ctx *c) {
    if ((int64_t)c->it_sys.size() > c->items_reserved) throw Error(PDG_EINVAL, "internal: item plan exceeds its slot");
    std::vector<ItemDesc> desc(c->it_sys.size());
    for (size_t k = 0; k < desc.size(); ++k) {
        ItemDesc &d = desc[k];
        const int s = c->it_sys[k];
        d = ItemDesc{};
        d.s = s;
        d.I = c->it_row[k];
        d.j0 = c->it_j0[k];
        d.nj = c->it_nj[k];
        d.owner = c->it_own[k];
        d.n = c->ds_n[s];
        d.toff = (int32_t)c->ds_toff[s];
        d.cbase = (int32_t)c->ds_cbase[s];
        d.dof0 = (int32_t)c->ds_dof0[s];
        d.rbase = (int32_t)c->ds_rbase[s];
        d.f32 = c->ds_f32[s];
    }
    upload(c, c->w.idesc, desc);
    // p-update records (they name items, so they follow the item plan)
    {
        const int64_t nd = c->mesh.nd, N = c->mesh.n_elem * nd, nb = (N + 255) / 256;
        const int nq = c->pc.q > 0 ? c->pc.nq0 : 0;
        auto src = [&](int32_t rt_lane) {
            const int rt = rt_lane >> 6;
            ZSrc z{};
            z.it0 = c->rt_item0[rt];
            z.cb = (int32_t)c->rt_cbase[rt];
            z.knt = (c->rt_k[rt] << 16) | c->rt_nt[rt];
            z.nl = ((c->rt_item0[rt + 1] - c->rt_item0[rt]) << 8) | (rt_lane & 63);
            return z;
        };
        std::vector<ZSrc> ds(N);
        for (int64_t i = 0; i < N; ++i) ds[i] = src(c->dof_rt[i]);
        const std::vector<int32_t> cr = pupdate_coarse_ranges(c), cbase = coarse_value_base(c);
        std::vector<PuBlk> bl(nb);
        std::vector<ZSrc> cs(std::max<int64_t>(1, nb * kPupdateKmax * std::max(nq, 1)));
        for (int64_t k = 0; k < nb; ++k) {
            PuBlk &b = bl[k];
            const int64_t i0 = k * 256, i1 = std::min(N, i0 + 256) - 1;
            b.s_lo = c->elem_sys[i0 / nd];
            b.s_hi = c->elem_sys[i1 / nd];
            b.c_lo = cr[2 * k];
            b.n_c = cr[2 * k + 1];
            b.it0 = c->r_item[b.s_lo];
            b.it1 = c->r_item[b.s_lo + 1];
            b.u0 = c->r_upd[b.s_lo];
            b.u1 = c->r_upd[b.s_lo + 1];
            if (nq > 0 && b.n_c <= kPupdateKmax)
                for (int t = 0; t < b.n_c * nq; ++t) {
                    const int gi = cbase[b.c_lo + t / nq] + t % nq;
                    cs[k * kPupdateKmax * nq + t] = src(gi);
                }
        }
        upload(c, c->w.dsrc, ds);
        upload(c, c->w.pblk, bl);
        upload(c, c->w.bcsrc, cs);
    }
    upload(c, c->w.rtit0, c->rt_item0);
    upload(c, c->w.ritem, c->r_item);
    HIPCHK(hipStreamSynchronize(c->stream));
}

pdg_status map_status(int st) {
    switch (st) {
    case ST_CONV:
    case ST_ZERO_RHS: return PDG_OK;
    case ST_NOCONV: return PDG_ENOCONV;
    case ST_BREAKDOWN: return PDG_EBREAKDOWN;
    case ST_NONFINITE: return PDG_ENONFINITE;
    default: return PDG_ENOCONV;
    }
}

SysRanges ranges(pdg_ctx *c) {
    SysRanges r{};
    r.n_sys = c->n_sys;
    r.spmv = wptr<int32_t>(c, c->w.rspmv);
    r.upd = wptr<int32_t>(c, c->w.rupd);
    r.item = wptr<int32_t>(c, c->w.ritem);
    r.owner = wptr<int32_t>(c, c->w.rowner);
    return r;
}

SchwarzArgs schwarz_args(pdg_ctx *c, int mode, const double *r, DevScalars *sc) {
    SchwarzArgs a{};
    a.mode = mode;
    a.nd = c->mesh.nd;
    a.n_sub = c->pc.n_sub;
    a.nq0 = c->pc.q > 0 ? c->pc.nq0 : 0;
    a.part = wptr<double>(c, c->w.rowpart);
    a.itemdot = wptr<double>(c, c->w.itdot);
    a.colpart = wptr<double>(c, c->w.colp);
    a.csys_ce0 = wptr<int32_t>(c, c->w.csys0);
    a.tiles_local = wptr<void>(c, c->w.tloc);
    a.tiles_coarse = wptr<void>(c, c->w.tcoa);
    a.sub_ptr = wptr<int32_t>(c, c->w.subptr);
    a.sub_elems = wptr<int32_t>(c, c->w.subel);
    a.cchunk_ptr = wptr<int32_t>(c, c->w.cchunk);
    a.r = r;
    a.r0part = wptr<double>(c, c->w.r0p);
    a.sc = sc;
    a.item_desc = wptr<ItemDesc>(c, c->w.idesc);
    a.n_sys_one = c->n_sys == 1 ? 1 : 0;
    if (c->pc.local_prec == PDG_BF16) {
        a.dscale = wptr<float>(c, c->w.dsc);
        a.tiles_fallback = wptr<char>(c, c->w.tfb);
    }
    return a;
}

void launch_schwarz_plain(pdg_ctx *c, const SchwarzArgs &a, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr) {
    HIPCHK(launch_schwarz(a, (int)c->it_sys.size(), store_kind(c->pc.local_prec), store_kind(c->pc.coarse_prec),
                          c->max_nj, c->stream, e0, e1));
}

// With kernel timing on, every `timing`-th Schwarz launch of a solve carries
// a pair of pool events that the dispatch itself stamps at kernel start and
// end (a timed launch costs the iteration a few microseconds more).
void launch_schwarz_timed(pdg_ctx *c, const SchwarzArgs &a) {
    const int64_t k = c->t_seq++;
    if (!c->timing || k % c->timing != 0) {
        launch_schwarz_plain(c, a);
        return;
    }
    if (c->ev_used == c->ev_pool.size()) {
        hipEvent_t x, y;
        HIPCHK(hipEventCreate(&x));
        HIPCHK(hipEventCreate(&y));
        c->ev_pool.push_back({x, y});
        c->ev_idx.push_back(0);
    }
    c->ev_idx[c->ev_used] = k;
    launch_schwarz_plain(c, a, c->ev_pool[c->ev_used].first, c->ev_pool[c->ev_used].second);
    c->ev_used++;
}

// Starts the launch count of a solve (or of a single apply).
void reset_timing_seq(pdg_ctx *c) {
    c->ev_used = 0;
    c->t_seq = 0;
}

// Collects the timings of the recorded Schwarz launches among the first `keep`
// launches of the last solve (launches queued past convergence exit at once
// and are dropped).
void harvest_timing(pdg_ctx *c, size_t keep) {
    if (c->timing)
        for (size_t k = 0; k < c->ev_used; ++k) {
            if (c->ev_idx[k] >= (int64_t)keep) continue;
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, c->ev_pool[k].first, c->ev_pool[k].second));
            c->t_ms += ms;
            c->t_launches++;
        }
    reset_timing_seq(c);
}

UpdateArgs update_args(pdg_ctx *c, int init, double *x, double *r, DevScalars *sc) {
    UpdateArgs u{};
    u.init = init;
    u.pre_pq = c->pre_pq;
    u.nd = c->mesh.nd;
    u.nq0 = c->pc.q > 0 && !c->no_precond ? c->pc.nq0 : 0;
    u.grp_ptr = wptr<int32_t>(c, c->w.grpptr);
    u.grp_elems = wptr<int32_t>(c, c->w.grpel);
    u.n_wg = (int)c->upd_wg_c0.size() - 1;
    u.x = x;
    u.r = r;
    u.p = wptr<double>(c, c->w.p);
    u.q = wptr<double>(c, c->w.q);
    u.P = u.nq0 > 0 ? wptr<double>(c, c->w.P) : nullptr;
    u.r0part = wptr<double>(c, c->w.r0p);
    u.pqpart = wptr<double>(c, c->w.part);
    u.rrpart = wptr<double>(c, c->w.rrpart);
    u.lanczos = sc == c->sc ? wptr<double2>(c, c->w.lanc) : nullptr;
    u.lcap = c->lcap;
    u.rng = ranges(c);
    u.sc = sc;
    u.wg_desc = wptr<UpdDesc>(c, c->w.updesc);
    return u;
}

// The Schwarz kernel stores its partials in FP32 when both tile stores
// accumulate in FP32 (the same rule as its template's partial type).
bool f32_partials(const pdg_ctx *c) {
    return store_kind(c->pc.local_prec) != STORE_F64 && store_kind(c->pc.coarse_prec) != STORE_F64;
}

// r: the residual the preconditioner acts on (read directly when B = I).
PupdateArgs pupdate_args(pdg_ctx *c, int mode, double *out, const double *r, DevScalars *sc) {
    PupdateArgs p{};
    p.f32part = f32_partials(c) ? 1 : 0;
    p.mode = mode;
    p.pre_rz = c->no_precond ? c->pre_rr : c->pre_rz;
    p.nd = c->mesh.nd;
    p.nq0 = c->pc.q > 0 && !c->no_precond ? c->pc.nq0 : 0;
    p.r_ident = c->no_precond ? r : nullptr;
    p.n_elem = c->mesh.n_elem;
    p.P = p.nq0 > 0 ? wptr<double>(c, c->w.P) : nullptr;
    p.elem_coarse = p.nq0 > 0 ? wptr<int32_t>(c, c->w.ecoa) : nullptr;
    p.coarse_base = wptr<int32_t>(c, c->w.cbase);
    p.elem_sys = wptr<int32_t>(c, c->w.elsys);
    p.rt_item0 = wptr<int32_t>(c, c->w.rtit0);
    p.rt_k = wptr<int32_t>(c, c->w.rtk);
    p.rt_nt = wptr<int32_t>(c, c->w.rtnt);
    p.rt_cbase = wptr<int64_t>(c, c->w.rtcb);
    p.part = wptr<double>(c, c->w.rowpart);
    p.colpart = wptr<double>(c, c->w.colp);
    p.itemdot = wptr<double>(c, c->w.itdot);
    p.rrpart = wptr<double>(c, c->w.rrpart);
    p.bbpart = wptr<double>(c, c->w.part);
    p.rng = ranges(c);
    p.blk = wptr<PuBlk>(c, c->w.pblk);
    p.dof_src = wptr<ZSrc>(c, c->w.dsrc);
    p.blk_csrc = wptr<ZSrc>(c, c->w.bcsrc);
    p.p = out;
    p.lanczos = sc == c->sc ? wptr<double2>(c, c->w.lanc) : nullptr;
    p.lcap = c->lcap;
    p.sc = sc;
    return p;
}

double *vec(pdg_ctx *c, int item) { return wptr<double>(c, item); }

// The Schwarz apply on the internal residual and the optional pre-summed
// (r, z); with B = I only the pre-summed (r, r).
void launch_precond(pdg_ctx *c, int mode, DevScalars *sc, bool timed) {
    hipStream_t s = c->stream;
    if (c->no_precond) {
        if (c->pre_rr) HIPCHK(launch_reduce(wptr<double>(c, c->w.rrpart), wptr<int32_t>(c, c->w.rupd), c->n_sys, 1, sc, s));
        return;
    }
    if (timed) launch_schwarz_timed(c, schwarz_args(c, mode, vec(c, c->w.r), sc));
    else launch_schwarz_plain(c, schwarz_args(c, mode, vec(c, c->w.r), sc));
    if (c->pre_rz) HIPCHK(launch_reduce(vec(c, c->w.itdot), wptr<int32_t>(c, c->w.ritem), c->n_sys, 1, sc, s));
}

// The four launches of one PCG iteration on the internal vectors (no
// iteration index: the kernels take it from the device scalars).
void launch_iteration(pdg_ctx *c, bool timed) {
    hipStream_t s = c->stream;
    SpmvArgs q{};
    q.mode = SPMV_PQ;
    q.x = vec(c, c->w.p);
    q.y = vec(c, c->w.q);
    q.part = vec(c, c->w.part);
    q.sc = c->sc;
    HIPCHK(launch_spmv(c->dA, q, s));
    if (c->pre_pq) HIPCHK(launch_reduce(q.part, wptr<int32_t>(c, c->w.rspmv), c->n_sys, 0, c->sc, s));
    HIPCHK(launch_update(update_args(c, 0, vec(c, c->w.x), vec(c, c->w.r), c->sc), s));
    launch_precond(c, 2, c->sc, timed);
    HIPCHK(launch_pupdate(pupdate_args(c, 2, vec(c, c->w.p), vec(c, c->w.r), c->sc), s));
}

// Captures one chunk of iterations as a graph (once per chunk length).
void ensure_graph(pdg_ctx *c) {
    if (c->gexec && c->gexec_chunk == c->chunk) return;
    drop_graph(c);
    HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    try {
        for (int k = 0; k < c->chunk; ++k) launch_iteration(c, false);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(c->stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamEndCapture(c->stream, &g));
    hipGraphExec_t e = nullptr;
    const hipError_t er = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (er != hipSuccess) throw Error(PDG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(er));
    c->gexec = e;
    c->gexec_chunk = c->chunk;
}

// PCG from x0 = x on K x = b for every system of the context: residual,
// z0 = B r0, p0 = z0.  step_mode: b is built from x (= U^k) and the ion term,
// and u_prev receives U^k.  Enqueue only.
void pcg_begin(pdg_ctx *c, double *x, const double *b, bool step_mode, double *u_prev, const double *f_ext,
               double tol, int maxit, const double *guess = nullptr) {
    if (maxit < 0) throw Error(PDG_EINVAL, "maxit < 0");
    if (!(tol >= 0.0)) throw Error(PDG_EINVAL, "tol must be >= 0");
    hipStream_t s = c->stream;
    DevScalars *sc = c->sc;
    HIPCHK(launch_status_reset(sc, c->n_sys, tol * tol, maxit, 0, s));
    SpmvArgs a{};
    a.x = x;
    a.part = vec(c, c->w.part);
    a.sc = sc;
    a.xcopy = vec(c, c->w.x);
    a.y = vec(c, c->w.r);
    if (step_mode && guess) {
        // b, then the residuals of u and of the guess; each system starts from
        // the one with the smaller residual norm
        SpmvArgs rb = a;
        rb.mode = SPMV_RHS;
        rb.y = vec(c, c->w.b);
        rb.xcopy = nullptr;
        rb.I = vec(c, c->w.I);
        rb.f = f_ext;
        rb.two_c = 2.0 * c->c;
        rb.chi = c->chi;
        HIPCHK(launch_spmv(c->dA, rb, s));
        a.mode = SPMV_RESID;
        a.b = vec(c, c->w.b);
        a.u_prev = u_prev;
        HIPCHK(launch_spmv(c->dA, a, s));
        HIPCHK(launch_sum_partials(a.part, wptr<int32_t>(c, c->w.rspmv), c->n_sys, 1, sc, s));
        SpmvArgs ag = a;
        ag.x = guess;
        ag.y = vec(c, c->w.t);
        ag.xcopy = nullptr;
        ag.u_prev = nullptr;
        HIPCHK(launch_spmv(c->dA, ag, s));
        ChooseArgs ch{};
        ch.nd = c->mesh.nd;
        ch.grp_ptr = wptr<int32_t>(c, c->w.grpptr);
        ch.grp_elems = wptr<int32_t>(c, c->w.grpel);
        ch.grp_sys = wptr<int32_t>(c, c->w.upsys);
        ch.sys_chunk0 = wptr<int32_t>(c, c->w.chunk0);
        ch.n_grp = (int)c->grp_ptr.size() - 1;
        ch.part = a.part;
        ch.g = guess;
        ch.r_g = vec(c, c->w.t);
        ch.x = vec(c, c->w.x);
        ch.r = vec(c, c->w.r);
        ch.rng = ranges(c);
        ch.sc = sc;
        HIPCHK(launch_choose(ch, s));
    } else if (step_mode) {
        a.mode = SPMV_STEP;
        a.I = vec(c, c->w.I);
        a.f = f_ext;
        a.u_prev = u_prev;
        a.two_c = 2.0 * c->c;
        a.chi = c->chi;
        // b is kept for the optional true-residual check
        SpmvArgs rb = a;
        rb.mode = SPMV_RHS;
        rb.y = vec(c, c->w.b);
        rb.xcopy = nullptr;
        if (c->true_resid) HIPCHK(launch_spmv(c->dA, rb, s));
        HIPCHK(launch_spmv(c->dA, a, s));
    } else {
        a.mode = SPMV_RESID;
        a.b = b;
        HIPCHK(launch_spmv(c->dA, a, s));
    }
    HIPCHK(launch_update(update_args(c, 1, vec(c, c->w.x), vec(c, c->w.r), sc), s));
    reset_timing_seq(c);
    launch_precond(c, 1, sc, true);
    HIPCHK(launch_pupdate(pupdate_args(c, 1, vec(c, c->w.p), vec(c, c->w.r), sc), s));
    PcgRun &R = c->run;
    R = PcgRun();
    R.x = x;
    R.b = step_mode ? vec(c, c->w.b) : b;
    R.step = step_mode;
    R.maxit = maxit;
    R.j = 1;
    R.next = c->prev_iters > 0 ? c->prev_iters : c->chunk;
    R.active = true;
}

void launch_finish_of(pdg_ctx *c) {
    HIPCHK(launch_finish(vec(c, c->w.x), c->run.x, wptr<int32_t>(c, c->w.elsys), c->mesh.nd, c->mesh.n_elem, c->sc,
                         c->stream));
}

// Launches the next chunk of iterations, the copy of the iterate to the
// caller's x and the copy of the device scalars.  The iterate is copied after
// every chunk (a few microseconds), so when the poll finds every system
// stopped the output is already complete: no further launch and wait.
void pcg_launch(pdg_ctx *c) {
    PcgRun &R = c->run;
    const int count = std::min(R.next, R.maxit - R.j + 1);
    if (count > 0) {
        if (c->use_graph && !c->timing) {
            ensure_graph(c);
            const int reps = (count + c->gexec_chunk - 1) / c->gexec_chunk;
            for (int k = 0; k < reps; ++k) HIPCHK(hipGraphLaunch(c->gexec, c->stream));
            R.j += reps * c->gexec_chunk;
        } else {
            for (int k = 0; k < count; ++k) launch_iteration(c, true);
            R.j += count;
        }
    }
    R.next = c->chunk;
    launch_finish_of(c);
    HIPCHK(hipMemcpyAsync(c->sc_host, c->sc, c->n_sys * sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream));
}

// Waits for the last pcg_launch; true when every system has stopped.
bool pcg_poll(pdg_ctx *c) {
    HIPCHK(hipStreamSynchronize(c->stream));
    PcgRun &R = c->run;
    bool all = true;
    for (int b = 0; b < c->n_sys && all; ++b) all = c->sc_host[b].done != 0;
    return all || R.j > R.maxit;
}

// Writes the iterate to the caller's x, computes the optional true residuals
// and the per-system results; returns the first non-OK system status.
pdg_status pcg_end(pdg_ctx *c, pdg_solve_info *info, int *bad_sys) {
    PcgRun &R = c->run;
    R.active = false;
    c->lanczos_ok = true;
    hipStream_t s = c->stream;
    const int n_sys = c->n_sys;
    c->last.assign(c->sc_host, c->sc_host + n_sys);
    int max_it = 0;
    for (const DevScalars &h : c->last) max_it = std::max(max_it, h.iters);
    // Schwarz launches that did work: init + iterations 1..max iters
    harvest_timing(c, (size_t)max_it + 1);
    // the caller's x was written after the last chunk, before the poll's wait
    c->last_true.assign(n_sys, -1.0);
    if (c->true_resid) {
        SpmvArgs t{};
        t.mode = SPMV_RESID;
        t.x = R.x;
        t.b = R.b;
        t.y = vec(c, c->w.t);
        t.part = vec(c, c->w.part);
        t.sc = c->sc;
        HIPCHK(launch_spmv(c->dA, t, s));
        HIPCHK(launch_sum_partials(vec(c, c->w.part), wptr<int32_t>(c, c->w.rspmv), n_sys, 1, c->sc, s));
        HIPCHK(hipMemcpyAsync(c->sc_host, c->sc, n_sys * sizeof(DevScalars), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int b = 0; b < n_sys; ++b)
            if (c->last[b].bb > 0) c->last_true[b] = std::sqrt(c->sc_host[b].tr / c->last[b].bb);
    }
    pdg_solve_info out{};
    out.guess_used = -1;
    out.local_fp32 = c->pc.n_fallback;
    for (const DevScalars &h : c->last)
        if (h.guess >= 0) out.guess_used = std::max(out.guess_used, 0) + h.guess;
    double bb = 0.0;
    out.true_relres = c->true_resid ? 0.0 : -1.0;
    pdg_status st = PDG_OK;
    if (bad_sys) *bad_sys = -1;
    for (int b = 0; b < n_sys; ++b) {
        const DevScalars &h = c->last[b];
        out.iters = std::max(out.iters, h.iters);
        bb += h.bb;
        out.relres = std::max(out.relres, h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0);
        if (c->true_resid) out.true_relres = std::max(out.true_relres, c->last_true[b]);
        const pdg_status sb = map_status(h.status == ST_RUN ? ST_NOCONV : h.status);
        if (sb != PDG_OK && st == PDG_OK) {
            st = sb;
            if (bad_sys) *bad_sys = b;
        }
    }
    out.bnorm = std::sqrt(bb);
    if (info) *info = out;
    c->prev_iters = max_it;
    return st;
}

pdg_status run_pcg(pdg_ctx *c, double *x, const double *b, bool step_mode, double *u_prev, const double *f_ext,
                   double tol, int maxit, pdg_solve_info *info, int *bad_sys, const double *guess = nullptr) {
    pcg_begin(c, x, b, step_mode, u_prev, f_ext, tol, maxit, guess);
    do pcg_launch(c);
    while (!pcg_poll(c));
    return pcg_end(c, info, bad_sys);
}

void launch_ionic_step(pdg_ctx *c, const double *u, const double *u_prev, double *ions, double *I) {
    c->lanczos_ok = false;
    HIPCHK(launch_status_reset(c->sc, c->n_sys, 0.0, 0, 1, c->stream));
    IonicArgs a{};
    a.dim = c->mesh.dim;
    a.p = c->mesh.p;
    a.nd = c->mesh.nd;
    a.n_elem = c->mesh.n_elem;
    a.qp_ptr = wptr<int64_t>(c, c->w.qpptr);
    a.qp_xi = vec(c, c->w.qpxi);
    a.qp_w = vec(c, c->w.qpw);
    a.norm = vec(c, c->w.norm);
    a.minv = vec(c, c->w.minv);
    a.u = u;
    a.u_prev = u_prev;
    a.y = ions;
    a.I = I;
    a.prm = vec(c, c->w.prm);
    a.dt = c->dt;
    a.ext_now = c->ion_endpoint ? 2.0 : 1.5;
    a.ext_prev = c->ion_endpoint ? -1.0 : -0.5;
    a.bad = &c->sc[0].ionic_bad;
    HIPCHK(launch_ionic(a, c->stream));
}

std::string pcg_message(pdg_status st, int bad_sys, int n_sys) {
    std::string m = std::string("PCG: ") + pdg_status_string(st);
    if (n_sys > 1 && bad_sys >= 0) m += " (system " + std::to_string(bad_sys) + ")";
    return m;
}

}  // namespace

extern "C" {

const char *pdg_status_string(int32_t s) {
    switch (s) {
    case PDG_OK: return "PDG_OK";
    case PDG_EINVAL: return "PDG_EINVAL";
    case PDG_ENOMEM: return "PDG_ENOMEM";
    case PDG_EHIP: return "PDG_EHIP";
    case PDG_ENOTSPD: return "PDG_ENOTSPD";
    case PDG_ENOCONV: return "PDG_ENOCONV";
    case PDG_EBREAKDOWN: return "PDG_EBREAKDOWN";
    case PDG_ENONFINITE: return "PDG_ENONFINITE";
    case PDG_ESTATE: return "PDG_ESTATE";
    }
    return "unknown status";
}

pdg_status pdg_create(pdg_ctx **out, int32_t hip_device, void *hip_stream) {
    if (!out) return PDG_EINVAL;
    *out = nullptr;
    pdg_ctx *c = nullptr;
    try {
        c = new pdg_ctx();
    } catch (...) {
        return PDG_ENOMEM;
    }
    pdg_status st = guard(c, [&] {
        c->device = hip_device;
        c->stream = reinterpret_cast<hipStream_t>(hip_stream);
        if (hip_device >= 0) {
            int n = 0;
            HIPCHK(hipGetDeviceCount(&n));
            if (hip_device >= n) throw Error(PDG_EINVAL, "no such HIP device");
            HIPCHK(hipSetDevice(hip_device));
            // device address of the static scratch of pdg_precond_apply_noalloc
            HIPCHK(static_scratch_init(hip_device));
        }
    });
    if (st != PDG_OK) {
        delete c;
        return st;
    }
    *out = c;
    return PDG_OK;
}

void pdg_destroy(pdg_ctx *c) {
    if (!c) return;
    if (c->device >= 0) {
        if (c->state >= S_BOUND) (void)hipStreamSynchronize(c->stream);
        drop_graph(c);
        for (auto &e : c->ev_pool) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
        if (c->sc_host) (void)hipHostFree(c->sc_host);
    }
    delete c;
}

const char *pdg_last_error(const pdg_ctx *c) { return c ? c->err.c_str() : "ctx is NULL"; }

pdg_status pdg_set_mesh(pdg_ctx *c, const pdg_mesh *mesh, int32_t p) {
    return guard(c, [&] {
        require(c, S_CREATED, "pdg_set_mesh");
        if (c->state >= S_MESH) throw Error(PDG_ESTATE, "pdg_set_mesh: mesh already set");
        build_mesh(c->mesh, mesh, p);
        c->n_sys = 1;
        c->sys_elem_ptr = {0, c->mesh.n_elem};
        c->elem_sys.assign(c->mesh.n_elem, 0);
        c->state = S_MESH;
    });
}

pdg_status pdg_set_systems(pdg_ctx *c, int32_t n_sys, const int64_t *elem_ptr) {
    return guard(c, [&] {
        require(c, S_MESH, "pdg_set_systems");
        if (c->state >= S_PRECOND) throw Error(PDG_ESTATE, "pdg_set_systems: call before pdg_setup_preconditioner");
        const int64_t n = c->mesh.n_elem;
        if (n_sys < 1 || !elem_ptr) throw Error(PDG_EINVAL, "n_sys < 1 or elem_ptr is NULL");
        if (elem_ptr[0] != 0 || elem_ptr[n_sys] != n) throw Error(PDG_EINVAL, "elem_ptr must run from 0 to n_elem");
        for (int b = 0; b < n_sys; ++b)
            if (elem_ptr[b + 1] <= elem_ptr[b]) throw Error(PDG_EINVAL, "empty system");
        std::vector<int32_t> es(n);
        for (int b = 0; b < n_sys; ++b)
            for (int64_t e = elem_ptr[b]; e < elem_ptr[b + 1]; ++e) es[e] = b;
        for (int64_t f = 0; f < c->mesh.n_facet; ++f) {
            const int64_t a = c->mesh.facet_elem[2 * f], b = c->mesh.facet_elem[2 * f + 1];
            if (b >= 0 && es[a] != es[b]) throw Error(PDG_EINVAL, "a facet joins two systems");
        }
        c->n_sys = n_sys;
        c->sys_elem_ptr.assign(elem_ptr, elem_ptr + n_sys + 1);
        c->elem_sys = std::move(es);
    });
}

pdg_status pdg_get_sizes(const pdg_ctx *cc, int64_t *n_elem, int32_t *nd, int64_t *n_dof, int64_t *nnzb) {
    pdg_ctx *c = const_cast<pdg_ctx *>(cc);
    return guard(c, [&] {
        require(c, S_MESH, "pdg_get_sizes");
        if (n_elem) *n_elem = c->mesh.n_elem;
        if (nd) *nd = c->mesh.nd;
        if (n_dof) *n_dof = c->mesh.n_elem * c->mesh.nd;
        if (nnzb) *nnzb = c->state >= S_ASSEMBLED ? c->K.nnzb : 0;
    });
}

pdg_status pdg_assemble(pdg_ctx *c, double chi_m, double c_m, double dt, double eta0) {
    return guard(c, [&] {
        require(c, S_MESH, "pdg_assemble");
        if (c->state >= S_PRECOND) throw Error(PDG_ESTATE, "pdg_assemble: preconditioner already set up");
        if (!(chi_m > 0) || !(c_m > 0) || !(dt > 0) || !(eta0 >= 0)) throw Error(PDG_EINVAL, "bad constants");
        c->chi = chi_m;
        c->cm = c_m;
        c->dt = dt;
        c->eta0 = eta0;
        c->c = chi_m * c_m / dt;
        assemble(c->mesh, c->c, eta0, c->M, c->K);
        const int nd = c->mesh.nd;
        c->Minv.assign(c->M.size(), 0.0);
        for (int64_t e = 0; e < c->mesh.n_elem; ++e)
            element_inverse(nd, &c->M[e * nd * nd], &c->Minv[e * nd * nd]);
        c->state = S_ASSEMBLED;
    });
}

pdg_status pdg_get_matrix(const pdg_ctx *cc, int64_t *row_ptr, int32_t *col, double *val, double *mass) {
    pdg_ctx *c = const_cast<pdg_ctx *>(cc);
    return guard(c, [&] {
        require(c, S_ASSEMBLED, "pdg_get_matrix");
        if (row_ptr) std::copy(c->K.row_ptr.begin(), c->K.row_ptr.end(), row_ptr);
        if (col) std::copy(c->K.col.begin(), c->K.col.end(), col);
        if (val) std::copy(c->K.val.begin(), c->K.val.end(), val);
        if (mass) std::copy(c->M.begin(), c->M.end(), mass);
    });
}

pdg_status pdg_set_ionic(pdg_ctx *c, const double *params, int32_t n_params) {
    return guard(c, [&] {
        require(c, S_CREATED, "pdg_set_ionic");
        if (!params || n_params != kIonicParams) throw Error(PDG_EINVAL, "ionic parameters: need 24 values");
        for (int k = 0; k < n_params; ++k)
            if (!std::isfinite(params[k])) throw Error(PDG_EINVAL, "ionic parameter not finite");
        c->ionic.assign(params, params + n_params);
        c->has_ionic = true;
        if (c->state >= S_BOUND) {
            HIPCHK(hipMemcpyAsync(vec(c, c->w.prm), c->ionic.data(), kIonicParams * 8, hipMemcpyHostToDevice,
                                  c->stream));
            HIPCHK(hipStreamSynchronize(c->stream));
        }
    });
}

pdg_status pdg_setup_preconditioner(pdg_ctx *c, const pdg_precond_desc *d) {
    return guard(c, [&] {
        require(c, S_ASSEMBLED, "pdg_setup_preconditioner");
        if (c->state >= S_PRECOND) throw Error(PDG_ESTATE, "preconditioner already set up");
        setup_precond(c->mesh, c->K, c->M, d, c->elem_sys, c->n_sys, c->pc, c->n_threads,
                      std::ldexp(1.0, -c->bf16_margin_log2));
        build_group_ell(c);
        plan_chunks(c);
        c->coarse_split = default_coarse_split(c);
        plan_items(c, c->item_kb, false);
        // room for the finest split the autotuner tries (64 KiB items, coarse items cut in four)
        const int cs = c->coarse_split;
        c->coarse_split = std::max(cs, kMaxCoarseSplit);
        c->items_reserved = std::max<int64_t>((int64_t)c->it_sys.size(), plan_items(c, std::min(c->item_kb, 64), true));
        c->coarse_split = cs;
        c->r_owner.assign(c->n_sys, 0);
        for (int b = 0; b < c->n_sys; ++b) c->r_owner[b] = (int32_t)(c->sys_elem_ptr[b] * c->mesh.nd / 256);
        choose_reductions(c);
        // algorithmic bytes of one Schwarz apply: the rows of the stored tiles
        // that hold dofs (the last tile row of a system is zero-padded), below
        // the diagonal in full and of each diagonal tile the pieces (16 bytes,
        // 8 for BF16 tiles) that reach its diagonal; plus input gathers and outputs
        int64_t tile_bytes = 0;
        for (size_t sidx = 0; sidx < c->pc.sys.size(); ++sidx) {
            const DenseSys &S = c->pc.sys[sidx];
            const int64_t es = (int64_t)tile_elem_bytes(sys_prec(c->pc, sidx));
            const int piece = es == 2 ? 8 : 16;  // bytes per lane load (BF16 tiles: 8)
            const int cw = (int)(piece / es);
            for (int64_t I = 0; I < S.nt; ++I) {
                const int rows = (int)std::min<int64_t>(kTile, S.n - I * kTile);
                int64_t diag_pieces = 0;
                for (int r = 0; r < rows; ++r) diag_pieces += r / cw + 1;
                tile_bytes += I * rows * kTile * es + diag_pieces * piece;
            }
        }
        const int64_t N = c->mesh.n_elem * c->mesh.nd;
        c->schwarz_bytes = tile_bytes + 3 * N * 8 + 3 * std::max<int64_t>(c->pc.N0, 0) * 8;
        if (c->pc.local_prec == PDG_BF16) c->schwarz_bytes += N * 4;  // the FP32 scales
        c->state = S_PRECOND;
    });
}

pdg_status pdg_get_precond_sizes(const pdg_ctx *cc, int32_t sub, int64_t *n_i, int64_t *n0, int32_t *nq0) {
    pdg_ctx *c = const_cast<pdg_ctx *>(cc);
    return guard(c, [&] {
        require(c, S_PRECOND, "pdg_get_precond_sizes");
        if (sub < 0 || sub >= c->pc.n_sub) throw Error(PDG_EINVAL, "subdomain index out of range");
        if (n_i) *n_i = c->pc.sys[sub].n;
        if (n0) *n0 = c->pc.N0;
        if (nq0) *nq0 = c->pc.q > 0 ? c->pc.nq0 : 0;
    });
}

pdg_status pdg_get_local_inverse(const pdg_ctx *cc, int32_t sub, double *out) {
    pdg_ctx *c = const_cast<pdg_ctx *>(cc);
    return guard(c, [&] {
        require(c, S_PRECOND, "pdg_get_local_inverse");
        if (!out || sub < 0 || sub >= c->pc.n_sub) throw Error(PDG_EINVAL, "bad arguments");
        std::vector<double> D;
        dense_inverse_of_system(c->pc, sub, D);
        std::copy(D.begin(), D.end(), out);
    });
}

pdg_status pdg_get_coarse(const pdg_ctx *cc, double *P, double *K0) {
    pdg_ctx *c = const_cast<pdg_ctx *>(cc);
    return guard(c, [&] {
        require(c, S_PRECOND, "pdg_get_coarse");
        const Precond &pc = c->pc;
        if (pc.q == 0) throw Error(PDG_ESTATE, "no coarse level");
        if (P) std::copy(pc.P.begin(), pc.P.end(), P);
        if (K0) {
            // block diagonal over the systems, in the caller's coarse labels
            const int nq = pc.nq0;
            const int64_t N0 = pc.N0;
            std::fill(K0, K0 + N0 * N0, 0.0);
            for (int b = 0; b < c->n_sys; ++b) {
                const int c0 = pc.csys_ce0[b];
                const int64_t n0 = (int64_t)(pc.csys_ce0[b + 1] - c0) * nq;
                for (int64_t i = 0; i < n0; ++i)
                    for (int64_t j = 0; j < n0; ++j) {
                        const int64_t gi = (int64_t)pc.coarse_orig[c0 + i / nq] * nq + i % nq;
                        const int64_t gj = (int64_t)pc.coarse_orig[c0 + j / nq] * nq + j % nq;
                        K0[gi * N0 + gj] = pc.K0blk[b][i * n0 + j];
                    }
            }
        }
    });
}

pdg_status pdg_workspace_query(pdg_ctx *c, size_t *bytes) {
    return guard(c, [&] {
        require(c, S_PRECOND, "pdg_workspace_query");
        if (!bytes) throw Error(PDG_EINVAL, "bytes is NULL");
        plan_layout(c);
        *bytes = c->lay.total;
    });
}

pdg_status pdg_bind_workspace(pdg_ctx *c, void *dev_ptr, size_t bytes) {
    return guard(c, [&] {
        require(c, S_PRECOND, "pdg_bind_workspace");
        if (c->device < 0) throw Error(PDG_ESTATE, "host-only context");
        if (c->state >= S_BOUND) throw Error(PDG_ESTATE, "workspace already bound");
        plan_layout(c);
        if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255)) throw Error(PDG_EINVAL, "workspace must be 256-byte aligned");
        if (bytes < c->lay.total) throw Error(PDG_ENOMEM, "workspace too small");
        HIPCHK(hipSetDevice(c->device));
        if (!c->sc_host) {
            void *h = nullptr;
            HIPCHK(hipHostMalloc(&h, c->n_sys * sizeof(DevScalars), hipHostMallocDefault));
            c->sc_host = reinterpret_cast<DevScalars *>(h);
            std::memset(c->sc_host, 0, c->n_sys * sizeof(DevScalars));
        }
        c->ws = reinterpret_cast<char *>(dev_ptr);
        c->ws_bytes = bytes;
        const Mesh &m = c->mesh;
        const Precond &pc = c->pc;
        const Ws &w = c->w;
        const int nd = m.nd;
        // matrix
        upload(c, w.grows, c->grp_rows);
        upload(c, w.gslot, c->grp_slot_off);
        upload(c, w.gcol, c->grp_col);
        upload(c, w.gval, c->grp_val);
        upload(c, w.mass, c->M);
        upload(c, w.minv, c->Minv);
        upload(c, w.qpptr, m.qp_ptr);
        upload(c, w.qpxi, m.qp_xi);
        upload(c, w.qpw, m.qp_w);
        upload(c, w.norm, m.norm);
        std::vector<double> prm(kIonicParams, 0.0);
        if (c->has_ionic) prm = c->ionic;
        upload(c, w.prm, prm);
        upload(c, w.subptr, pc.sub_ptr);
        upload(c, w.subel, pc.sub_elems);
        upload(c, w.rtk, c->rt_k);
        upload(c, w.rtnt, c->rt_nt);
        upload(c, w.rtcb, c->rt_cbase);
        upload(c, w.csys0, pc.q > 0 ? pc.csys_ce0 : std::vector<int32_t>(c->n_sys + 1, 0));
        upload(c, w.rspmv, c->r_spmv);
        upload(c, w.rupd, c->r_upd);
        upload(c, w.rowner, c->r_owner);
        {
            std::vector<SpDesc> sd(c->spmv_wg_g0.size() - 1);
            for (size_t k = 0; k < sd.size(); ++k) {
                SpDesc &d = sd[k];
                d.g_begin = c->spmv_wg_g0[k];
                d.g_end = c->spmv_wg_g0[k + 1];
                d.sys = c->grp_sys[d.g_begin];
                d.s0 = c->grp_slot_off[d.g_begin];
                d.s1 = c->grp_slot_off[d.g_begin + 1];
            }
            upload(c, w.spdesc, sd);
        }
        upload(c, w.chunk0, std::vector<int32_t>(c->r_chunk.begin(), c->r_chunk.end() - 1));
        upload(c, w.elsys, c->elem_sys);
        std::vector<int32_t> sys_n;
        std::vector<int64_t> sys_toff, sys_cb;
        int64_t nloc_tiles = 0;
        for (int sidx = 0; sidx < pc.n_sub; ++sidx) nloc_tiles += pc.sys[sidx].nt * (pc.sys[sidx].nt + 1) / 2;
        // BF16 local store: FP32 fallback systems get offsets in the fallback store
        const bool loc_b16 = pc.local_prec == PDG_BF16;
        std::vector<int64_t> fb_off(pc.sys.size(), -1), rbase(pc.sys.size(), 0);
        std::vector<int32_t> sys_f32(pc.sys.size(), 0);
        int64_t fb_tiles = 0;
        if (loc_b16)
            for (int sidx = 0; sidx < pc.n_sub; ++sidx) {
                rbase[sidx] = pc.rbase[sidx];
                if (!pc.fallback[sidx]) continue;
                sys_f32[sidx] = 1;
                fb_off[sidx] = fb_tiles;
                fb_tiles += pc.sys[sidx].nt * (pc.sys[sidx].nt + 1) / 2;
            }
        for (size_t sidx = 0; sidx < pc.sys.size(); ++sidx) {
            sys_n.push_back((int32_t)pc.sys[sidx].n);
            // local systems index the local store (or the fallback store),
            // coarse systems the coarse store
            sys_toff.push_back(fb_off[sidx] >= 0 ? fb_off[sidx]
                               : (int)sidx < pc.n_sub ? pc.sys[sidx].tile_off
                                                      : pc.sys[sidx].tile_off - nloc_tiles);
            sys_cb.push_back(pc.sys[sidx].tile_off);
        }
        if (loc_b16) upload(c, w.dsc, pc.dscale);
        // the item descriptors hold these in 32 bits
        const int64_t lim = (int64_t)1 << 31;
        if (pc.n_tiles >= lim || m.n_elem * nd >= lim) throw Error(PDG_EINVAL, "problem too large for 32-bit tile or dof indices");
        c->ds_n = sys_n;
        c->ds_toff = sys_toff;
        c->ds_cbase = sys_cb;
        c->ds_f32 = sys_f32;
        c->ds_rbase = rbase;
        // subdomains whose elements form one contiguous run gather r directly
        std::vector<int64_t> sys_dof0(pc.sys.size(), -1);
        for (int sidx = 0; sidx < pc.n_sub; ++sidx) {
            const int a0 = pc.sub_ptr[sidx], a1 = pc.sub_ptr[sidx + 1];
            bool contiguous = true;
            for (int k = a0 + 1; k < a1 && contiguous; ++k) contiguous = pc.sub_elems[k] == pc.sub_elems[k - 1] + 1;
            if (contiguous) sys_dof0[sidx] = (int64_t)pc.sub_elems[a0] * nd;
        }
        c->ds_dof0 = sys_dof0;
        // tiles, converted to the storage precision
        const int64_t nloc = nloc_tiles * kTile * kTile;
        const int64_t ncoa = (int64_t)pc.inv64.size() - nloc;
        std::vector<float> f32;
        std::vector<uint16_t> b16;
        auto put_tiles = [&](int item, const double *src, int64_t count, int prec) {
            if (count <= 0) return;
            if (prec == PDG_F64) {
                HIPCHK(hipMemcpyAsync(c->ws + c->lay.items[item].off, src, count * 8, hipMemcpyHostToDevice, c->stream));
            } else if (prec == PDG_F32) {
                f32.resize(count);
                for (int64_t k = 0; k < count; ++k) f32[k] = (float)src[k];
                HIPCHK(hipMemcpyAsync(c->ws + c->lay.items[item].off, f32.data(), count * 4, hipMemcpyHostToDevice, c->stream));
                HIPCHK(hipStreamSynchronize(c->stream));
            } else {
                b16.resize(count);
                for (int64_t k = 0; k < count; ++k) b16[k] = bf16_bits(src[k]);
                HIPCHK(hipMemcpyAsync(c->ws + c->lay.items[item].off, b16.data(), count * 2, hipMemcpyHostToDevice, c->stream));
                HIPCHK(hipStreamSynchronize(c->stream));
            }
        };
        if (loc_b16) {
            // scaled BF16 tiles formed at setup; FP32 tiles of the fallback systems
            if (nloc > 0)
                HIPCHK(hipMemcpyAsync(c->ws + c->lay.items[w.tloc].off, pc.tiles_b16.data(), nloc * 2,
                                      hipMemcpyHostToDevice, c->stream));
            for (int sidx = 0; sidx < pc.n_sub; ++sidx) {
                if (!pc.fallback[sidx]) continue;
                const int64_t cnt = pc.sys[sidx].nt * (pc.sys[sidx].nt + 1) / 2 * kTile * kTile;
                f32.resize(cnt);
                const double *src = pc.inv64.data() + pc.sys[sidx].tile_off * kTile * kTile;
                for (int64_t k = 0; k < cnt; ++k) f32[k] = (float)src[k];
                HIPCHK(hipMemcpyAsync(c->ws + c->lay.items[w.tfb].off + fb_off[sidx] * kTile * kTile * 4, f32.data(),
                                      cnt * 4, hipMemcpyHostToDevice, c->stream));
                HIPCHK(hipStreamSynchronize(c->stream));
            }
            HIPCHK(hipStreamSynchronize(c->stream));
        } else {
            put_tiles(w.tloc, pc.inv64.data(), nloc, pc.local_prec);
        }
        put_tiles(w.tcoa, pc.inv64.data() + nloc, ncoa, pc.coarse_prec);
        upload(c, w.P, pc.P);
        upload(c, w.ecoa, pc.elem_coarse);
        upload(c, w.cbase, coarse_value_base(c));
        upload(c, w.grpptr, c->grp_ptr);
        upload(c, w.grpel, c->grp_elems);
        {
            // update workgroup records (chunks, system, SpMV partial range, first chunk)
            std::vector<UpdDesc> ud(c->upd_wg_c0.size() - 1);
            for (size_t k = 0; k < ud.size(); ++k) {
                UpdDesc &d = ud[k];
                d.c_begin = c->upd_wg_c0[k];
                d.c_end = c->upd_wg_c0[k + 1];
                d.b = c->upd_sys[d.c_begin];
                d.g0 = c->r_spmv[d.b];
                d.g1 = c->r_spmv[d.b + 1];
                d.f_e0 = c->grp_ptr[d.c_begin];
                d.f_n = c->grp_ptr[d.c_begin + 1] - d.f_e0;
                bool run = true;
                for (int k2 = 1; k2 < d.f_n && run; ++k2) run = c->grp_elems[d.f_e0 + k2] == c->grp_elems[d.f_e0] + k2;
                d.e_first = run ? c->grp_elems[d.f_e0] : -1;
            }
            upload(c, w.updesc, ud);
        }
        upload(c, w.upsys, c->upd_sys);
        upload(c, w.cchunk, c->cchunk_ptr);
        for (int k : {w.sc, w.sca})
            HIPCHK(hipMemsetAsync(c->ws + c->lay.items[k].off, 0, c->lay.items[k].bytes, c->stream));
        for (int k : {w.x, w.r, w.z, w.p, w.q, w.I, w.t, w.b})
            HIPCHK(hipMemsetAsync(c->ws + c->lay.items[k].off, 0, c->lay.items[k].bytes, c->stream));
        upload_items(c);  // synchronises
        c->dA.nd = nd;
        c->dA.G = c->G;
        c->dA.wpg = c->spmv_wpg;
        // matrices that cannot stay in the 256 MB last-level cache stream non-temporally
        c->dA.nt = c->grp_val.size() * 8 > ((size_t)192 << 20) ? 1 : 0;
        c->dA.n_rows = m.n_elem;
        c->dA.n_groups = c->n_groups;
        c->dA.grp_rows = wptr<int32_t>(c, w.grows);
        c->dA.grp_slot_off = wptr<int64_t>(c, w.gslot);
        c->dA.grp_col = wptr<int32_t>(c, w.gcol);
        c->dA.grp_val = wptr<double>(c, w.gval);
        c->dA.mass = wptr<double>(c, w.mass);
        c->dA.n_wg = (int)c->spmv_wg_g0.size() - 1;
        c->dA.wg_desc = wptr<SpDesc>(c, w.spdesc);
        c->dA.one_sys = c->n_sys == 1 ? 1 : 0;
        c->sc = wptr<DevScalars>(c, w.sc);
        c->sc_apply = wptr<DevScalars>(c, w.sca);
        c->state = S_BOUND;
    });
}

pdg_status pdg_set_option(pdg_ctx *c, int32_t option, int64_t value) {
    return guard(c, [&] {
        require(c, S_CREATED, "pdg_set_option");
        if (c->run.active) throw Error(PDG_ESTATE, "pdg_set_option: a solve is in progress");
        switch (option) {
        case PDG_OPT_TRUE_RESIDUAL: c->true_resid = value != 0; break;
        case PDG_OPT_CHUNK:
            if (value < 1 || value > 1000) throw Error(PDG_EINVAL, "chunk must be in 1..1000");
            c->chunk = (int)value;
            break;
        case PDG_OPT_KERNEL_TIMING:
            if (value < 0 || value > (1 << 20)) throw Error(PDG_EINVAL, "kernel timing period must be 0..2^20");
            c->timing = (int)value;
            break;
        case PDG_OPT_SCHWARZ_ITEM_KB:
            if (value < 32 || value > 8192) throw Error(PDG_EINVAL, "item size must be in 32..8192 KiB");
            if (c->state >= S_PRECOND) throw Error(PDG_ESTATE, "set the item size before pdg_setup_preconditioner");
            c->item_kb = (int)value;
            break;
        case PDG_OPT_GRAPH:
            if (value != 0 && c->stream == nullptr)
                throw Error(PDG_EINVAL, "graph replay needs a non-default stream (capture is not possible on it)");
            c->use_graph = value != 0;
            break;
        case PDG_OPT_SPMV_WAVES:
            if (value != 1 && value != 2 && value != 4 && value != 8) throw Error(PDG_EINVAL, "SpMV waves must be 1, 2, 4 or 8");
            c->spmv_wpg = (int)value;
            c->dA.wpg = (int)value;
            drop_graph(c);
            break;
        case PDG_OPT_ION_EXTRAPOLATION:
            if (value != 0 && value != 1) throw Error(PDG_EINVAL, "ion extrapolation must be 0 or 1");
            c->ion_endpoint = (int)value;
            break;
        case PDG_OPT_LANCZOS_CAP:
            if (value < 1 || value > (1 << 20)) throw Error(PDG_EINVAL, "Lanczos cap must be in 1..2^20");
            if (c->state >= S_BOUND) throw Error(PDG_ESTATE, "set the Lanczos cap before pdg_bind_workspace");
            c->lcap = (int)value;
            break;
        case PDG_OPT_PRECONDITIONER:
            if (value != 0 && value != 1) throw Error(PDG_EINVAL, "preconditioner must be 0 (none) or 1 (Schwarz)");
            c->no_precond = value == 0;
            drop_graph(c);
            break;
        case PDG_OPT_BF16_MARGIN:
            if (value < 0 || value > 40) throw Error(PDG_EINVAL, "BF16 margin exponent must be in 0..40");
            if (c->state >= S_PRECOND) throw Error(PDG_ESTATE, "set the BF16 margin before pdg_setup_preconditioner");
            c->bf16_margin_log2 = (int)value;
            break;
        case PDG_OPT_PRESUM:
            if (value != 0 && value != 1) throw Error(PDG_EINVAL, "pre-summed reductions must be 0 (automatic) or 1 (always)");
            c->force_presum = (int)value;
            if (c->state >= S_PRECOND) choose_reductions(c);
            drop_graph(c);
            break;
        default: throw Error(PDG_EINVAL, "unknown option");
        }
    });
}

pdg_status pdg_kernel_timing(pdg_ctx *c, int64_t *launches, double *total_ms, double *bytes_per_launch) {
    return guard(c, [&] {
        require_gpu(c);
        HIPCHK(hipStreamSynchronize(c->stream));
        if (launches) *launches = c->t_launches;
        if (total_ms) *total_ms = c->t_ms;
        if (bytes_per_launch) *bytes_per_launch = (double)c->schwarz_bytes;
        c->t_launches = 0;
        c->t_ms = 0.0;
    });
}

pdg_status pdg_project_p0(pdg_ctx *c, const double *vals, int32_t ncomp, double *coeff) {
    return guard(c, [&] {
        require_gpu(c);
        if (!vals || !coeff || ncomp < 1) throw Error(PDG_EINVAL, "bad arguments");
        HIPCHK(launch_project_p0(vals, ncomp, c->mesh.n_elem, c->mesh.nd, vec(c, c->w.norm), coeff, c->stream));
    });
}

pdg_status pdg_spmv(pdg_ctx *c, const double *x, double *y) {
    return guard(c, [&] {
        require_gpu(c);
        if (!x || !y) throw Error(PDG_EINVAL, "NULL vector");
        SpmvArgs a{};
        a.mode = SPMV_PLAIN;
        a.x = x;
        a.y = y;
        HIPCHK(launch_spmv(c->dA, a, c->stream));
    });
}

pdg_status pdg_precond_apply(pdg_ctx *c, const double *r, double *z) {
    return guard(c, [&] {
        require_gpu(c);
        if (!r || !z) throw Error(PDG_EINVAL, "NULL vector");
        DevScalars *sc = c->sc_apply;
        HIPCHK(launch_status_reset(sc, c->n_sys, -1.0, 0, 0, c->stream));
        // restriction only (init mode: x and r untouched)
        HIPCHK(launch_update(update_args(c, 1, vec(c, c->w.t), const_cast<double *>(r), sc), c->stream));
        reset_timing_seq(c);
        if (!c->no_precond) launch_schwarz_timed(c, schwarz_args(c, 0, r, sc));
        HIPCHK(launch_pupdate(pupdate_args(c, 0, z, r, sc), c->stream));
        if (c->timing) {
            HIPCHK(hipStreamSynchronize(c->stream));
            harvest_timing(c, 1);
        }
    });
}

pdg_status pdg_precond_apply_noalloc(pdg_ctx *c, const double *r, double *z) {
    return guard(c, [&] {
        require_gpu(c);
        if (!r || !z) throw Error(PDG_EINVAL, "NULL vector");
        char *base = static_cast<char *>(static_scratch(c->device));
        if (!base) throw Error(PDG_ESTATE, "device scratch not set up");
        // the scratch buffers of the apply (device scalars, restriction shares,
        // update partials, Schwarz row and column partials), carved out of the
        // device's static array
        const Precond &pc = c->pc;
        int64_t tiles = 0;
        for (const DenseSys &S : pc.sys) tiles += S.nt * (S.nt + 1) / 2;
        const int64_t n_chunks = (int64_t)c->grp_ptr.size() - 1, n_items = (int64_t)c->it_sys.size();
        const size_t sz[6] = {c->n_sys * sizeof(DevScalars),
                              (size_t)std::max<int64_t>(1, n_chunks * std::max(pc.nq0, 1)) * 8,
                              (size_t)std::max<int64_t>(1, (int64_t)c->upd_wg_c0.size()) * 8,
                              (size_t)n_items * kTile * 8,
                              (size_t)tiles * kTile * 8,
                              (size_t)std::max<int64_t>(1, n_items) * 8};
        size_t off[6], total = 0;
        for (int k = 0; k < 6; ++k) {
            off[k] = total;
            total = align256(total + sz[k]);
        }
        if (total > kStaticScratchBytes)
            throw Error(PDG_EINVAL, "pdg_precond_apply_noalloc: this system needs " + std::to_string(total) +
                                        " bytes of scratch, above the static limit of " +
                                        std::to_string(kStaticScratchBytes) + " (use pdg_precond_apply)");
        DevScalars *sc = reinterpret_cast<DevScalars *>(base + off[0]);
        double *r0p = reinterpret_cast<double *>(base + off[1]);
        double *rrp = reinterpret_cast<double *>(base + off[2]);
        double *rowp = reinterpret_cast<double *>(base + off[3]);
        double *colp = reinterpret_cast<double *>(base + off[4]);
        double *itd = reinterpret_cast<double *>(base + off[5]);
        hipStream_t s = c->stream;
        // the scalars the kernels read are set by a kernel (no memset node
        // if the caller captures this call in a graph)
        HIPCHK(launch_status_reset(sc, c->n_sys, -1.0, 0, 0, s));
        UpdateArgs u = update_args(c, 1, vec(c, c->w.t), const_cast<double *>(r), sc);
        u.r0part = r0p;
        u.rrpart = rrp;
        HIPCHK(launch_update(u, s));
        if (!c->no_precond) {
            SchwarzArgs a = schwarz_args(c, 0, r, sc);
            a.part = rowp;
            a.colpart = colp;
            a.itemdot = itd;
            a.r0part = r0p;
            launch_schwarz_plain(c, a);
        }
        PupdateArgs pu = pupdate_args(c, 0, z, r, sc);
        pu.part = rowp;
        pu.colpart = colp;
        pu.itemdot = itd;
        pu.rrpart = rrp;
        HIPCHK(launch_pupdate(pu, s));
    });
}

pdg_status pdg_ionic(pdg_ctx *c, const double *u, const double *u_prev, double *ions, double *I) {
    return guard(c, [&] {
        require_gpu(c);
        if (!c->has_ionic) throw Error(PDG_ESTATE, "pdg_set_ionic not called");
        if (!u || !u_prev || !ions || !I) throw Error(PDG_EINVAL, "NULL vector");
        launch_ionic_step(c, u, u_prev, ions, I);
        HIPCHK(hipMemcpyAsync(c->sc_host, c->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        if (c->sc_host->ionic_bad) throw Error(PDG_ENONFINITE, "ionic: non-positive concentration before a logarithm");
    });
}

pdg_status pdg_rhs(pdg_ctx *c, const double *u, const double *I, const double *f_ext, double *b) {
    return guard(c, [&] {
        require_gpu(c);
        if (!u || !I || !b) throw Error(PDG_EINVAL, "NULL vector");
        SpmvArgs a{};
        a.mode = SPMV_RHS;
        a.x = u;
        a.I = I;
        a.f = f_ext;
        a.y = b;
        a.two_c = 2.0 * c->c;
        a.chi = c->chi;
        HIPCHK(launch_spmv(c->dA, a, c->stream));
    });
}

pdg_status pdg_solve(pdg_ctx *c, const double *rhs, double *x, double tol, int32_t maxit, pdg_solve_info *info) {
    return guard(c, [&] {
        require_gpu(c);
        if (!rhs || !x) throw Error(PDG_EINVAL, "NULL vector");
        int bad = -1;
        const pdg_status st = run_pcg(c, x, rhs, false, nullptr, nullptr, tol, maxit, info, &bad);
        if (st != PDG_OK) throw Error(st, pcg_message(st, bad, c->n_sys));
    });
}

pdg_status pdg_step(pdg_ctx *c, double *u, double *u_prev, double *ions, const double *f_ext, double tol,
                    int32_t maxit, pdg_solve_info *info) {
    return guard(c, [&] {
        require_gpu(c);
        if (!c->has_ionic) throw Error(PDG_ESTATE, "pdg_set_ionic not called");
        if (!u || !u_prev || !ions) throw Error(PDG_EINVAL, "NULL vector");
        launch_ionic_step(c, u, u_prev, ions, vec(c, c->w.I));
        int bad = -1;
        const pdg_status st = run_pcg(c, u, nullptr, true, u_prev, f_ext, tol, maxit, info, &bad);
        if (c->sc_host[0].ionic_bad) throw Error(PDG_ENONFINITE, "ionic: non-positive concentration before a logarithm");
        if (st != PDG_OK) throw Error(st, pcg_message(st, bad, c->n_sys));
    });
}

pdg_status pdg_step_guess(pdg_ctx *c, double *u, double *u_prev, double *ions, const double *f_ext,
                          const double *guess, double tol, int32_t maxit, pdg_solve_info *info) {
    return guard(c, [&] {
        require_gpu(c);
        if (!c->has_ionic) throw Error(PDG_ESTATE, "pdg_set_ionic not called");
        if (!u || !u_prev || !ions || !guess) throw Error(PDG_EINVAL, "NULL vector");
        if (guess == u || guess == u_prev) throw Error(PDG_EINVAL, "guess must not alias u or u_prev");
        launch_ionic_step(c, u, u_prev, ions, vec(c, c->w.I));
        int bad = -1;
        const pdg_status st = run_pcg(c, u, nullptr, true, u_prev, f_ext, tol, maxit, info, &bad, guess);
        if (c->sc_host[0].ionic_bad) throw Error(PDG_ENONFINITE, "ionic: non-positive concentration before a logarithm");
        if (st != PDG_OK) throw Error(st, pcg_message(st, bad, c->n_sys));
    });
}

pdg_status pdg_guess_extrapolate(pdg_ctx *c, const double *u, const double *u1, const double *u2, int32_t order,
                                 double *guess) {
    return guard(c, [&] {
        require_gpu(c);
        if (order != 1 && order != 2) throw Error(PDG_EINVAL, "order must be 1 or 2");
        if (!u || !u1 || !guess || (order == 2 && !u2)) throw Error(PDG_EINVAL, "NULL vector");
        HIPCHK(launch_extrapolate(u, u1, order == 2 ? u2 : u1, order, c->mesh.n_elem * c->mesh.nd, guess, c->stream));
    });
}

pdg_status pdg_step_batch(pdg_ctx *const *ctxs, int32_t n_ctx, double *const *u, double *const *u_prev,
                          double *const *ions, const double *const *f_ext, double tol, int32_t maxit,
                          pdg_solve_info *info) {
    if (!ctxs || n_ctx < 1 || !ctxs[0]) return PDG_EINVAL;
    pdg_ctx *c0 = ctxs[0];
    pdg_status result = PDG_OK;
    const pdg_status g = guard(c0, [&] {
        if (!u || !u_prev || !ions) throw Error(PDG_EINVAL, "NULL pointer array");
        for (int k = 0; k < n_ctx; ++k) {
            pdg_ctx *c = ctxs[k];
            require_gpu(c);
            if (!c->has_ionic) throw Error(PDG_ESTATE, "pdg_set_ionic not called");
            if (!u[k] || !u_prev[k] || !ions[k]) throw Error(PDG_EINVAL, "NULL vector");
            for (int l = 0; l < k; ++l)
                if (ctxs[l] == c) throw Error(PDG_EINVAL, "a context appears twice");
        }
        std::vector<char> live(n_ctx, 1);
        for (int k = 0; k < n_ctx; ++k) {
            pdg_ctx *c = ctxs[k];
            launch_ionic_step(c, u[k], u_prev[k], ions[k], vec(c, c->w.I));
            pcg_begin(c, u[k], nullptr, true, u_prev[k], f_ext ? f_ext[k] : nullptr, tol, maxit);
        }
        // chunks of all live contexts are queued before any poll waits
        for (int n_live = n_ctx; n_live > 0;) {
            for (int k = 0; k < n_ctx; ++k)
                if (live[k]) pcg_launch(ctxs[k]);
            for (int k = 0; k < n_ctx; ++k)
                if (live[k] && pcg_poll(ctxs[k])) {
                    live[k] = 0;
                    --n_live;
                }
        }
        std::string msg;
        for (int k = 0; k < n_ctx; ++k) {
            pdg_ctx *c = ctxs[k];
            int bad = -1;
            pdg_status st = pcg_end(c, info ? &info[k] : nullptr, &bad);
            if (c->sc_host[0].ionic_bad && st == PDG_OK) st = PDG_ENONFINITE;
            if (st != PDG_OK && result == PDG_OK) {
                result = st;
                msg = "context " + std::to_string(k) + ": " +
                      (c->sc_host[0].ionic_bad ? std::string("ionic: non-positive concentration before a logarithm")
                                               : pcg_message(st, bad, c->n_sys));
            }
        }
        if (result != PDG_OK) throw Error(result, msg);
    });
    return g;
}

pdg_status pdg_get_system_info(const pdg_ctx *cc, int32_t sys, pdg_solve_info *info, int32_t *status) {
    pdg_ctx *c = const_cast<pdg_ctx *>(cc);
    return guard(c, [&] {
        require_gpu(c);
        if (sys < 0 || sys >= c->n_sys) throw Error(PDG_EINVAL, "system index out of range");
        if (c->last.empty()) throw Error(PDG_ESTATE, "no solve yet");
        const DevScalars &h = c->last[sys];
        if (info) {
            info->guess_used = h.guess;
            info->iters = h.iters;
            info->bnorm = std::sqrt(h.bb);
            info->relres = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
            info->true_relres = c->last_true[sys];
            info->local_fp32 = 0;
            for (int s = 0; s < c->pc.n_sub && !c->pc.fallback.empty(); ++s)
                if (c->pc.sub_bsys[s] == sys) info->local_fp32 += c->pc.fallback[s];
        }
        if (status) *status = map_status(h.status == ST_RUN ? ST_NOCONV : h.status);
    });
}

pdg_status pdg_lanczos(pdg_ctx *c, int32_t sys, double *kappa, double *lambda_min, double *lambda_max) {
    return guard(c, [&] {
        require_gpu(c);
        if (sys < 0 || sys >= c->n_sys) throw Error(PDG_EINVAL, "system index out of range");
        if (!c->lanczos_ok) throw Error(PDG_ESTATE, "pdg_lanczos: call right after pdg_solve / pdg_step");
        if (c->last[sys].iters > c->lcap)
            throw Error(PDG_EINVAL, "more iterations than coefficients kept (raise PDG_OPT_LANCZOS_CAP)");
        HIPCHK(launch_lanczos(wptr<double2>(c, c->w.lanc), c->lcap, c->n_sys, c->sc, c->stream));
        HIPCHK(hipMemcpyAsync(c->sc_host, c->sc, c->n_sys * sizeof(DevScalars), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        const DevScalars &h = c->sc_host[sys];
        if (lambda_min) *lambda_min = h.lmin;
        if (lambda_max) *lambda_max = h.lmax;
        if (kappa) *kappa = h.lmax / h.lmin;
    });
}

pdg_status pdg_get_pcg_coefficients(pdg_ctx *c, int32_t sys, double *alpha, double *beta, int32_t n) {
    return guard(c, [&] {
        require_gpu(c);
        if (sys < 0 || sys >= c->n_sys || n < 0) throw Error(PDG_EINVAL, "bad arguments");
        if (!c->lanczos_ok) throw Error(PDG_ESTATE, "pdg_get_pcg_coefficients: call right after pdg_solve / pdg_step");
        const int m = std::min({n, c->last[sys].iters, c->lcap});
        std::vector<double> h(2 * (size_t)std::max(m, 1));
        if (m > 0)
            HIPCHK(hipMemcpyAsync(h.data(), wptr<double2>(c, c->w.lanc) + (size_t)sys * c->lcap, m * 16,
                                  hipMemcpyDeviceToHost, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        for (int j = 0; j < m; ++j) {
            if (alpha) alpha[j] = h[2 * j];
            if (beta) beta[j] = h[2 * j + 1];
        }
    });
}

pdg_status pdg_autotune(pdg_ctx *c, int32_t reps, pdg_tune_result *out) {
    return guard(c, [&] {
        require_gpu(c);
        if (reps < 1 || reps > 1000) throw Error(PDG_EINVAL, "reps must be in 1..1000");
        if (c->run.active) throw Error(PDG_ESTATE, "pdg_autotune: a solve is in progress");
        hipStream_t s = c->stream;
        HIPCHK(hipStreamSynchronize(s));
        drop_graph(c);
        // synthetic system: b with entries from a fixed linear congruential
        // sequence in [-1, 1), x0 = 0; tol = 0, so no system stops while timed
        const int64_t N = c->mesh.n_elem * c->mesh.nd;
        {
            std::vector<double> hb(N), hx(N, 0.0);
            uint64_t st = 0x9e3779b97f4a7c15ull;
            for (int64_t i = 0; i < N; ++i) {
                st = st * 6364136223846793005ull + 1442695040888963407ull;
                hb[i] = (double)(st >> 11) * 0x1.0p-52 - 1.0;
            }
            HIPCHK(hipMemcpyAsync(vec(c, c->w.b), hb.data(), N * 8, hipMemcpyHostToDevice, s));
            HIPCHK(hipMemcpyAsync(vec(c, c->w.z), hx.data(), N * 8, hipMemcpyHostToDevice, s));
            HIPCHK(hipStreamSynchronize(s));
        }
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        // mean time of one PCG iteration (the four launches back to back, no
        // host synchronisation between them) after two untimed iterations;
        // negative if a system stopped during the measurement
        auto iter_ms = [&]() -> double {
            pcg_begin(c, vec(c, c->w.z), vec(c, c->w.b), false, nullptr, nullptr, 0.0, 1 << 30);
            c->run.active = false;
            for (int k = 0; k < 2; ++k) launch_iteration(c, false);
            HIPCHK(hipEventRecord(e0, s));
            for (int k = 0; k < reps; ++k) launch_iteration(c, false);
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipMemcpyAsync(c->sc_host, c->sc, c->n_sys * sizeof(DevScalars), hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            for (int b = 0; b < c->n_sys; ++b)
                if (c->sc_host[b].done) return -1.0;
            return (double)ms / reps;
        };
        auto apply_plan = [&](int kb, int cs) {
            c->coarse_split = cs;
            plan_items(c, kb, false);
            upload_items(c);
            c->item_kb = kb;
            choose_reductions(c);
        };
        auto plan_fits = [&](int kb, int cs) {
            const int old = c->coarse_split;
            c->coarse_split = cs;
            const int64_t n = plan_items(c, kb, true);
            c->coarse_split = old;
            return n <= c->items_reserved;
        };
        pdg_tune_result res{};
        const int timing = c->timing;
        c->timing = 0;
        try {
            int kb = c->item_kb, cs = c->coarse_split, wv = c->spmv_wpg;
            const double t_start = std::min(iter_ms(), iter_ms());
            if (t_start < 0) throw Error(PDG_EBREAKDOWN, "pdg_autotune: the synthetic solve stopped while timed");
            double t_final = t_start;
            int timed = 2;
            // one knob at a time; each candidate is timed twice (in two sweeps)
            // and keeps its faster time; the current value is replaced only by
            // a candidate more than 1 % faster
            auto sweep = [&](const std::vector<int> &vals, int cur, auto &&set) {
                std::vector<double> t(vals.size(), 1e300);
                for (int pass = 0; pass < 2; ++pass)
                    for (size_t i = 0; i < vals.size(); ++i) {
                        if (!set(vals[i])) continue;
                        const double ms = iter_ms();
                        ++timed;
                        if (ms > 0) t[i] = std::min(t[i], ms);
                    }
                double t_cur = 1e300;
                for (size_t i = 0; i < vals.size(); ++i)
                    if (vals[i] == cur) t_cur = t[i];
                int pick = cur;
                double t_pick = t_cur;
                for (size_t i = 0; i < vals.size(); ++i)
                    if (t[i] < 0.99 * t_pick) {
                        pick = vals[i];
                        t_pick = t[i];
                    }
                set(pick);
                if (t_pick < 1e300) t_final = t_pick;
                return pick;
            };
            if (!c->no_precond) {
                kb = sweep({64, 96, 128, 192, 256, 384}, kb, [&](int v) {
                    if (!plan_fits(v, cs)) return false;
                    apply_plan(v, cs);
                    return true;
                });
                if (c->pc.q > 0)
                    cs = sweep({1, 2, 3, 4}, cs, [&](int v) {
                        if (!plan_fits(kb, v)) return false;
                        apply_plan(kb, v);
                        return true;
                    });
            }
            wv = sweep({1, 2, 4, 8}, wv, [&](int v) {
                c->spmv_wpg = v;
                c->dA.wpg = v;
                return true;
            });
            res.item_kb = kb;
            res.coarse_split = cs;
            res.spmv_waves = wv;
            res.candidates = timed;
            res.iter_us_before = t_start * 1e3;
            res.iter_us = t_final * 1e3;
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            c->prev_iters = 0;
            c->timing = timing;
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        c->prev_iters = 0;
        c->timing = timing;
        if (out) *out = res;
    });
}

}  // extern "C"
