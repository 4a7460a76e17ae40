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

uint16_t to_bf16(double v) {
    float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf/nan
    u += 0x7fffu + ((u >> 16) & 1u);                                     // round to nearest even
    return (uint16_t)(u >> 16);
}

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

}  // namespace

struct pdg_ctx {
    int device = -1;
    hipStream_t stream = nullptr;
    int state = S_CREATED;
    std::string err;
    int n_threads = 0;
    // options
    int true_resid = 0, chunk = 4, timing = 0, item_kb = 256;
    int prev_iters = 0;
    // host data
    Mesh mesh;
    Bsr K;
    std::vector<double> M, Minv;
    double chi = 1, cm = 1, dt = 1, eta0 = 10, c = 1;
    std::vector<double> ionic;
    bool has_ionic = false;
    Precond pc;
    std::vector<int32_t> grp_ptr, grp_elems;  // update chunks (element runs inside one coarse element)
    std::vector<int32_t> cchunk_ptr;          // [n_coarse+1] chunks of each coarse element
    // Schwarz work items
    std::vector<int32_t> it_sys, it_row, it_j0, it_nj, it_rt, rt_item0;
    int max_nj = 1;
    // group-ELL matrix (host staging)
    int G = 1;
    int64_t n_groups = 0, n_slots = 0;
    std::vector<int32_t> grp_rows, grp_col;
    std::vector<int64_t> grp_slot_off;
    std::vector<double> grp_val;
    // device
    Layout lay;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    DevMatrix dA{};
    DevScalars *sc = nullptr, *sc_apply = nullptr, *sc_host = nullptr;
    int64_t *d_qp_ptr = nullptr;
    double *d_qp_xi = nullptr, *d_qp_w = nullptr, *d_norm = nullptr, *d_minv = nullptr, *d_prm = nullptr;
    int32_t *d_sub_ptr = nullptr, *d_sub_elems = nullptr;
    int32_t *d_sys_n = nullptr, *d_sys_nt = nullptr, *d_elem_coarse = nullptr;
    int32_t *d_grp_ptr = nullptr, *d_grp_elems = nullptr, *d_cchunk_ptr = nullptr;
    int32_t *d_it_sys = nullptr, *d_it_row = nullptr, *d_it_j0 = nullptr, *d_it_nj = nullptr, *d_it_rt = nullptr,
            *d_rt_item0 = nullptr;
    int32_t *d_dof_rt = nullptr;
    double *d_part = nullptr, *d_r0part = nullptr, *d_itemdot = nullptr, *d_spart = nullptr, *d_rrpart = nullptr;
    std::vector<int32_t> dof_rt;
    int coarse_rt0 = -1;
    int64_t *d_sys_toff = nullptr, *d_sys_dof0 = nullptr, *d_sys_cbase = nullptr, *d_rt_cbase = nullptr;
    int32_t *d_rt_k = nullptr, *d_rt_nt = nullptr;
    double *d_colpart = nullptr;
    std::vector<int32_t> rt_k, rt_nt;
    std::vector<int64_t> rt_cbase;
    void *d_tiles_local = nullptr, *d_tiles_coarse = nullptr;
    double *d_P = nullptr;
    double *v_r = nullptr, *v_z = nullptr, *v_p = nullptr, *v_q = nullptr, *v_I = nullptr, *v_t = nullptr,
           *v_b = nullptr, *v_z0 = nullptr;
    int max_sys_n = 0;
    int64_t schwarz_bytes = 0;
    // kernel timing
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
    size_t ev_used = 0;
    int64_t t_launches = 0;
    double t_ms = 0.0;
};

namespace {

void require(pdg_ctx *c, int st, const char *what) {
    if (!c) throw Error(PDG_EINVAL, "ctx is NULL");
    if (c->state < st) throw Error(PDG_ESTATE, std::string(what) + ": call out of order");
}
void require_gpu(pdg_ctx *c) {
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

void build_group_ell(pdg_ctx *c) {
    const int nd = c->mesh.nd;
    const int64_t n = c->K.n_rows;
    c->G = nd <= 64 ? 64 / nd : 1;
    const int G = c->G;
    std::vector<int32_t> perm(n);
    std::iota(perm.begin(), perm.end(), 0);
    auto nb = [&](int32_t r) { return c->K.row_ptr[r + 1] - c->K.row_ptr[r]; };
    std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return nb(a) > nb(b); });
    c->n_groups = (n + G - 1) / G;
    c->grp_rows.assign(c->n_groups * G, -1);
    c->grp_slot_off.assign(c->n_groups + 1, 0);
    for (int64_t g = 0; g < c->n_groups; ++g) {
        int64_t smax = 0;
        for (int r = 0; r < G; ++r) {
            int64_t k = g * G + r;
            if (k < n) {
                c->grp_rows[k] = perm[k];
                smax = std::max<int64_t>(smax, nb(perm[k]));
            }
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
                if (blk)
                    for (int j = 0; j < nd; ++j)
                        for (int i = 0; i < nd; ++i)
                            c->grp_val[(s0 + s) * G * nd * nd + (j * G + r) * nd + i] = blk[i * nd + j];
            }
        }
    }
}

size_t tile_elem_bytes(int prec) { return prec == PDG_F64 ? 8 : (prec == PDG_F32 ? 4 : 2); }

enum WsItem {
    W_GROWS, W_GSLOT, W_GCOL, W_GVAL, W_MASS, W_MINV, W_QPPTR, W_QPXI, W_QPW, W_NORM, W_PRM,
    W_SUBPTR, W_SUBEL, W_ITSYS, W_ITROW, W_ITJ0, W_ITNJ, W_ITRT, W_RTIT0, W_DOFRT, W_ITDOT, W_SPART,
    W_SYSN, W_SYSNT, W_SYSTOFF, W_SYSDOF0, W_SYSCB, W_RTK, W_RTNT, W_RTCB, W_COLP, W_TLOC, W_TCOA, W_P, W_ECOA, W_GRPPTR, W_GRPEL, W_CCHUNK,
    W_R, W_Z, W_PV, W_Q, W_I, W_T, W_B, W_R0P, W_Z0, W_SC, W_SCA, W_PART, W_RRPART, W_COUNT
};

void plan_layout(pdg_ctx *c) {
    const int64_t n = c->mesh.n_elem, nd = c->mesh.nd, N = n * nd, nq = c->mesh.qp_ptr[n];
    const Precond &pc = c->pc;
    const int64_t n_sys = (int64_t)pc.sys.size();
    int64_t local_tiles = 0, coarse_tiles = 0;
    for (int s = 0; s < pc.n_sub; ++s) local_tiles += pc.sys[s].nt * (pc.sys[s].nt + 1) / 2;
    if (pc.q > 0) coarse_tiles = pc.sys[pc.n_sub].nt * (pc.sys[pc.n_sub].nt + 1) / 2;
    const int64_t N0 = std::max<int64_t>(1, pc.N0);
    int64_t max_grid = std::max<int64_t>({(int64_t)spmv_blocks(DevMatrix{(int)nd, c->G, n, c->n_groups}),
                                          (int64_t)c->grp_ptr.size(), 1});
    const int64_t n_items = (int64_t)c->it_sys.size(), n_rt = (int64_t)c->rt_item0.size() - 1;
    Layout &L = c->lay;
    L = Layout();
    L.add(c->grp_rows.size() * 4);
    L.add(c->grp_slot_off.size() * 8);
    L.add(c->grp_col.size() * 4);
    L.add(c->grp_val.size() * 8);
    L.add(N * nd * 8);
    L.add(N * nd * 8);
    L.add((n + 1) * 8);
    L.add(nq * c->mesh.dim * 8);
    L.add(nq * 8);
    L.add(N * 8);
    L.add(kIonicParams * 8);
    L.add(pc.sub_ptr.size() * 4);
    L.add(pc.sub_elems.size() * 4);
    for (int k = 0; k < 5; ++k) L.add(n_items * 4);   // item sys/row/j0/nj/rt
    L.add((n_rt + 1) * 4);
    L.add(N * 4);
    L.add(n_items * 8);
    L.add(n_items * kTile * 8);
    L.add(n_sys * 4);
    L.add(n_sys * 4);
    L.add(n_sys * 8);
    L.add(n_sys * 8);
    L.add(n_sys * 8);
    L.add(n_rt * 4);
    L.add(n_rt * 4);
    L.add(n_rt * 8);
    L.add((local_tiles + coarse_tiles) * kTile * 8);
    L.add(local_tiles * kTile * kTile * tile_elem_bytes(pc.local_prec));
    L.add(coarse_tiles * kTile * kTile * tile_elem_bytes(pc.coarse_prec));
    L.add(pc.P.size() * 8);
    L.add(pc.elem_coarse.size() * 4);
    L.add(c->grp_ptr.size() * 4);
    L.add(c->grp_elems.size() * 4);
    L.add(c->cchunk_ptr.size() * 4);
    for (int k = 0; k < 7; ++k) L.add(N * 8);  // r z p q I t b
    L.add(std::max<int64_t>(1, (int64_t)c->grp_ptr.size() * std::max(pc.nq0, 1)) * 8);  // r0 shares per chunk
    L.add(N0 * 8);
    L.add(sizeof(DevScalars));
    L.add(sizeof(DevScalars));
    L.add(std::max<int64_t>(1, c->n_groups) * 2 * 8);   // SpMV partials
    L.add(std::max<int64_t>(1, (int64_t)c->grp_ptr.size()) * 8);  // update partials
}

template <class T>
T *wptr(pdg_ctx *c, int item) { return reinterpret_cast<T *>(c->ws + c->lay.items[item].off); }

template <class T>
void upload(pdg_ctx *c, int item, const std::vector<T> &v) {
    if (v.empty()) return;
    HIPCHK(hipMemcpyAsync(c->ws + c->lay.items[item].off, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice,
                          c->stream));
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

int store_kind(int prec) { return prec == PDG_F64 ? STORE_F64 : (prec == PDG_F32 ? STORE_F32 : STORE_BF16); }

SchwarzArgs schwarz_args(pdg_ctx *c, int mode, const double *r, DevScalars *sc) {
    SchwarzArgs a{};
    a.mode = mode;
    a.nd = c->mesh.nd;
    a.n_sub = c->pc.n_sub;
    a.nq0 = c->pc.q > 0 ? c->pc.nq0 : 0;
    a.item_sys = c->d_it_sys;
    a.item_row = c->d_it_row;
    a.item_j0 = c->d_it_j0;
    a.item_nj = c->d_it_nj;
    a.part = c->d_part;
    a.itemdot = c->d_itemdot;
    a.sys_n = c->d_sys_n;
    a.sys_nt = c->d_sys_nt;
    a.sys_toff = c->d_sys_toff;
    a.sys_dof0 = c->d_sys_dof0;
    a.sys_cbase = c->d_sys_cbase;
    a.colpart = c->d_colpart;
    a.tiles_local = c->d_tiles_local;
    a.tiles_coarse = c->d_tiles_coarse;
    a.sub_ptr = c->d_sub_ptr;
    a.sub_elems = c->d_sub_elems;
    a.cchunk_ptr = c->d_cchunk_ptr;
    a.r = r;
    a.r0part = c->d_r0part;
    a.sc = sc;
    return a;
}

void launch_schwarz_timed(pdg_ctx *c, const SchwarzArgs &a) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->timing) {
        if (c->ev_used == c->ev_pool.size()) {
            hipEvent_t x, y;
            HIPCHK(hipEventCreate(&x));
            HIPCHK(hipEventCreate(&y));
            c->ev_pool.push_back({x, y});
        }
        e0 = c->ev_pool[c->ev_used].first;
        e1 = c->ev_pool[c->ev_used].second;
        HIPCHK(hipEventRecord(e0, c->stream));
    }
    HIPCHK(launch_schwarz(a, (int)c->it_sys.size(), store_kind(c->pc.local_prec),
                          store_kind(c->pc.coarse_prec), c->max_nj, c->stream));
    if (c->timing) {
        HIPCHK(hipEventRecord(e1, c->stream));
        c->ev_used++;
    }
}

// Collects the timings of the first `keep` recorded Schwarz launches of the
// last solve (launches queued past convergence exit at once and are dropped).
void harvest_timing(pdg_ctx *c, size_t keep) {
    if (!c->timing) return;
    for (size_t k = 0; k < c->ev_used && k < keep; ++k) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, c->ev_pool[k].first, c->ev_pool[k].second));
        c->t_ms += ms;
        c->t_launches++;
    }
    c->ev_used = 0;
}

UpdateArgs update_args(pdg_ctx *c, int init, int iter, double *x, double *r, DevScalars *sc) {
    UpdateArgs u{};
    u.init = init;
    u.iter = iter;
    u.nd = c->mesh.nd;
    u.nq0 = c->pc.q > 0 ? c->pc.nq0 : 0;
    u.grp_ptr = c->d_grp_ptr;
    u.grp_elems = c->d_grp_elems;
    u.n_grp = (int)c->grp_ptr.size() - 1;
    u.x = x;
    u.r = r;
    u.p = c->v_p;
    u.q = c->v_q;
    u.P = c->d_P;
    u.r0part = c->d_r0part;
    u.pqpart = c->d_spart;
    u.n_pq = (int)c->n_groups;
    u.rrpart = c->d_rrpart;
    u.sc = sc;
    return u;
}

PupdateArgs pupdate_args(pdg_ctx *c, int mode, int iter, double *out, DevScalars *sc) {
    PupdateArgs p{};
    p.mode = mode;
    p.iter = iter;
    p.nd = c->mesh.nd;
    p.nq0 = c->pc.q > 0 ? c->pc.nq0 : 0;
    p.n_elem = c->mesh.n_elem;
    p.P = c->d_P;
    p.elem_coarse = c->d_elem_coarse;
    p.dof_rt = c->d_dof_rt;
    p.rt_item0 = c->d_rt_item0;
    p.rt_k = c->d_rt_k;
    p.rt_nt = c->d_rt_nt;
    p.rt_cbase = c->d_rt_cbase;
    p.colpart = c->d_colpart;
    p.coarse_rt0 = c->coarse_rt0;
    p.part = c->d_part;
    p.itemdot = c->d_itemdot;
    p.n_items = (int)c->it_sys.size();
    p.rrpart = c->d_rrpart;
    p.n_rr = (int)c->grp_ptr.size() - 1;
    p.bbpart = c->d_spart;
    p.n_bb = (int)c->n_groups;
    p.p = out;
    p.sc = sc;
    return p;
}

// PCG from x0 = x on K x = b.  step_mode: b is built from x (= U^k) and the
// ion term, and u_prev receives U^k.
pdg_status run_pcg(pdg_ctx *c, double *x, const double *b, bool step_mode, double *u_prev, const double *f_ext,
                   double tol, int maxit, pdg_solve_info *info) {
    if (maxit < 0) throw Error(PDG_EINVAL, "maxit < 0");
    if (!(tol >= 0.0)) throw Error(PDG_EINVAL, "tol must be >= 0");
    hipStream_t s = c->stream;
    DevScalars *sc = c->sc;
    HIPCHK(launch_status_reset(sc, tol * tol, maxit, 0, s));
    SpmvArgs a{};
    a.x = x;
    a.part = c->d_spart;
    a.sc = sc;
    if (step_mode) {
        a.mode = SPMV_STEP;
        a.y = c->v_r;
        a.I = c->v_I;
        a.f = f_ext;
        a.u_prev = u_prev;
        a.two_c = 2.0 * c->c;
        a.chi = c->chi;
        // b is kept for the optional true-residual check
        SpmvArgs rb = a;
        rb.mode = SPMV_RHS;
        rb.y = c->v_b;
        if (c->true_resid) HIPCHK(launch_spmv(c->dA, rb, s));
    } else {
        a.mode = SPMV_RESID;
        a.b = b;
        a.y = c->v_r;
    }
    HIPCHK(launch_spmv(c->dA, a, s));
    HIPCHK(launch_update(update_args(c, 1, 0, x, c->v_r, sc), s));
    c->ev_used = 0;
    launch_schwarz_timed(c, schwarz_args(c, 1, c->v_r, sc));
    HIPCHK(launch_pupdate(pupdate_args(c, 1, 0, c->v_p, sc), s));
    int j = 1;
    int chunk = c->prev_iters > 0 ? std::max(1, c->prev_iters) : c->chunk;
    bool done = false;
    while (!done) {
        for (int k = 0; k < chunk && j <= maxit; ++k, ++j) {
            SpmvArgs q{};
            q.mode = SPMV_PQ;
            q.x = c->v_p;
            q.y = c->v_q;
            q.part = c->d_spart;
            q.sc = sc;
            HIPCHK(launch_spmv(c->dA, q, s));
            HIPCHK(launch_update(update_args(c, 0, j, x, c->v_r, sc), s));
            launch_schwarz_timed(c, schwarz_args(c, 2, c->v_r, sc));
            HIPCHK(launch_pupdate(pupdate_args(c, 2, j, c->v_p, sc), s));
        }
        HIPCHK(hipMemcpyAsync(c->sc_host, sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        done = c->sc_host->done || j > maxit;
        chunk = c->chunk;
    }
    const DevScalars h = *c->sc_host;
    // Schwarz launches that did work: init + iterations 1..iters (convergence is
    // detected after the Schwarz kernel of the converged iteration)
    harvest_timing(c, (size_t)h.iters + 1);
    if (h.status == ST_ZERO_RHS) HIPCHK(launch_zero(x, c->mesh.n_elem * c->mesh.nd, s));
    pdg_solve_info out{};
    out.iters = h.iters;
    out.bnorm = std::sqrt(h.bb);
    out.relres = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
    out.true_relres = -1.0;
    if (c->true_resid && h.bb > 0) {
        SpmvArgs t{};
        t.mode = SPMV_RESID;
        t.x = x;
        t.b = step_mode ? c->v_b : b;
        t.y = c->v_t;
        t.part = c->d_spart;
        t.sc = sc;
        HIPCHK(launch_spmv(c->dA, t, s));
        HIPCHK(launch_sum_partials(c->d_spart, (int)c->n_groups, 1, &sc->tr, s));
        HIPCHK(hipMemcpyAsync(c->sc_host, sc, sizeof(DevScalars), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        out.true_relres = std::sqrt(c->sc_host->tr / h.bb);
    }
    if (info) *info = out;
    c->prev_iters = h.iters;
    int st = h.status;
    if (st == ST_RUN) st = ST_NOCONV;
    return map_status(st);
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
            void *h = nullptr;
            HIPCHK(hipHostMalloc(&h, sizeof(DevScalars), hipHostMallocDefault));
            c->sc_host = reinterpret_cast<DevScalars *>(h);
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
        if (c->stream || c->state >= S_BOUND) (void)hipStreamSynchronize(c->stream);
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
        build_mesh(c->mesh, mesh, p);
        c->state = S_MESH;
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
        build_group_ell(c);
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
        if (c->state >= S_BOUND)
            HIPCHK(hipMemcpyAsync(c->d_prm, c->ionic.data(), kIonicParams * 8, hipMemcpyHostToDevice, c->stream));
        if (c->state >= S_BOUND) HIPCHK(hipStreamSynchronize(c->stream));
    });
}

pdg_status pdg_setup_preconditioner(pdg_ctx *c, const pdg_precond_desc *d) {
    return guard(c, [&] {
        require(c, S_ASSEMBLED, "pdg_setup_preconditioner");
        if (c->state >= S_BOUND) throw Error(PDG_ESTATE, "preconditioner already bound to a workspace");
        if (d && d->coarse_q > 1) throw Error(PDG_EINVAL, "coarse_q must be 0 or 1");
        setup_precond(c->mesh, c->K, c->M, d, c->pc, c->n_threads);
        if (c->pc.q > 0 && c->pc.N0 > kMaxLocalDofs) throw Error(PDG_EINVAL, "coarse system exceeds 6144 dofs");
        // update chunks: runs of at most 32 elements inside one coarse element
        // (or over the element order without a coarse level)
        constexpr int kChunk = 32;
        c->grp_ptr.assign(1, 0);
        c->grp_elems.clear();
        c->cchunk_ptr.assign(1, 0);
        if (c->pc.q > 0) {
            for (int cc = 0; cc < c->pc.n_coarse; ++cc) {
                const int a0 = c->pc.coarse_ptr[cc], a1 = c->pc.coarse_ptr[cc + 1];
                for (int e = a0; e < a1; e += kChunk) {
                    for (int k = e; k < std::min(a1, e + kChunk); ++k) c->grp_elems.push_back(c->pc.coarse_elems[k]);
                    c->grp_ptr.push_back((int32_t)c->grp_elems.size());
                }
                c->cchunk_ptr.push_back((int32_t)c->grp_ptr.size() - 1);
            }
        } else {
            const int64_t n = c->mesh.n_elem;
            for (int64_t e = 0; e < n; e += kChunk) {
                for (int64_t k = e; k < std::min<int64_t>(n, e + kChunk); ++k) c->grp_elems.push_back((int32_t)k);
                c->grp_ptr.push_back((int32_t)c->grp_elems.size());
            }
        }
        // Schwarz work items: the stored tiles (I, J <= I) of each packed tile
        // row, split into runs of ~item_kb KiB
        c->it_sys.clear(); c->it_row.clear(); c->it_j0.clear(); c->it_nj.clear(); c->it_rt.clear();
        c->rt_item0.assign(1, 0);
        c->rt_k.clear(); c->rt_nt.clear(); c->rt_cbase.clear();
        c->max_nj = 1;
        int64_t nloc_tiles = 0;
        for (int sidx = 0; sidx < c->pc.n_sub; ++sidx) nloc_tiles += c->pc.sys[sidx].nt * (c->pc.sys[sidx].nt + 1) / 2;
        for (size_t sidx = 0; sidx < c->pc.sys.size(); ++sidx) {
            const int64_t nt = c->pc.sys[sidx].nt;
            const int prec = (int)sidx < c->pc.n_sub ? c->pc.local_prec : c->pc.coarse_prec;
            const int64_t jc = std::max<int64_t>(1, ((int64_t)c->item_kb * 1024) / (kTile * kTile * (int64_t)tile_elem_bytes(prec)));
            const int64_t cbase = (int)sidx < c->pc.n_sub ? c->pc.sys[sidx].tile_off : nloc_tiles;
            for (int64_t I = 0; I < nt; ++I) {
                const int32_t rt = (int32_t)c->rt_item0.size() - 1;
                const int64_t ntile = I + 1, nc = (ntile + jc - 1) / jc;
                for (int64_t k = 0; k < nc; ++k) {
                    const int64_t j0 = k * ntile / nc, j1 = (k + 1) * ntile / nc;
                    c->it_sys.push_back((int32_t)sidx);
                    c->it_row.push_back((int32_t)I);
                    c->it_j0.push_back((int32_t)j0);
                    c->it_nj.push_back((int32_t)(j1 - j0));
                    c->it_rt.push_back(rt);
                    c->max_nj = std::max<int>(c->max_nj, (int)(j1 - j0));
                }
                c->rt_item0.push_back((int32_t)c->it_sys.size());
                c->rt_k.push_back((int32_t)I);
                c->rt_nt.push_back((int32_t)nt);
                c->rt_cbase.push_back(cbase);
            }
        }
        // tile row (and row inside it) of every fine dof, for assembling z
        {
            const int nd = c->mesh.nd;
            c->dof_rt.assign(c->mesh.n_elem * nd, 0);
            int32_t rt0 = 0;
            for (int sidx = 0; sidx < c->pc.n_sub; ++sidx) {
                const int a0 = c->pc.sub_ptr[sidx], a1 = c->pc.sub_ptr[sidx + 1];
                for (int le = 0; le < a1 - a0; ++le)
                    for (int i = 0; i < nd; ++i) {
                        const int pos = le * nd + i;
                        c->dof_rt[(int64_t)c->pc.sub_elems[a0 + le] * nd + i] = (rt0 + pos / kTile) * kTile + pos % kTile;
                    }
                rt0 += (int32_t)c->pc.sys[sidx].nt;
            }
            c->coarse_rt0 = c->pc.q > 0 ? rt0 : -1;
        }
        c->max_sys_n = 0;
        for (auto &S : c->pc.sys) c->max_sys_n = std::max<int>(c->max_sys_n, (int)S.n);
        // algorithmic bytes of one Schwarz apply: stored tiles + input gathers + outputs
        int64_t lt = 0, ctl = 0;
        for (int s = 0; s < c->pc.n_sub; ++s) lt += c->pc.sys[s].nt * (c->pc.sys[s].nt + 1) / 2;
        if (c->pc.q > 0) ctl = c->pc.sys[c->pc.n_sub].nt * (c->pc.sys[c->pc.n_sub].nt + 1) / 2;
        const int64_t N = c->mesh.n_elem * c->mesh.nd;
        c->schwarz_bytes = lt * kTile * kTile * (int64_t)tile_elem_bytes(c->pc.local_prec) +
                           ctl * kTile * kTile * (int64_t)tile_elem_bytes(c->pc.coarse_prec) + 3 * N * 8 +
                           3 * std::max<int64_t>(c->pc.N0, 0) * 8;
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
        if (c->pc.q == 0) throw Error(PDG_ESTATE, "no coarse level");
        if (P) std::copy(c->pc.P.begin(), c->pc.P.end(), P);
        if (K0) std::copy(c->pc.K0.begin(), c->pc.K0.end(), K0);
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
        c->ws = reinterpret_cast<char *>(dev_ptr);
        c->ws_bytes = bytes;
        const Mesh &m = c->mesh;
        const Precond &pc = c->pc;
        const int64_t n = m.n_elem;
        const int nd = m.nd;
        // matrix
        upload(c, W_GROWS, c->grp_rows);
        upload(c, W_GSLOT, c->grp_slot_off);
        upload(c, W_GCOL, c->grp_col);
        upload(c, W_GVAL, c->grp_val);
        upload(c, W_MASS, c->M);
        upload(c, W_MINV, c->Minv);
        upload(c, W_QPPTR, m.qp_ptr);
        upload(c, W_QPXI, m.qp_xi);
        upload(c, W_QPW, m.qp_w);
        upload(c, W_NORM, m.norm);
        std::vector<double> prm(kIonicParams, 0.0);
        if (c->has_ionic) prm = c->ionic;
        upload(c, W_PRM, prm);
        upload(c, W_SUBPTR, pc.sub_ptr);
        upload(c, W_SUBEL, pc.sub_elems);
        upload(c, W_ITSYS, c->it_sys);
        upload(c, W_ITROW, c->it_row);
        upload(c, W_ITJ0, c->it_j0);
        upload(c, W_ITNJ, c->it_nj);
        upload(c, W_ITRT, c->it_rt);
        upload(c, W_RTIT0, c->rt_item0);
        std::vector<int32_t> sys_n, sys_nt;
        std::vector<int64_t> sys_toff;
        for (size_t s = 0; s < pc.sys.size(); ++s) {
            sys_n.push_back((int32_t)pc.sys[s].n);
            sys_nt.push_back((int32_t)pc.sys[s].nt);
            // local systems index the local store; the coarse system its own store
            sys_toff.push_back((int)s < pc.n_sub ? pc.sys[s].tile_off : 0);
        }
        upload(c, W_SYSN, sys_n);
        upload(c, W_SYSNT, sys_nt);
        upload(c, W_SYSTOFF, sys_toff);
        // subdomains whose elements form one contiguous run gather r directly
        std::vector<int64_t> sys_dof0(pc.sys.size(), -1);
        for (int sidx = 0; sidx < pc.n_sub; ++sidx) {
            const int a0 = pc.sub_ptr[sidx], a1 = pc.sub_ptr[sidx + 1];
            bool contiguous = true;
            for (int k = a0 + 1; k < a1 && contiguous; ++k) contiguous = pc.sub_elems[k] == pc.sub_elems[k - 1] + 1;
            if (contiguous) sys_dof0[sidx] = (int64_t)pc.sub_elems[a0] * nd;
        }
        upload(c, W_SYSDOF0, sys_dof0);
        {
            int64_t nloc_tiles = 0;
            for (int sidx = 0; sidx < pc.n_sub; ++sidx) nloc_tiles += pc.sys[sidx].nt * (pc.sys[sidx].nt + 1) / 2;
            std::vector<int64_t> sys_cbase(pc.sys.size());
            for (size_t sidx = 0; sidx < pc.sys.size(); ++sidx)
                sys_cbase[sidx] = (int)sidx < pc.n_sub ? pc.sys[sidx].tile_off : nloc_tiles;
            upload(c, W_SYSCB, sys_cbase);
        }
        upload(c, W_RTK, c->rt_k);
        upload(c, W_RTNT, c->rt_nt);
        upload(c, W_RTCB, c->rt_cbase);
        // tiles, converted to the storage precision
        int64_t local_tiles = 0;
        for (int s = 0; s < pc.n_sub; ++s) local_tiles += pc.sys[s].nt * (pc.sys[s].nt + 1) / 2;
        const int64_t nloc = local_tiles * kTile * kTile;
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
                for (int64_t k = 0; k < count; ++k) b16[k] = to_bf16(src[k]);
                HIPCHK(hipMemcpyAsync(c->ws + c->lay.items[item].off, b16.data(), count * 2, hipMemcpyHostToDevice, c->stream));
                HIPCHK(hipStreamSynchronize(c->stream));
            }
        };
        put_tiles(W_TLOC, pc.inv64.data(), nloc, pc.local_prec);
        put_tiles(W_TCOA, pc.inv64.data() + nloc, ncoa, pc.coarse_prec);
        upload(c, W_P, pc.P);
        upload(c, W_ECOA, pc.elem_coarse);
        upload(c, W_GRPPTR, c->grp_ptr);
        upload(c, W_GRPEL, c->grp_elems);
        upload(c, W_CCHUNK, c->cchunk_ptr);
        upload(c, W_DOFRT, c->dof_rt);
        HIPCHK(hipMemsetAsync(c->ws + c->lay.items[W_SC].off, 0, 2 * 256, c->stream));
        for (int k = W_R; k <= W_Z0; ++k)
            HIPCHK(hipMemsetAsync(c->ws + c->lay.items[k].off, 0, c->lay.items[k].bytes, c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        // device pointers
        c->dA.nd = nd;
        c->dA.G = c->G;
        c->dA.n_rows = n;
        c->dA.n_groups = c->n_groups;
        c->dA.grp_rows = wptr<int32_t>(c, W_GROWS);
        c->dA.grp_slot_off = wptr<int64_t>(c, W_GSLOT);
        c->dA.grp_col = wptr<int32_t>(c, W_GCOL);
        c->dA.grp_val = wptr<double>(c, W_GVAL);
        c->dA.mass = wptr<double>(c, W_MASS);
        c->d_minv = wptr<double>(c, W_MINV);
        c->d_qp_ptr = wptr<int64_t>(c, W_QPPTR);
        c->d_qp_xi = wptr<double>(c, W_QPXI);
        c->d_qp_w = wptr<double>(c, W_QPW);
        c->d_norm = wptr<double>(c, W_NORM);
        c->d_prm = wptr<double>(c, W_PRM);
        c->d_sub_ptr = wptr<int32_t>(c, W_SUBPTR);
        c->d_sub_elems = wptr<int32_t>(c, W_SUBEL);
        c->d_it_sys = wptr<int32_t>(c, W_ITSYS);
        c->d_it_row = wptr<int32_t>(c, W_ITROW);
        c->d_it_j0 = wptr<int32_t>(c, W_ITJ0);
        c->d_it_nj = wptr<int32_t>(c, W_ITNJ);
        c->d_it_rt = wptr<int32_t>(c, W_ITRT);
        c->d_rt_item0 = wptr<int32_t>(c, W_RTIT0);
        c->d_dof_rt = wptr<int32_t>(c, W_DOFRT);
        c->d_itemdot = wptr<double>(c, W_ITDOT);
        c->d_spart = wptr<double>(c, W_PART);
        c->d_rrpart = wptr<double>(c, W_RRPART);
        c->d_part = wptr<double>(c, W_SPART);
        c->d_cchunk_ptr = wptr<int32_t>(c, W_CCHUNK);
        c->d_sys_n = wptr<int32_t>(c, W_SYSN);
        c->d_sys_nt = wptr<int32_t>(c, W_SYSNT);
        c->d_sys_toff = wptr<int64_t>(c, W_SYSTOFF);
        c->d_sys_dof0 = wptr<int64_t>(c, W_SYSDOF0);
        c->d_sys_cbase = wptr<int64_t>(c, W_SYSCB);
        c->d_rt_k = wptr<int32_t>(c, W_RTK);
        c->d_rt_nt = wptr<int32_t>(c, W_RTNT);
        c->d_rt_cbase = wptr<int64_t>(c, W_RTCB);
        c->d_colpart = wptr<double>(c, W_COLP);
        c->d_tiles_local = wptr<void>(c, W_TLOC);
        c->d_tiles_coarse = wptr<void>(c, W_TCOA);
        c->d_P = pc.q > 0 ? wptr<double>(c, W_P) : nullptr;
        c->d_elem_coarse = pc.q > 0 ? wptr<int32_t>(c, W_ECOA) : nullptr;
        c->d_grp_ptr = wptr<int32_t>(c, W_GRPPTR);
        c->d_grp_elems = wptr<int32_t>(c, W_GRPEL);
        c->v_r = wptr<double>(c, W_R);
        c->v_z = wptr<double>(c, W_Z);
        c->v_p = wptr<double>(c, W_PV);
        c->v_q = wptr<double>(c, W_Q);
        c->v_I = wptr<double>(c, W_I);
        c->v_t = wptr<double>(c, W_T);
        c->v_b = wptr<double>(c, W_B);
        c->d_r0part = wptr<double>(c, W_R0P);
        c->v_z0 = wptr<double>(c, W_Z0);
        c->sc = wptr<DevScalars>(c, W_SC);
        c->sc_apply = wptr<DevScalars>(c, W_SCA);
        c->state = S_BOUND;
    });
}

pdg_status pdg_set_option(pdg_ctx *c, int32_t option, int64_t value) {
    return guard(c, [&] {
        require(c, S_CREATED, "pdg_set_option");
        switch (option) {
        case PDG_OPT_TRUE_RESIDUAL: c->true_resid = value != 0; break;
        case PDG_OPT_CHUNK:
            if (value < 1 || value > 1000) throw Error(PDG_EINVAL, "chunk must be in 1..1000");
            c->chunk = (int)value;
            break;
        case PDG_OPT_KERNEL_TIMING: c->timing = value != 0; break;
        case PDG_OPT_SCHWARZ_ITEM_KB:
            if (value < 32 || value > 8192) throw Error(PDG_EINVAL, "item size must be in 32..8192 KiB");
            if (c->state >= S_PRECOND) throw Error(PDG_ESTATE, "set the item size before pdg_setup_preconditioner");
            c->item_kb = (int)value;
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
        HIPCHK(launch_project_p0(vals, ncomp, c->mesh.n_elem, c->mesh.nd, c->d_norm, coeff, c->stream));
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
        HIPCHK(launch_status_reset(sc, -1.0, 0, 0, c->stream));
        // restriction only (init mode: x and r untouched)
        HIPCHK(launch_update(update_args(c, 1, 0, c->v_t, const_cast<double *>(r), sc), c->stream));
        c->ev_used = 0;
        launch_schwarz_timed(c, schwarz_args(c, 0, r, sc));
        HIPCHK(launch_pupdate(pupdate_args(c, 0, 0, z, sc), c->stream));
        if (c->timing) {
            HIPCHK(hipStreamSynchronize(c->stream));
            harvest_timing(c, 1);
        }
    });
}

pdg_status pdg_ionic(pdg_ctx *c, const double *u, const double *u_prev, double *ions, double *I) {
    return guard(c, [&] {
        require_gpu(c);
        if (!c->has_ionic) throw Error(PDG_ESTATE, "pdg_set_ionic not called");
        if (!u || !u_prev || !ions || !I) throw Error(PDG_EINVAL, "NULL vector");
        HIPCHK(launch_status_reset(c->sc, 0.0, 0, 1, c->stream));
        IonicArgs a{};
        a.dim = c->mesh.dim;
        a.p = c->mesh.p;
        a.nd = c->mesh.nd;
        a.n_elem = c->mesh.n_elem;
        a.qp_ptr = c->d_qp_ptr;
        a.qp_xi = c->d_qp_xi;
        a.qp_w = c->d_qp_w;
        a.norm = c->d_norm;
        a.minv = c->d_minv;
        a.u = u;
        a.u_prev = u_prev;
        a.y = ions;
        a.I = I;
        a.prm = c->d_prm;
        a.dt = c->dt;
        a.sc = c->sc;
        HIPCHK(launch_ionic(a, c->stream));
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
    pdg_status st = PDG_OK;
    pdg_status g = guard(c, [&] {
        require_gpu(c);
        if (!rhs || !x) throw Error(PDG_EINVAL, "NULL vector");
        st = run_pcg(c, x, rhs, false, nullptr, nullptr, tol, maxit, info);
        if (st != PDG_OK) throw Error(st, std::string("PCG: ") + pdg_status_string(st));
    });
    return g;
}

pdg_status pdg_step(pdg_ctx *c, double *u, double *u_prev, double *ions, const double *f_ext, double tol,
                    int32_t maxit, pdg_solve_info *info) {
    return guard(c, [&] {
        require_gpu(c);
        if (!c->has_ionic) throw Error(PDG_ESTATE, "pdg_set_ionic not called");
        if (!u || !u_prev || !ions) throw Error(PDG_EINVAL, "NULL vector");
        HIPCHK(launch_status_reset(c->sc, 0.0, 0, 1, c->stream));
        IonicArgs a{};
        a.dim = c->mesh.dim;
        a.p = c->mesh.p;
        a.nd = c->mesh.nd;
        a.n_elem = c->mesh.n_elem;
        a.qp_ptr = c->d_qp_ptr;
        a.qp_xi = c->d_qp_xi;
        a.qp_w = c->d_qp_w;
        a.norm = c->d_norm;
        a.minv = c->d_minv;
        a.u = u;
        a.u_prev = u_prev;
        a.y = ions;
        a.I = c->v_I;
        a.prm = c->d_prm;
        a.dt = c->dt;
        a.sc = c->sc;
        HIPCHK(launch_ionic(a, c->stream));
        pdg_status st = run_pcg(c, u, nullptr, true, u_prev, f_ext, tol, maxit, info);
        if (c->sc_host->ionic_bad) throw Error(PDG_ENONFINITE, "ionic: non-positive concentration before a logarithm");
        if (st != PDG_OK) throw Error(st, std::string("PCG: ") + pdg_status_string(st));
    });
}

}  // extern "C"
