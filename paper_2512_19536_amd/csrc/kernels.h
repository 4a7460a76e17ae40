// Kernel launch interface of libpdg (host side of kernels.hip).
//
// A context holds a batch of n_sys independent systems (one for a plain
// solve).  Elements, dofs, SpMV groups, update chunks and Schwarz items are
// ordered by system and never straddle two systems, so every per-workgroup
// partial belongs to one system and each system runs its own PCG (own alpha,
// beta and stopping test) inside the same launches.  No kernel takes an
// iteration index: the counter lives in the device scalars, so a chunk of
// iterations is a fixed sequence of launches that can be replayed as a graph.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstddef>
#include <cstdint>

namespace pdg {

// Device-resident scalars of one system's PCG.  Every field has one writer per
// launch (the system's owner workgroup, thread 0); later launches read it.
struct DevScalars {
    double bb, rr, pq, alpha, beta, tol2;
    double tr;          // ||b - K x||^2 (true residual, optional)
    double pq_sum;      // (p, q) summed by the reduction kernel (when the update kernel does not sum it)
    double rz_sum;      // (r, z) summed by the reduction kernel (when the p-update kernel does not sum it)
    double lmin, lmax;  // extreme eigenvalues of the Lanczos matrix of the last solve (on request)
    double rz[2];       // (r, z) of the search directions of even / odd index
    int32_t done;       // 1 = this system stops
    int32_t status;     // 0 running, 1 converged, 2 zero rhs, -5 noconv, -6 breakdown, -7 nonfinite
    int32_t iters;      // completed iterations
    int32_t jcur;       // iteration in progress (set by the update kernel, read by the p-update kernel)
    int32_t maxit;
    int32_t ionic_bad;  // a concentration <= 0 met before a logarithm (system 0 holds the batch flag)
    int32_t guess;      // -1 no initial guess offered, 0 rejected (x0 = U^k), 1 used
    int32_t pad;
};

enum { ST_RUN = 0, ST_CONV = 1, ST_ZERO_RHS = 2, ST_NOCONV = -5, ST_BREAKDOWN = -6, ST_NONFINITE = -7 };

// Element blocks of more than 32 rows (one element row per SpMV group) are
// stored in chunks of this many consecutive slots of a row, and inside a
// chunk trial-index major: value (slot c0 + sl, trial j, test i) of a group
// whose slots start at s0 sits at
//   (s0 + c0) * nd * nd + j * (nch * nd) + sl * nd + i,   nch = slots in the chunk,
// so for each j the chunk's (slot, test) pairs are one contiguous run.
constexpr int kWideChunk = 16;
constexpr int kWideMinNd = 33;

// Per-system ranges of the partial-sum producers (workgroups of the SpMV,
// update and Schwarz kernels, one partial each): system s owns [x[s], x[s+1]).
struct SysRanges {
    int n_sys;
    const int32_t *spmv;    // SpMV workgroups
    const int32_t *upd;     // update workgroups
    const int32_t *item;    // Schwarz workgroups
    const int32_t *owner;   // [n_sys] p-update workgroup holding the system's first dof
};

// What an SpMV workgroup needs first, in one 32-byte record: its groups
// [g_begin, g_end), their system, and the slot range [s0, s1) of its first
// group.
struct alignas(32) SpDesc {
    int32_t g_begin, g_end, sys, pad0;
    int64_t s0, s1;
};

// Matrix in interleaved group-ELL form (see the SpMV kernel).
struct DevMatrix {
    int nd, G;              // block size, block rows per group
    int wpg;                // wavefronts per group (1, 2, 4 or 8)
    int nt;                 // 1: stream the values with non-temporal loads (matrix larger than the cache)
    int64_t n_rows, n_groups;
    const int32_t *grp_rows;     // [n_groups*G] row ids (-1 = padding)
    const int64_t *grp_slot_off; // [n_groups+1] slot offsets
    const int32_t *grp_col;      // [slots*G]
    const double *grp_val;       // [slots*G*nd*nd]
    const double *mass;          // [n_rows][nd][nd]
    int n_wg;
    const SpDesc *wg_desc;       // [n_wg]
    int one_sys;                 // 1: one system (its stop flag is sc[0])
};

enum SpmvMode { SPMV_PLAIN = 0, SPMV_PQ = 1, SPMV_RESID = 2, SPMV_STEP = 3, SPMV_RHS = 4 };

struct SpmvArgs {
    int mode;
    const double *x;        // multiplied vector (p, x, or u)
    double *y;              // plain: Kx; PQ: q; RESID: r; STEP: r; RHS: b
    const double *b;        // RESID: right-hand side
    const double *I;        // STEP/RHS: ion term
    const double *f;        // STEP/RHS: optional applied current (nullable)
    double *u_prev;         // STEP, RESID: receives a copy of x (nullable in RESID)
    double *xcopy;          // STEP/RESID: receives a copy of x (the PCG iterate), nullable
    double two_c, chi;      // STEP/RHS constants
    double *part;           // [groups][2] per-workgroup sums (PQ: (p,q); RESID: ||b||^2, ||r||^2; STEP: ||b||^2)
    DevScalars *sc;         // [n_sys]
};

// What an update workgroup needs first, in one 32-byte record: its chunks
// [c_begin, c_end), its system b and that system's SpMV workgroups
// [g0, g1), and its first chunk: elements grp_elems[f_e0 .. f_e0 + f_n) of
// grp_ptr, which are the run e_first .. e_first + f_n - 1 if e_first >= 0.
struct alignas(32) UpdDesc {
    int32_t c_begin, c_end, b, g0, g1, f_e0, f_n, e_first;
};

struct UpdateArgs {
    int init;               // 1: no x/r update (iteration 0)
    int pre_pq;             // 1: take (p, q) from sc.pq_sum instead of summing the SpMV partials
    int nd, nq0;
    const int32_t *grp_ptr, *grp_elems;  // update chunks: element runs inside one coarse element
    int n_wg;
    double *x, *r;
    const double *p, *q;
    const double *P;        // [n_elem][nd][nq0] or null
    double *r0part;         // [n_grp][nq0] per-chunk restriction, or null
    const double *pqpart;   // SpMV partials ((p, q) in slot 0)
    double *rrpart;         // [n_wg] per-workgroup ||r||^2
    double2 *lanczos;       // [n_sys][lcap] (alpha_j, beta_j) of each iteration j, or null
    int lcap;
    SysRanges rng;
    DevScalars *sc;
    const UpdDesc *wg_desc; // [n_wg]
};

// Everything a Schwarz workgroup needs to know about its item, in one
// 64-byte line: the item (system s, tile row I, tiles j0 .. j0 + nj - 1),
// the batch system that owns it, and the dense system's size n, tile offset
// in its store, global index of its first tile, first dof of a contiguous
// subdomain (else -1), first row of its BF16 scales and its FP32-fallback
// flag.
struct alignas(64) ItemDesc {
    int32_t s, I, j0, nj;
    int32_t owner, n, toff, cbase;
    int32_t dof0, rbase, f32, pad0;
    int32_t pad1[4];
};

// Work item of the Schwarz kernel: stored tiles (I, J), J in [j0, j0 + nj),
// of packed tile row I of dense system `sys` (a subdomain, or the coarse
// system of one batch system; all J <= I).  Each stored tile is read once and
// used twice: as stored for z_I (accumulated over the item, written as the
// item's row partial) and transposed for z_J, J < I (written as the tile's
// column partial).  The consumer adds the partials in fixed order.
struct SchwarzArgs {
    int mode;               // 0 apply only, 1/2 inside PCG (also writes the (r, z) shares)
    int nd, n_sub, nq0;
    // Row and column partials, stored in FP64, or in FP32 (the first half of
    // each buffer) when both the local and the coarse store accumulate in FP32.
    double *part;                // [n_items][64] row partials
    double *colpart;             // [n_tiles_total][64] column partials (indexed by global tile index)
    double *itemdot;             // [n_items] shares of (r, z) + (r0, z0)
    const int32_t *csys_ce0;     // [n_sys+1] first coarse element of each batch system
    const void *tiles_local;     // tile store of the local systems
    const void *tiles_coarse;    // tile store of the coarse systems
    const int32_t *sub_ptr, *sub_elems;
    const int32_t *cchunk_ptr;   // [n_coarse+1] update chunks of each coarse element
    const double *r;        // fine residual
    const double *r0part;   // per-chunk coarse restriction (summed on gather)
    DevScalars *sc;
    const ItemDesc *item_desc;   // [n_items]
    int n_sys_one;               // 1: one system in the context (its stop flag is sc[0])
    // BF16 local store only (else null): the stored tiles of local system s
    // hold C = D^{-1} K_s^{-1} D^{-1}; d of its row i is dscale[rbase + i] (rbase
    // and the FP32-fallback flag are in the item descriptor).  Systems flagged
    // FP32 are stored unscaled in tiles_fallback (their descriptor's tile
    // offset indexes that store).
    const float *dscale;
    const void *tiles_fallback;
};

// Assembles z = B r from the Schwarz partials (row partials of the items of
// a tile row, column partials of the stored tiles below it, and P z0) and
// updates the search direction; in PCG modes it also closes each system's
// iteration: (r, z), beta, convergence on ||r||^2.
// Coarse elements whose values a p-update block keeps in LDS.
constexpr int kPupdateKmax = 8;

// Where one value of z = B r is assembled from (a tile row of a dense system
// and a row inside it), in one 16-byte record: the first of the tile row's
// nit items, the global index cb of the dense system's first tile, the
// tile row K inside the system and the system's nt tile rows, the row lane.
struct alignas(16) ZSrc {
    int32_t it0, cb, knt /* K << 16 | nt */, nl /* nit << 8 | lane */;
};

// Per p-update block (256 dofs), in one 32-byte record: the batch systems of
// its first and last dof, the coarse elements its dofs touch (first and
// count, or kPupdateKmax + 1), and the Schwarz-item and update-workgroup
// ranges of its first system.
struct alignas(32) PuBlk {
    int32_t s_lo, s_hi, c_lo, n_c, it0, it1, u0, u1;
};

struct PupdateArgs {
    int mode;               // 0: out = z; 1: PCG init, p = z; 2: PCG, p = z + beta p
    int pre_rz;             // 1: take (r, z) from sc.rz_sum instead of summing the Schwarz shares
    int nd, nq0;
    const double *r_ident;  // non-null: no preconditioner (z = r_ident, (r, z) from the update partials)
    int64_t n_elem;
    const double *P;
    const int32_t *elem_coarse;  // coarse element of each element (system-contiguous numbering)
    const int32_t *elem_sys;     // batch system of each element
    const int32_t *rt_item0;     // [n_rt+1] first item of each tile row
    const int32_t *rt_k, *rt_nt; // tile-row index inside its dense system, tile rows of the system
    const int64_t *rt_cbase;     // global tile index of the dense system's first tile
    const int32_t *coarse_base;  // [n_coarse] value j of coarse element c: tile row (base + j) / 64,
                                 // row (base + j) % 64
    const double *part;          // Schwarz row partials
    const double *colpart;       // Schwarz column partials
    int f32part;                 // 1: the Schwarz partials are stored in FP32
    const double *itemdot;
    const double *rrpart;        // update partials
    const double *bbpart;        // SpMV partials of the right-hand side (init only)
    SysRanges rng;
    double *p;                   // output
    double2 *lanczos;            // [n_sys][lcap] (alpha_j, beta_j), or null
    int lcap;
    DevScalars *sc;
    const PuBlk *blk;            // [blocks]
    const ZSrc *dof_src;         // [N] fine value of every dof
    const ZSrc *blk_csrc;        // [blocks][kPupdateKmax * nq0] coarse values kept by each block
};

struct IonicArgs {
    int dim, p, nd;
    int64_t n_elem;
    const int64_t *qp_ptr;
    const double *qp_xi, *qp_w, *norm, *minv;
    const double *u, *u_prev;
    double *y;              // [5][n_elem][nd] in place
    double *I;
    const double *prm;      // 24 ionic parameters
    double dt;
    double ext_now, ext_prev;  // u~ = ext_now u^k + ext_prev u^(k-1) in the ion term
    int32_t *bad;           // set to 1 when a concentration <= 0 is met
};

enum LocalStorage { STORE_F64 = 0, STORE_F32 = 1, STORE_BF16 = 2 };

hipError_t launch_spmv(const DevMatrix &A, const SpmvArgs &a, hipStream_t s);
hipError_t launch_update(const UpdateArgs &a, hipStream_t s);
// One block per item (grid = number of items); with events, the dispatch
// records its own start and stop times in them.
hipError_t launch_schwarz(const SchwarzArgs &a, int grid, int local_store, int coarse_store,
                          int max_nj, hipStream_t s, hipEvent_t e0 = nullptr, hipEvent_t e1 = nullptr);
// LDS bytes the Schwarz kernel needs for items of up to max_nj tiles.
size_t schwarz_lds_bytes(int local_store, int coarse_store, int max_nj);
hipError_t launch_pupdate(const PupdateArgs &a, hipStream_t s);
hipError_t launch_ionic(const IonicArgs &a, hipStream_t s);
hipError_t launch_project_p0(const double *vals, int ncomp, int64_t n_elem, int nd, const double *norm,
                             double *coeff, hipStream_t s);
hipError_t launch_status_reset(DevScalars *sc, int n_sys, double tol2, int maxit, int reset_ionic,
                               hipStream_t s);
// One block per system: sc[s].pq_sum = sum of the system's SpMV partials
// (slot 0, stride 2) if which == 0, sc[s].rz_sum = sum of its Schwarz shares
// if which == 1.
hipError_t launch_reduce(const double *part, const int32_t *ranges, int n_sys, int which, DevScalars *sc,
                         hipStream_t s);
// One block per system: extreme eigenvalues of the Lanczos matrix built from
// the recorded PCG coefficients of the last solve (T_11 = 1/alpha_1,
// T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_j,j+1 = sqrt(beta_j)/alpha_j,
// j <= iters) into sc[s].lmin / lmax.
hipError_t launch_lanczos(const double2 *hist, int lcap, int n_sys, DevScalars *sc, hipStream_t s);
// Sums the SpMV partials (stride 2, slot `slot`) of each system into sc[s].tr.
hipError_t launch_sum_partials(const double *part, const int32_t *ranges, int n_sys, int slot, DevScalars *sc,
                               hipStream_t s);
// Initial guess choice, per system: where ||b - K g||^2 (SpMV partials, slot 1)
// is below ||b - K u||^2 (sc.tr), x = g and r = r_g; else x and r stay those of u.
struct ChooseArgs {
    int nd;
    const int32_t *grp_ptr, *grp_elems, *grp_sys;  // update chunks
    const int32_t *sys_chunk0;                     // [n_sys] first chunk of each system
    int n_grp;
    const double *part;      // SpMV partials of the guess residual
    const double *g, *r_g;   // guess and its residual
    double *x, *r;           // PCG iterate and residual (hold those of u)
    SysRanges rng;
    DevScalars *sc;
};
hipError_t launch_choose(const ChooseArgs &a, hipStream_t s);
// guess = 2 u - u1 (order 1) or 3 u - 3 u1 + u2 (order 2)
hipError_t launch_extrapolate(const double *u, const double *u1, const double *u2, int order, int64_t n,
                              double *guess, hipStream_t s);
// out = x on every dof, except 0 on the dofs of systems that stopped with a zero right-hand side.
hipError_t launch_finish(const double *x, double *out, const int32_t *elem_sys, int nd, int64_t n_elem,
                         const DevScalars *sc, hipStream_t s);

// Scratch of the allocation-free preconditioner apply: a static device array
// of kStaticScratchBytes per device.  static_scratch_init looks up its address
// on `device`, which must be the current device (once per device; later calls
// return at once); static_scratch returns that address, or null before init.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
hipError_t static_scratch_init(int device);
void *static_scratch(int device);

}  // namespace pdg
