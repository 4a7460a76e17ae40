// Kernel launch interface of libpdg (host side of kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace pdg {

// Device-resident scalars of one PCG solve.  Written only by the last
// workgroup of a reduction; read by every later kernel on the stream.
struct DevScalars {
    double bb, rr, rz_unused, pq, alpha, beta, tol2;
    double tr;          // ||b - K x||^2 (true residual, optional)
    int32_t done;       // 1 = stop launching work
    int32_t status;     // 0 running/ok, 1 converged, 2 zero rhs, -5 noconv, -6 breakdown, -7 nonfinite
    int32_t iters;
    int32_t maxit;
    int32_t ionic_bad;  // a concentration <= 0 met before a logarithm
    int32_t pad[3];
    double rz[2];       // (r, z) of iterations of even / odd index
};

enum { ST_RUN = 0, ST_CONV = 1, ST_ZERO_RHS = 2, ST_NOCONV = -5, ST_BREAKDOWN = -6, ST_NONFINITE = -7 };

// Matrix in interleaved group-ELL form (see spmv kernel).
struct DevMatrix {
    int nd, G;              // block size, block rows per group
    int64_t n_rows, n_groups;
    const int32_t *grp_rows;     // [n_groups*G] row ids (-1 = padding)
    const int64_t *grp_slot_off; // [n_groups+1] slot offsets
    const int32_t *grp_col;      // [slots*G]
    const double *grp_val;       // [slots*G*nd*nd]
    const double *mass;          // [n_rows][nd][nd]
};

enum SpmvMode { SPMV_PLAIN = 0, SPMV_PQ = 1, SPMV_RESID = 2, SPMV_STEP = 3, SPMV_RHS = 4 };

struct SpmvArgs {
    int mode;
    const double *x;        // multiplied vector (p, x, or u)
    double *y;              // plain: Kx; PQ: q; RESID: r; STEP: r; RHS: b
    const double *b;        // RESID: right-hand side
    const double *I;        // STEP/RHS: ion term
    const double *f;        // STEP/RHS: optional applied current (nullable)
    double *u_prev;         // STEP: receives a copy of x
    double two_c, chi;      // STEP/RHS constants
    double *part;           // [gridDim][2] per-workgroup sums (PQ: (p,q); RESID: ||b||^2, ||r||^2; STEP: ||b||^2)
    DevScalars *sc;
};

struct UpdateArgs {
    int init;               // 1: no x/r update, iteration 0
    int iter;               // iteration index j (1-based) for the update
    int nd, nq0;
    const int32_t *grp_ptr, *grp_elems;  // update chunks: element ranges, each inside one coarse element
    int n_grp;
    double *x, *r;
    const double *p, *q;
    const double *P;        // [n_elem][nd][nq0] or null
    double *r0part;         // [n_grp][nq0] per-chunk restriction, or null
    const double *pqpart;   // [n_pq][2] SpMV partials ((p, q) in slot 0)
    int n_pq;
    double *rrpart;         // [n_grp] per-chunk ||r||^2
    DevScalars *sc;
};

// Work item of the Schwarz kernel: stored tiles (I, J), J in [j0, j0 + nj),
// of packed tile row I of system `sys` (all J <= I).  Each stored tile is
// read once and used twice: as stored for z_I (accumulated over the item,
// written as the item's row partial) and transposed for z_J, J < I (written as
// the tile's column partial).  The consumer adds the partials in fixed order.
struct SchwarzArgs {
    int mode;               // 0 apply only, 1/2 inside PCG (also writes the (r, z) shares)
    int nd, n_sub, nq0;
    const int32_t *item_sys, *item_row, *item_j0, *item_nj;
    double *part;                // [n_items][64] row partials
    double *colpart;             // [n_tiles_total][64] column partials (indexed by global tile index)
    double *itemdot;             // [n_items] shares of (r, z) + (r0, z0)
    const int32_t *sys_n, *sys_nt;
    const int64_t *sys_toff;     // tile offset of each system inside its own store
    const int64_t *sys_cbase;    // global tile index of each system's first tile (column partials)
    const int64_t *sys_dof0;     // first dof of a subdomain whose elements are one contiguous run, else -1
    const void *tiles_local;     // tile store of the local systems (storage type per launch)
    const void *tiles_coarse;    // tile store of the coarse system
    const int32_t *sub_ptr, *sub_elems;
    const int32_t *cchunk_ptr;   // [n_coarse+1] update chunks of each coarse element
    const double *r;        // fine residual
    const double *r0part;   // per-chunk coarse restriction (summed on gather)
    DevScalars *sc;
};

// Assembles z = B r from the Schwarz partials (row partials of the items of
// a tile row, column partials of the stored tiles below it, and P z0) and
// updates the search direction; in PCG modes it also closes the iteration:
// (r, z), beta, convergence on ||r||^2.
struct PupdateArgs {
    int mode;               // 0: out = z; 1: PCG init, p = z; 2: PCG, p = z + beta p
    int iter;
    int nd, nq0;
    int64_t n_elem;
    const double *P;
    const int32_t *elem_coarse;
    const int32_t *dof_rt;       // [N] tile row * 64 + row inside the tile, of every fine dof
    const int32_t *rt_item0;     // [n_rt+1] first item of each tile row
    const int32_t *rt_k, *rt_nt; // tile-row index inside its system, tile rows of the system
    const int64_t *rt_cbase;     // global tile index of the system's first tile
    int coarse_rt0;              // first tile row of the coarse system (or -1)
    const double *part;          // Schwarz row partials
    const double *colpart;       // Schwarz column partials
    const double *itemdot;
    int n_items;
    const double *rrpart;        // update partials
    int n_rr;
    const double *bbpart;        // SpMV partials of the right-hand side (init only)
    int n_bb;
    double *p;                   // output
    DevScalars *sc;
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
    DevScalars *sc;
};

enum LocalStorage { STORE_F64 = 0, STORE_F32 = 1, STORE_BF16 = 2 };

hipError_t launch_spmv(const DevMatrix &A, const SpmvArgs &a, hipStream_t s);
int spmv_blocks(const DevMatrix &A);
hipError_t launch_update(const UpdateArgs &a, hipStream_t s);
// Launches the Schwarz kernel over items [item0, item0 + n_items) with the
// given storage type; the coarse items (if any) use coarse_store.
hipError_t launch_schwarz(const SchwarzArgs &a, int n_items, int local_store, int coarse_store,
                          int max_nj, hipStream_t s);
hipError_t launch_pupdate(const PupdateArgs &a, hipStream_t s);
hipError_t launch_ionic(const IonicArgs &a, hipStream_t s);
hipError_t launch_project_p0(const double *vals, int ncomp, int64_t n_elem, int nd, const double *norm,
                             double *coeff, hipStream_t s);
hipError_t launch_zero(double *x, int64_t n, hipStream_t s);
hipError_t launch_status_reset(DevScalars *sc, double tol2, int maxit, int reset_ionic, hipStream_t s);
// Sums `n` partials (stride 2, slot `slot`) into *out with one workgroup.
hipError_t launch_sum_partials(const double *part, int n, int slot, double *out, hipStream_t s);

}  // namespace pdg
