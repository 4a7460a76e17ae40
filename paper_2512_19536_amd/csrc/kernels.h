// Kernel launch interface of libpdg (host side of kernels.hip).
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace pdg {

// Device-resident scalars of one PCG solve.  Written only by the last
// workgroup of a reduction; read by every later kernel on the stream.
struct DevScalars {
    double bb, rr, rz, pq, alpha, beta, tol2;
    double tr;          // ||b - K x||^2 (true residual, optional)
    int32_t done;       // 1 = stop launching work
    int32_t status;     // 0 running/ok, 1 converged, 2 zero rhs, -5 noconv, -6 breakdown, -7 nonfinite
    int32_t iters;
    int32_t maxit;
    int32_t ionic_bad;  // a concentration <= 0 met before a logarithm
    int32_t pad[3];
};

enum { ST_RUN = 0, ST_CONV = 1, ST_ZERO_RHS = 2, ST_NOCONV = -5, ST_BREAKDOWN = -6, ST_NONFINITE = -7 };

struct RedSlot {            // one deterministic two-stage reduction
    double *partials;       // [n_blocks][nv]
    uint32_t *counter;      // zero between launches
};

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
    RedSlot red;
    DevScalars *sc;
    double *bb_out;         // RESID/STEP: destination of the first sum (||b||^2)
    double *rr_out;         // RESID: destination of the second sum (||r||^2), nullable
};

struct UpdateArgs {
    int init;               // 1: no x/r update, iteration 0
    int iter;               // iteration index j (1-based) for the update
    int nd, nq0;
    const int32_t *grp_ptr, *grp_elems;  // update groups (coarse elements or chunks)
    int n_grp;
    double *x, *r;
    const double *p, *q;
    const double *P;        // [n_elem][nd][nq0] or null
    double *r0;             // [n_grp*nq0] or null
    RedSlot red;
    DevScalars *sc;
};

struct SchwarzArgs {
    int mode;               // 0 apply only, 1 PCG init (beta = 0), 2 PCG (beta = rz'/rz)
    int nd, n_sub;
    const int32_t *item_sys, *item_row;
    const int32_t *sys_n, *sys_nt;
    const int64_t *sys_toff;
    const void *tiles_local;     // tile store of the local systems (storage type per launch)
    const void *tiles_coarse;    // tile store of the coarse system
    const int32_t *sub_ptr, *sub_elems;
    const double *r;        // fine residual
    const double *r0;       // coarse residual
    double *z;              // local part of B r (element-dof layout)
    double *z0;             // coarse solution
    RedSlot red;
    DevScalars *sc;
};

struct PupdateArgs {
    int mode;               // 0: out = z + P z0; 1: p = z + P z0; 2: p = z + P z0 + beta p
    int nd, nq0;
    int64_t n_elem;
    const double *z, *z0, *P;
    const int32_t *elem_coarse;
    double *p;              // output
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
                          int max_n, hipStream_t s);
hipError_t launch_pupdate(const PupdateArgs &a, hipStream_t s);
hipError_t launch_ionic(const IonicArgs &a, hipStream_t s);
hipError_t launch_project_p0(const double *vals, int ncomp, int64_t n_elem, int nd, const double *norm,
                             double *coeff, hipStream_t s);
hipError_t launch_zero(double *x, int64_t n, hipStream_t s);
hipError_t launch_status_reset(DevScalars *sc, double tol2, int maxit, int reset_ionic, hipStream_t s);

}  // namespace pdg
