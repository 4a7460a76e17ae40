// HIP kernels of libpdg for gfx950 (CDNA4, wave64).
//
// Per PCG iteration (Section 4: PCG with the additive Schwarz operator of
// eq. (5)) the stream runs four kernels:
//   k_spmv   (mode PQ)  q = K p, (p, q)              -> alpha = (r, z) / (p, q)
//   k_update            x += alpha p, r -= alpha q, ||r||^2, r0 = P^T r
//   k_schwarz           z = K_i^{-1} r_i (all subdomains), z0 = K_0^{-1} r0,
//                       (r, z) + (r0, z0)              -> beta
//   k_pupdate           p = z + P z0 + beta p
// Global sums use a deterministic two-stage reduction: each workgroup writes a
// partial sum, the last workgroup to finish (integer ticket) adds the partials
// in a fixed order and writes the scalar.  No floating-point atomics, so two
// runs on the same input give bitwise-equal results.  Every kernel returns at
// once when the device-side "done" flag is set, so surplus iterations queued
// past convergence cost a launch each and change nothing.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace pdg {

constexpr int TILE = 64;

// ---------------------------------------------------------------------------
// reductions
template <int NV>
__device__ inline void wave_sum(double (&v)[NV]) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] += __shfl_xor(v[k], off, 64);
}

// Block totals of v (valid in thread 0 only).
template <int NV, int BS>
__device__ inline void block_sum(double (&v)[NV], double (&tot)[NV]) {
    __shared__ double sh[BS / 64][NV];
    wave_sum<NV>(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[w][k] = v[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = 0.0;
            for (int ww = 0; ww < BS / 64; ++ww) s += sh[ww][k];
            tot[k] = s;
        }
    }
    __syncthreads();
}

// Writes this block's partial (thread 0's `part`) and returns true in every
// thread of the last block to arrive, with the grid totals in `tot` (thread 0).
template <int NV, int BS>
__device__ inline bool grid_sum(const double (&part)[NV], RedSlot red, double (&tot)[NV]) {
    __shared__ int is_last;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) red.partials[(int64_t)blockIdx.x * NV + k] = part[k];
        __threadfence();
        const unsigned t = atomicAdd(red.counter, 1u);
        is_last = (t == gridDim.x - 1);
    }
    __syncthreads();
    if (!is_last) return false;
    __threadfence();
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = 0.0;
    for (int b = threadIdx.x; b < (int)gridDim.x; b += BS)
#pragma unroll
        for (int k = 0; k < NV; ++k) acc[k] += __builtin_nontemporal_load(&red.partials[(int64_t)b * NV + k]);
    block_sum<NV, BS>(acc, tot);
    if (threadIdx.x == 0) *red.counter = 0u;
    return true;
}

__device__ inline bool finite(double x) { return __builtin_isfinite(x); }

// ---------------------------------------------------------------------------
// Block-sparse SpMV over element rows in interleaved group-ELL form.
// G = 64 / ND element rows form a group handled by one wavefront; lane
// (r, i) = (lane / ND, lane % ND) owns output row i of the group's r-th
// element.  Group values are stored slot-major so that for every (slot s,
// trial index j) the wavefront reads G*ND consecutive doubles:
//   val[((s * ND + j) * G + r) * ND + i] = K_{row_r, col_{s,r}}[i][j].
template <int ND, int WPB>
__global__ __launch_bounds__(64 * WPB) void k_spmv(DevMatrix A, SpmvArgs a) {
    constexpr int G = ND <= 64 ? 64 / ND : 1;
    if (a.mode == SPMV_PQ && a.sc->done) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t g = (int64_t)blockIdx.x * WPB + w;
    const int r = lane / ND, i = lane - (lane / ND) * ND;
    double acc = 0.0;
    int row = -1;
    if (g < A.n_groups && r < G) {
        row = A.grp_rows[g * G + r];
        const int64_t s0 = A.grp_slot_off[g], ns = A.grp_slot_off[g + 1] - s0;
        const int32_t *colp = A.grp_col + s0 * G + r;
        const double *vp = A.grp_val + s0 * G * ND * ND + lane;
        for (int64_t s = 0; s < ns; ++s) {
            const double *xb = a.x + (int64_t)colp[s * G] * ND;
            const double *vs = vp + s * G * ND * ND;
            double v[ND];
#pragma unroll
            for (int j = 0; j < ND; ++j) v[j] = vs[j * G * ND];
#pragma unroll
            for (int j = 0; j < ND; ++j) acc = fma(v[j], xb[j], acc);
        }
    }
    double part[2] = {0.0, 0.0};
    if (row >= 0) {
        const int64_t idx = (int64_t)row * ND + i;
        switch (a.mode) {
        case SPMV_PLAIN:
            a.y[idx] = acc;
            break;
        case SPMV_PQ:
            a.y[idx] = acc;
            part[0] = a.x[idx] * acc;
            break;
        case SPMV_RESID: {
            const double bv = a.b[idx], rv = bv - acc;
            a.y[idx] = rv;
            part[0] = bv * bv;
            part[1] = rv * rv;
            break;
        }
        case SPMV_STEP:
        case SPMV_RHS: {
            const double *Mr = A.mass + (int64_t)row * ND * ND;
            const double *ur = a.x + (int64_t)row * ND;
            double mu = 0.0;
#pragma unroll
            for (int j = 0; j < ND; ++j) mu = fma(Mr[j * ND + i], ur[j], mu);
            double bv = a.two_c * mu - acc - a.chi * a.I[idx];
            if (a.f) bv += a.f[idx];
            if (a.mode == SPMV_RHS) {
                a.y[idx] = bv;
            } else {
                a.y[idx] = bv - acc;  // r0 = b - K u  (x0 = u)
                a.u_prev[idx] = ur[i];
                part[0] = bv * bv;
            }
            break;
        }
        }
    }
    if (a.mode == SPMV_PLAIN || a.mode == SPMV_RHS) return;
    double tot[2];
    block_sum<2, 64 * WPB>(part, tot);
    if (grid_sum<2, 64 * WPB>(tot, a.red, tot) && threadIdx.x == 0) {
        DevScalars *sc = a.sc;
        if (a.mode == SPMV_PQ) {
            const double pq = tot[0];
            sc->pq = pq;
            if (!finite(pq)) {
                sc->status = ST_NONFINITE;
                sc->done = 1;
            } else if (!(pq > 0.0)) {
                sc->status = ST_BREAKDOWN;
                sc->done = 1;
            } else {
                sc->alpha = sc->rz / pq;
            }
        } else {
            if (a.bb_out) *a.bb_out = tot[0];
            if (a.rr_out) *a.rr_out = tot[1];
        }
    }
}

// ---------------------------------------------------------------------------
// x += alpha p, r -= alpha q, ||r||^2 and the coarse restriction r0 = P^T r.
// One workgroup per update group (a coarse element, or a chunk of elements
// when there is no coarse level) so that r0[c] is a block-local sum.
template <int ND, int NQ>
__global__ __launch_bounds__(256) void k_update(UpdateArgs a) {
    DevScalars *sc = a.sc;
    if (sc->done) return;
    const double alpha = a.init ? 0.0 : sc->alpha;
    const int c = blockIdx.x;
    const int e0 = a.grp_ptr[c], ndof = (a.grp_ptr[c + 1] - e0) * ND;
    double v[1 + (NQ > 0 ? NQ : 1)];
#pragma unroll
    for (int k = 0; k < 1 + (NQ > 0 ? NQ : 1); ++k) v[k] = 0.0;
    for (int d = threadIdx.x; d < ndof; d += 256) {
        const int le = d / ND, i = d - le * ND;
        const int64_t idx = (int64_t)a.grp_elems[e0 + le] * ND + i;
        double rv = a.r[idx];
        if (!a.init) {
            a.x[idx] = fma(alpha, a.p[idx], a.x[idx]);
            rv = fma(-alpha, a.q[idx], rv);
            a.r[idx] = rv;
        }
        v[0] = fma(rv, rv, v[0]);
        if (NQ > 0) {
            const double *Pr = a.P + idx * NQ;
#pragma unroll
            for (int j = 0; j < NQ; ++j) v[1 + j] = fma(Pr[j], rv, v[1 + j]);
        }
    }
    constexpr int NV = 1 + (NQ > 0 ? NQ : 1);
    double tot[NV];
    block_sum<NV, 256>(v, tot);
    if (NQ > 0 && threadIdx.x == 0)
#pragma unroll
        for (int j = 0; j < NQ; ++j) a.r0[c * NQ + j] = tot[1 + j];
    double part[1] = {tot[0]}, rr[1];
    if (grid_sum<1, 256>(part, a.red, rr) && threadIdx.x == 0) {
        const double r2 = rr[0];
        sc->rr = r2;
        if (a.init) {
            sc->iters = 0;
            if (sc->bb == 0.0) {
                sc->status = ST_ZERO_RHS;
                sc->done = 1;
            } else if (!finite(r2) || !finite(sc->bb)) {
                sc->status = ST_NONFINITE;
                sc->done = 1;
            } else if (r2 <= sc->tol2 * sc->bb) {
                sc->status = ST_CONV;
                sc->done = 1;
            }
        } else {
            sc->iters = a.iter;
            if (!finite(r2)) {
                sc->status = ST_NONFINITE;
                sc->done = 1;
            } else if (r2 <= sc->tol2 * sc->bb) {
                sc->status = ST_CONV;
                sc->done = 1;
            } else if (a.iter >= sc->maxit) {
                sc->status = ST_NOCONV;
                sc->done = 1;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Schwarz apply: z_i = K_i^{-1} r_i for every subdomain and z0 = K_0^{-1} r0.
// Each inverse is symmetric and stored as packed lower-triangular 64x64 tiles
// (row-major inside a tile).  A workgroup (256 threads) owns one 64-row tile
// row I of one system and streams the nt tiles of that row: tile (I, J) for
// J <= I used as stored, tile (J, I) for J > I used transposed.  Each thread
// loads 16 bytes per tile row for RPT rows, so every load instruction of a
// wavefront reads whole contiguous tile rows.
template <typename E> struct AccT { using T = float; };
template <> struct AccT<double> { using T = double; };

struct alignas(16) Vec16 { uint32_t w[4]; };

template <typename E, int CW>
__device__ inline void unpack(const Vec16 &v, typename AccT<E>::T (&out)[CW]);

template <>
__device__ inline void unpack<double, 2>(const Vec16 &v, double (&out)[2]) {
    out[0] = __hiloint2double(v.w[1], v.w[0]);
    out[1] = __hiloint2double(v.w[3], v.w[2]);
}
template <>
__device__ inline void unpack<float, 4>(const Vec16 &v, float (&out)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) out[k] = __uint_as_float(v.w[k]);
}
template <>
__device__ inline void unpack<uint16_t, 8>(const Vec16 &v, float (&out)[8]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        out[2 * k] = __uint_as_float(v.w[k] << 16);
        out[2 * k + 1] = __uint_as_float(v.w[k] & 0xffff0000u);
    }
}

template <typename E>
__device__ inline void tile_row_product(const E *__restrict__ tiles, int64_t toff, int nt, int I,
                                        const typename AccT<E>::T *xs, typename AccT<E>::T *yout,
                                        typename AccT<E>::T *scratch) {
    using A = typename AccT<E>::T;
    constexpr int CW = 16 / sizeof(E);  // columns per 16-byte load
    constexpr int NC = TILE / CW;       // column groups per tile row
    constexpr int RG = 256 / NC;        // row groups
    constexpr int RPT = TILE / RG;      // rows per thread
    const int tid = threadIdx.x, cg = tid % NC, rg = tid / NC;
    A accR[RPT], accC[CW];
#pragma unroll
    for (int k = 0; k < RPT; ++k) accR[k] = 0;
#pragma unroll
    for (int c = 0; c < CW; ++c) accC[c] = 0;
    auto tile_ptr = [&](int J) -> const E * {
        const int64_t t = (J <= I) ? ((int64_t)I * (I + 1) / 2 + J) : ((int64_t)J * (J + 1) / 2 + I);
        return tiles + (toff + t) * (TILE * TILE) + (rg * RPT) * TILE + cg * CW;
    };
    Vec16 cur[RPT], nxt[RPT];
    {
        const E *tp = tile_ptr(0);
#pragma unroll
        for (int k = 0; k < RPT; ++k) cur[k] = *reinterpret_cast<const Vec16 *>(tp + k * TILE);
    }
    for (int J = 0; J < nt; ++J) {
        if (J + 1 < nt) {
            const E *tp = tile_ptr(J + 1);
#pragma unroll
            for (int k = 0; k < RPT; ++k) nxt[k] = *reinterpret_cast<const Vec16 *>(tp + k * TILE);
        }
        const A *xJ = xs + J * TILE;
        if (J <= I) {
            A xb[CW];
#pragma unroll
            for (int c = 0; c < CW; ++c) xb[c] = xJ[cg * CW + c];
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                A t[CW];
                unpack<E, CW>(cur[k], t);
#pragma unroll
                for (int c = 0; c < CW; ++c) accR[k] = fma(t[c], xb[c], accR[k]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                const A xa = xJ[rg * RPT + k];
                A t[CW];
                unpack<E, CW>(cur[k], t);
#pragma unroll
                for (int c = 0; c < CW; ++c) accC[c] = fma(t[c], xa, accC[c]);
            }
        }
        if (J + 1 < nt)
#pragma unroll
            for (int k = 0; k < RPT; ++k) cur[k] = nxt[k];
    }
    __syncthreads();  // scratch aliases xs
    A *sR = scratch, *sC = scratch + 256 * RPT;
#pragma unroll
    for (int k = 0; k < RPT; ++k) sR[(rg * NC + cg) * RPT + k] = accR[k];
#pragma unroll
    for (int c = 0; c < CW; ++c) sC[(rg * NC + cg) * CW + c] = accC[c];
    __syncthreads();
    if (tid < TILE) {
        const int a = tid;
        A y = 0;
        const int arg = a / RPT, ak = a % RPT;
        for (int c = 0; c < NC; ++c) y += sR[(arg * NC + c) * RPT + ak];
        const int acg = a / CW, ac = a % CW;
        for (int g = 0; g < RG; ++g) y += sC[(g * NC + acg) * CW + ac];
        yout[a] = y;
    }
    __syncthreads();
}

template <typename E>
__device__ inline void schwarz_item(const SchwarzArgs &a, const E *tiles, int s, int I, bool coarse,
                                    double *smem, double &y_out, int &out_idx_valid, int64_t &out_idx) {
    using A = typename AccT<E>::T;
    const int n = a.sys_n[s], nt = a.sys_nt[s];
    const int64_t toff = a.sys_toff[s];
    A *xs = reinterpret_cast<A *>(smem);
    __shared__ double yout_d[TILE];
    A *yout = reinterpret_cast<A *>(yout_d);
    const int nd = a.nd;
    int e0 = 0;
    if (!coarse) {
        e0 = a.sub_ptr[s];
        for (int t = threadIdx.x; t < nt * TILE; t += 256) {
            A v = 0;
            if (t < n) {
                const int le = t / nd, i = t - le * nd;
                v = (A)a.r[(int64_t)a.sub_elems[e0 + le] * nd + i];
            }
            xs[t] = v;
        }
    } else {
        for (int t = threadIdx.x; t < nt * TILE; t += 256) xs[t] = t < n ? (A)a.r0[t] : (A)0;
    }
    __syncthreads();
    tile_row_product<E>(tiles, toff, nt, I, xs, yout, xs);
    out_idx_valid = 0;
    if (threadIdx.x < TILE) {
        const int gi = I * TILE + threadIdx.x;
        if (gi < n) {
            y_out = (double)yout[threadIdx.x];
            out_idx_valid = 1;
            if (!coarse) {
                const int le = gi / nd, i = gi - le * nd;
                out_idx = (int64_t)a.sub_elems[e0 + le] * nd + i;
            } else {
                out_idx = gi;
            }
        }
    }
}

template <typename EL, typename EC>
__global__ __launch_bounds__(256) void k_schwarz(SchwarzArgs a) {
    if (a.mode != 0 && a.sc->done) return;
    extern __shared__ double smem[];
    const int item = blockIdx.x;
    const int s = a.item_sys[item], I = a.item_row[item];
    const bool coarse = s >= a.n_sub;
    double y = 0.0;
    int valid = 0;
    int64_t idx = 0;
    if (!coarse)
        schwarz_item<EL>(a, reinterpret_cast<const EL *>(a.tiles_local), s, I, false, smem, y, valid, idx);
    else
        schwarz_item<EC>(a, reinterpret_cast<const EC *>(a.tiles_coarse), s, I, true, smem, y, valid, idx);
    double part[1] = {0.0};
    if (valid) {
        if (!coarse) {
            a.z[idx] = y;
            part[0] = a.r[idx] * y;
        } else {
            a.z0[idx] = y;
            part[0] = a.r0[idx] * y;
        }
    }
    if (a.mode == 0) return;
    double tot[1];
    block_sum<1, 256>(part, tot);
    if (grid_sum<1, 256>(tot, a.red, tot) && threadIdx.x == 0) {
        DevScalars *sc = a.sc;
        const double rz = tot[0];
        if (!finite(rz)) {
            sc->status = ST_NONFINITE;
            sc->done = 1;
        } else if (!(rz > 0.0)) {
            sc->status = ST_BREAKDOWN;
            sc->done = 1;
        } else {
            sc->beta = (a.mode == 1) ? 0.0 : rz / sc->rz;
            sc->rz = rz;
        }
    }
}

// ---------------------------------------------------------------------------
// p = z + P z0 (+ beta p): prolongation of the coarse correction fused with
// the search-direction update.
template <int NQ>
__global__ __launch_bounds__(256) void k_pupdate(PupdateArgs a) {
    if (a.mode != 0 && a.sc->done) return;
    const int64_t n = a.n_elem * a.nd;
    const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (idx >= n) return;
    double zz = a.z[idx];
    if (NQ > 0) {
        const int64_t e = idx / a.nd;
        const double *z0 = a.z0 + (int64_t)a.elem_coarse[e] * NQ;
        const double *Pr = a.P + idx * NQ;
#pragma unroll
        for (int j = 0; j < NQ; ++j) zz = fma(Pr[j], z0[j], zz);
    }
    if (a.mode == 2) zz = fma(a.sc->beta, a.p[idx], zz);
    a.p[idx] = zz;
}

// ---------------------------------------------------------------------------
// Ionic model (Barreto-Cressman-type, five states n, h, K_o, Na_i, Ca_i).
__device__ inline double xexp(double x) {
    return fabs(x) < 1e-4 ? 1.0 + x * 0.5 + x * x / 12.0 : x / (1.0 - exp(-x));
}

__device__ inline void ionic_model(double V, const double *y, const double *prm, double &f, double *dy,
                                   int &bad) {
    const double n = y[0], h = y[1], ko = y[2], nai = y[3], cai = y[4];
    const double ki = prm[21] + (prm[22] - nai);
    const double nao = prm[23] - prm[10] * (nai - prm[22]);
    if (!(ko > 0.0) || !(nai > 0.0) || !(ki > 0.0) || !(nao > 0.0)) {
        bad = 1;
        f = 0.0;
        if (dy)
            for (int l = 0; l < 5; ++l) dy[l] = 0.0;
        return;
    }
    const double vna = prm[17] * log(nao / nai);
    const double vk = prm[17] * log(ko / ki);
    const double vcl = prm[17] * log(prm[15] / prm[16]);
    const double am = xexp(0.1 * (V + 30.0));
    const double bm = 4.0 * exp(-(V + 55.0) / 18.0);
    const double an = 0.1 * xexp(0.1 * (V + 34.0));
    const double bn = 0.125 * exp(-(V + 44.0) / 80.0);
    const double ah = 0.07 * exp(-(V + 44.0) / 20.0);
    const double bh = 1.0 / (1.0 + exp(-(V + 14.0) / 10.0));
    const double minf = am / (am + bm);
    const double ina = -prm[0] * minf * minf * minf * h * (V - vna) - prm[1] * (V - vna);
    const double n2 = n * n;
    const double ik = -(prm[2] * n2 * n2 + prm[4] * cai / (1.0 + cai)) * (V - vk) - prm[3] * (V - vk);
    const double icl = -prm[5] * (V - vcl);
    f = -(ina + ik + icl);
    if (dy) {
        const double ipump = prm[11] / (1.0 + exp((25.0 - nai) / 3.0)) / (1.0 + exp(5.5 - ko));
        const double iglia = prm[12] / (1.0 + exp((18.0 - ko) / 2.5));
        const double idiff = prm[13] * (ko - prm[14]);
        dy[0] = prm[8] * (an * (1.0 - n) - bn * n);
        dy[1] = prm[8] * (ah * (1.0 - h) - bh * h);
        dy[2] = (-prm[18] * ik - 2.0 * prm[10] * ipump - iglia - idiff) / prm[9];
        dy[3] = (prm[18] * ina / prm[10] - 3.0 * ipump) / prm[9];
        dy[4] = -prm[20] * prm[6] * (V - prm[7]) / (1.0 + exp(-(V + 25.0) / 2.5)) - cai / prm[19];
    }
}

// modal basis at a reference point (Legendre products, total degree <= P;
// total degree ascending, alpha_1 descending, alpha_2 descending)
template <int DIM, int P>
__device__ inline void basis_at(const double *xi, const double *nrm, double *phi) {
    double L[DIM][P + 1];
#pragma unroll
    for (int j = 0; j < DIM; ++j) {
        const double t = xi[j];
        L[j][0] = 1.0;
        if (P >= 1) L[j][1] = t;
#pragma unroll
        for (int k = 1; k < P; ++k) L[j][k + 1] = ((2.0 * k + 1.0) * t * L[j][k] - k * L[j][k - 1]) / (k + 1.0);
    }
    int b = 0;
#pragma unroll
    for (int deg = 0; deg <= P; ++deg)
#pragma unroll
        for (int a1 = deg; a1 >= 0; --a1) {
            if (DIM == 2) {
                phi[b] = nrm[b] * L[0][a1] * L[1][deg - a1];
                ++b;
            } else {
#pragma unroll
                for (int a2 = deg - a1; a2 >= 0; --a2) {
                    phi[b] = nrm[b] * L[0][a1] * L[1][a2] * L[DIM - 1][deg - a1 - a2];
                    ++b;
                }
            }
        }
}

template <int DIM, int P>
struct NB { static constexpr int v = DIM == 2 ? (P + 1) * (P + 2) / 2 : (P + 1) * (P + 2) * (P + 3) / 6; };

// One wavefront per element.  Pass 1: G_l = int m_l(u^k, y^k) phi and
// Y^(k+1) = Y^k - dt M^{-1} G (second line of eq. (4)).  Pass 2: the ion term
// I = int f(u~, y^(k+1)) phi with u~ = (3 u^k - u^(k-1)) / 2.
template <int DIM, int P>
__global__ __launch_bounds__(64) void k_ionic(IonicArgs a) {
    constexpr int ND = NB<DIM, P>::v;
    const int64_t e = blockIdx.x;
    const int lane = threadIdx.x;
    __shared__ double s_phi[64][ND + 1];
    __shared__ double s_w[64][6];
    __shared__ double s_u[ND], s_up[ND], s_y[5][ND], s_g[5][ND], s_nrm[ND];
    __shared__ double s_prm[24];
    __shared__ int s_bad;
    const int64_t n = a.n_elem;
    if (lane == 0) s_bad = 0;
    if (lane < 24) s_prm[lane] = a.prm[lane];
    for (int k = lane; k < ND; k += 64) {
        s_u[k] = a.u[e * ND + k];
        s_up[k] = a.u_prev[e * ND + k];
        s_nrm[k] = a.norm[e * ND + k];
    }
    for (int k = lane; k < 5 * ND; k += 64) {
        const int l = k / ND, i = k - l * ND;
        s_y[l][i] = a.y[((int64_t)l * n + e) * ND + i];
    }
    __syncthreads();
    const int64_t q0 = a.qp_ptr[e], q1 = a.qp_ptr[e + 1];
    constexpr int NOUT = (5 * ND + 63) / 64;
    double accG[NOUT];
#pragma unroll
    for (int t = 0; t < NOUT; ++t) accG[t] = 0.0;
    int bad = 0;
    for (int64_t c0 = q0; c0 < q1; c0 += 64) {
        const int64_t q = c0 + lane;
        double phi[ND];
        if (q < q1) {
            double xi[DIM];
#pragma unroll
            for (int d = 0; d < DIM; ++d) xi[d] = a.qp_xi[q * DIM + d];
            basis_at<DIM, P>(xi, s_nrm, phi);
            double u = 0.0, yv[5] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                u = fma(phi[k], s_u[k], u);
#pragma unroll
                for (int l = 0; l < 5; ++l) yv[l] = fma(phi[k], s_y[l][k], yv[l]);
            }
            double f, dy[5];
            ionic_model(u, yv, s_prm, f, dy, bad);
            const double w = a.qp_w[q];
#pragma unroll
            for (int l = 0; l < 5; ++l) s_w[lane][l] = w * dy[l];
#pragma unroll
            for (int k = 0; k < ND; ++k) s_phi[lane][k] = phi[k];
        } else {
#pragma unroll
            for (int l = 0; l < 5; ++l) s_w[lane][l] = 0.0;
#pragma unroll
            for (int k = 0; k < ND; ++k) s_phi[lane][k] = 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int t = 0; t < NOUT; ++t) {
            const int o = lane + 64 * t;
            if (o < 5 * ND) {
                const int l = o / ND, k = o - l * ND;
                double s = accG[t];
                for (int qq = 0; qq < 64; ++qq) s = fma(s_w[qq][l], s_phi[qq][k], s);
                accG[t] = s;
            }
        }
        __syncthreads();
    }
    // integral of dy/dt phi = -G; Y^(k+1) = Y^k + dt M^{-1} int(dy/dt phi)
#pragma unroll
    for (int t = 0; t < NOUT; ++t) {
        const int o = lane + 64 * t;
        if (o < 5 * ND) s_g[o / ND][o % ND] = accG[t];
    }
    __syncthreads();
    const double *Mi = a.minv + e * ND * ND;
    double ynew[NOUT];
#pragma unroll
    for (int t = 0; t < NOUT; ++t) {
        const int o = lane + 64 * t;
        ynew[t] = 0.0;
        if (o < 5 * ND) {
            const int l = o / ND, i = o - l * ND;
            double s = 0.0;
            for (int j = 0; j < ND; ++j) s = fma(Mi[i * ND + j], s_g[l][j], s);
            ynew[t] = s_y[l][i] + a.dt * s;
        }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < NOUT; ++t) {
        const int o = lane + 64 * t;
        if (o < 5 * ND) {
            const int l = o / ND, i = o - l * ND;
            s_y[l][i] = ynew[t];
            a.y[((int64_t)l * n + e) * ND + i] = ynew[t];
        }
    }
    __syncthreads();
    double accI = 0.0;
    for (int64_t c0 = q0; c0 < q1; c0 += 64) {
        const int64_t q = c0 + lane;
        if (q < q1) {
            double xi[DIM], phi[ND];
#pragma unroll
            for (int d = 0; d < DIM; ++d) xi[d] = a.qp_xi[q * DIM + d];
            basis_at<DIM, P>(xi, s_nrm, phi);
            double u = 0.0, up = 0.0, yv[5] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < ND; ++k) {
                u = fma(phi[k], s_u[k], u);
                up = fma(phi[k], s_up[k], up);
#pragma unroll
                for (int l = 0; l < 5; ++l) yv[l] = fma(phi[k], s_y[l][k], yv[l]);
            }
            double f;
            ionic_model(1.5 * u - 0.5 * up, yv, s_prm, f, nullptr, bad);
            s_w[lane][0] = a.qp_w[q] * f;
#pragma unroll
            for (int k = 0; k < ND; ++k) s_phi[lane][k] = phi[k];
        } else {
            s_w[lane][0] = 0.0;
#pragma unroll
            for (int k = 0; k < ND; ++k) s_phi[lane][k] = 0.0;
        }
        __syncthreads();
        if (lane < ND)
            for (int qq = 0; qq < 64; ++qq) accI = fma(s_w[qq][0], s_phi[qq][lane], accI);
        __syncthreads();
    }
    if (lane < ND) a.I[e * ND + lane] = accI;
    if (bad) s_bad = 1;
    __syncthreads();
    if (lane == 0 && s_bad) a.sc->ionic_bad = 1;
}

// ---------------------------------------------------------------------------
__global__ void k_project_p0(const double *vals, int ncomp, int64_t n_elem, int nd, const double *norm,
                             double *coeff) {
    const int64_t total = (int64_t)ncomp * n_elem * nd;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t ce = t / nd;
        const int k = (int)(t - ce * nd);
        const int64_t e = ce % n_elem;
        // the constant 1 equals phi_0 / norm_0 on the element (phi_0 is constant)
        coeff[t] = (k == 0) ? vals[ce] / norm[e * nd] : 0.0;
    }
}

__global__ void k_zero(double *x, int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        x[t] = 0.0;
}

__global__ void k_status_reset(DevScalars *sc, double tol2, int maxit, int reset_ionic) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (reset_ionic) sc->ionic_bad = 0;
        sc->bb = sc->rr = sc->rz = sc->pq = sc->alpha = sc->beta = sc->tr = 0.0;
        sc->tol2 = tol2;
        sc->done = 0;
        sc->status = ST_RUN;
        sc->iters = 0;
        sc->maxit = maxit;
    }
}

// ---------------------------------------------------------------------------
// launchers
constexpr int kSpmvWPB = 2;

int spmv_blocks(const DevMatrix &A) { return (int)((A.n_groups + kSpmvWPB - 1) / kSpmvWPB); }

template <int ND>
static hipError_t spmv_nd(const DevMatrix &A, const SpmvArgs &a, hipStream_t s) {
    hipLaunchKernelGGL((k_spmv<ND, kSpmvWPB>), dim3(spmv_blocks(A)), dim3(64 * kSpmvWPB), 0, s, A, a);
    return hipGetLastError();
}

hipError_t launch_spmv(const DevMatrix &A, const SpmvArgs &a, hipStream_t s) {
    switch (A.nd) {
    case 3: return spmv_nd<3>(A, a, s);
    case 4: return spmv_nd<4>(A, a, s);
    case 6: return spmv_nd<6>(A, a, s);
    case 10: return spmv_nd<10>(A, a, s);
    case 15: return spmv_nd<15>(A, a, s);
    case 20: return spmv_nd<20>(A, a, s);
    case 35: return spmv_nd<35>(A, a, s);
    }
    return hipErrorInvalidValue;
}

template <int ND>
static hipError_t update_nd(const UpdateArgs &a, hipStream_t s) {
    switch (a.nq0) {
    case 0: hipLaunchKernelGGL((k_update<ND, 0>), dim3(a.n_grp), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_update<ND, 3>), dim3(a.n_grp), dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_update<ND, 4>), dim3(a.n_grp), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_update(const UpdateArgs &a, hipStream_t s) {
    switch (a.nd) {
    case 3: return update_nd<3>(a, s);
    case 4: return update_nd<4>(a, s);
    case 6: return update_nd<6>(a, s);
    case 10: return update_nd<10>(a, s);
    case 15: return update_nd<15>(a, s);
    case 20: return update_nd<20>(a, s);
    case 35: return update_nd<35>(a, s);
    }
    return hipErrorInvalidValue;
}

template <typename E> static constexpr size_t acc_size() { return sizeof(typename AccT<E>::T); }
template <typename E> static constexpr size_t scratch_bytes() {
    constexpr int CW = 16 / sizeof(E), NC = TILE / CW, RG = 256 / NC, RPT = TILE / RG;
    return (size_t)256 * (RPT + CW) * acc_size<E>();
}

template <typename EL, typename EC>
static hipError_t schwarz_t(const SchwarzArgs &a, int n_items, int max_n, hipStream_t s) {
    const size_t nt_max = (size_t)(max_n + TILE - 1) / TILE;
    size_t bytes = nt_max * TILE * (acc_size<EL>() > acc_size<EC>() ? acc_size<EL>() : acc_size<EC>());
    const size_t sb = scratch_bytes<EL>() > scratch_bytes<EC>() ? scratch_bytes<EL>() : scratch_bytes<EC>();
    if (bytes < sb) bytes = sb;
    hipLaunchKernelGGL((k_schwarz<EL, EC>), dim3(n_items), dim3(256), bytes, s, a);
    return hipGetLastError();
}

hipError_t launch_schwarz(const SchwarzArgs &a, int n_items, int local_store, int coarse_store, int max_n,
                          hipStream_t s) {
    if (n_items <= 0) return hipSuccess;
    if (coarse_store == STORE_F64) {
        switch (local_store) {
        case STORE_F64: return schwarz_t<double, double>(a, n_items, max_n, s);
        case STORE_F32: return schwarz_t<float, double>(a, n_items, max_n, s);
        case STORE_BF16: return schwarz_t<uint16_t, double>(a, n_items, max_n, s);
        }
    } else {
        switch (local_store) {
        case STORE_F64: return schwarz_t<double, float>(a, n_items, max_n, s);
        case STORE_F32: return schwarz_t<float, float>(a, n_items, max_n, s);
        case STORE_BF16: return schwarz_t<uint16_t, float>(a, n_items, max_n, s);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_pupdate(const PupdateArgs &a, hipStream_t s) {
    const int blocks = (int)((a.n_elem * a.nd + 255) / 256);
    switch (a.nq0) {
    case 0: hipLaunchKernelGGL((k_pupdate<0>), dim3(blocks), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_pupdate<3>), dim3(blocks), dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_pupdate<4>), dim3(blocks), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ionic(const IonicArgs &a, hipStream_t s) {
    const dim3 g((unsigned)a.n_elem), b(64);
#define PDG_IONIC(D, P)                                                  \
    if (a.dim == D && a.p == P) {                                        \
        hipLaunchKernelGGL((k_ionic<D, P>), g, b, 0, s, a);              \
        return hipGetLastError();                                        \
    }
    PDG_IONIC(2, 1) PDG_IONIC(2, 2) PDG_IONIC(2, 3) PDG_IONIC(2, 4)
    PDG_IONIC(3, 1) PDG_IONIC(3, 2) PDG_IONIC(3, 3) PDG_IONIC(3, 4)
#undef PDG_IONIC
    return hipErrorInvalidValue;
}

hipError_t launch_project_p0(const double *vals, int ncomp, int64_t n_elem, int nd, const double *norm,
                             double *coeff, hipStream_t s) {
    const int64_t total = (int64_t)ncomp * n_elem * nd;
    const int blocks = (int)((total + 255) / 256 < 65536 ? (total + 255) / 256 : 65536);
    hipLaunchKernelGGL(k_project_p0, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, vals, ncomp, n_elem, nd,
                       norm, coeff);
    return hipGetLastError();
}

hipError_t launch_zero(double *x, int64_t n, hipStream_t s) {
    const int blocks = (int)((n + 255) / 256 < 65536 ? (n + 255) / 256 : 65536);
    hipLaunchKernelGGL(k_zero, dim3(blocks > 0 ? blocks : 1), dim3(256), 0, s, x, n);
    return hipGetLastError();
}

hipError_t launch_status_reset(DevScalars *sc, double tol2, int maxit, int reset_ionic, hipStream_t s) {
    hipLaunchKernelGGL(k_status_reset, dim3(1), dim3(64), 0, s, sc, tol2, maxit, reset_ionic);
    return hipGetLastError();
}

}  // namespace pdg
