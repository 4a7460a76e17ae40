// HIP kernels of libpdg for gfx950 (CDNA4, wave64).
//
// Per PCG iteration (Section 4: PCG with the additive Schwarz operator of
// eq. (5)) the stream runs four kernels:
//   k_spmv   (mode PQ)  q = K p, per-workgroup partials of (p, q)
//   k_update            alpha = (r, z) / (p, q); x += alpha p, r -= alpha q;
//                       per-chunk ||r||^2 and coarse restriction shares of P^T r
//   k_schwarz           partial products of z_i = K_i^{-1} r_i (all subdomains)
//                       and z0 = K_0^{-1} r0, with their shares of (r, z)
//   k_pupdate           z = B r assembled, beta = (r, z)' / (r, z), p = z + beta p,
//                       convergence test on ||r||^2
// A launch serves a batch of independent systems: every workgroup belongs to
// one system (the p-update kernel's dof blocks may touch several and handle
// each in turn), reads that system's device scalars and returns at once when
// the system has stopped.  No kernel synchronises workgroups with atomics or
// device-scope fences (on gfx950 a device-scope release fence writes back the
// L2 and costs tens of ns per workgroup).  Instead every kernel writes
// per-workgroup partial sums and the next kernel, after the kernel boundary,
// adds the partials of its system in a fixed order in each of its workgroups.
// All sums therefore have a fixed order and two runs give bitwise-equal
// results; a system gives the same bits alone or inside a batch.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <type_traits>

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

// Block totals of v, returned in every thread.
template <int NV, int BS>
__device__ inline void block_sum(double (&v)[NV], double (&tot)[NV]) {
    __shared__ double sh[BS / 64][NV];
    wave_sum<NV>(v);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh[w][k] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int ww = 0; ww < BS / 64; ++ww) s += sh[ww][k];
        tot[k] = s;
    }
    __syncthreads();
}

// This thread's share of the sum of part[k * stride + slot], k < n: the
// entries k = threadIdx.x + m * BS, loaded 16 per round (those past n read
// nothing) so that one memory round trip covers up to 16 * BS partials, and
// added into four running sums in a fixed order.
template <int BS>
__device__ inline double thread_sum_partials(const double *part, int n, int stride, int slot) {
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = threadIdx.x; k0 < n; k0 += 16 * BS) {
        double w[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int k = k0 + u * BS;
            w[u] = k < n ? part[(int64_t)k * stride + slot] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) acc[u & 3] += w[u];
    }
    return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

// Block total of one value per thread, in every thread.
template <int BS>
__device__ inline double block_total(double v) {
    double w[1] = {v}, t[1];
    block_sum<1, BS>(w, t);
    return t[0];
}

// Sum of part[k * stride + slot], k < n, in a fixed order, in every thread.
template <int BS>
__device__ inline double block_sum_partials(const double *part, int n, int stride, int slot) {
    return block_total<BS>(thread_sum_partials<BS>(part, n, stride, slot));
}

__device__ inline bool finite(double x) { return __builtin_isfinite(x); }

// Thread 0's value of v in every thread of the block.  Used for flags that
// another workgroup of the same launch may write, so that all wavefronts of a
// block take the same branch around its barriers.
template <int BS>
__device__ inline int block_bcast(int v) {
    __shared__ int s;
    if (threadIdx.x == 0) s = v;
    __syncthreads();
    const int r = s;
    __syncthreads();
    return r;
}

// Entry i of output row `row` for the launch mode, given acc = (K x)_row,i;
// adds the entry's share of the mode's dot products to part.
template <int ND>
__device__ inline void spmv_out(const DevMatrix &A, const SpmvArgs &a, int row, int i, double acc,
                                double (&part)[2]) {
    const int64_t idx = (int64_t)row * ND + i;
    switch (a.mode) {
    case SPMV_PLAIN:
        a.y[idx] = acc;
        break;
    case SPMV_PQ:
        a.y[idx] = acc;
        part[0] = fma(a.x[idx], acc, part[0]);
        break;
    case SPMV_RESID: {
        const double bv = a.b[idx], rv = bv - acc;
        a.y[idx] = rv;
        if (a.xcopy) a.xcopy[idx] = a.x[idx];
        if (a.u_prev) a.u_prev[idx] = a.x[idx];
        part[0] = fma(bv, bv, part[0]);
        part[1] = fma(rv, rv, part[1]);
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
            if (a.xcopy) a.xcopy[idx] = ur[i];
            part[0] = fma(bv, bv, part[0]);
        }
        break;
    }
    }
}

// ---------------------------------------------------------------------------
// Block-sparse SpMV over element rows in interleaved group-ELL form.
// G = 64 / ND element rows form a group; lane (r, i) = (lane / ND, lane % ND)
// owns output row i of the group's r-th element.  Group values are stored
// slot-major so that for every (slot s, trial index j) a wavefront reads G*ND
// consecutive doubles:  val[((s * ND + j) * G + r) * ND + i] = K_{row_r, col_{s,r}}[i][j].
// A workgroup owns a contiguous run of groups (of one system) and writes one
// partial sum; its WPG wavefronts take each group's slots round-robin and
// their sums are added in wave order through LDS (double-buffered, one
// barrier per group).
// Matrices larger than the last-level cache stream their values with
// non-temporal loads (NT), smaller ones stay cacheable across iterations.
template <int ND, int WPG, bool NT>
__global__ __launch_bounds__(64 * WPG) void k_spmv(DevMatrix A, SpmvArgs a) {
    constexpr int G = ND <= 64 ? 64 / ND : 1;
    // the workgroup's record (and, in a one-system context, the stop flag)
    // first: one memory round trip before the first slot's loads
    const SpDesc dsc = A.wg_desc[blockIdx.x];
    const int64_t g_begin = dsc.g_begin, g_end = dsc.g_end;
    if (a.mode == SPMV_PQ) {
        int32_t done;
        if (A.one_sys) done = a.sc[0].done;
        else done = a.sc[dsc.sys].done;
        if (done) return;
    }
    __shared__ double s_acc[2][WPG][64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int r = lane / ND, i = lane - (lane / ND) * ND;
    // U slots per loop trip, all of their loads issued before the first
    // multiply, so a wavefront keeps U slots of the matrix in flight
    constexpr int U = ND <= 6 ? 4 : (ND <= 10 ? 2 : 1);
    double part[2] = {0.0, 0.0};
    int par = 0;
    for (int64_t g = g_begin; g < g_end; ++g) {
        double acc = 0.0;
        // the output row, requested before the products
        const int row = (w == 0 && r < G) ? A.grp_rows[g * G + r] : -1;
        if (r < G) {
            const int64_t s0 = g == g_begin ? dsc.s0 : A.grp_slot_off[g];
            const int64_t ns = (g == g_begin ? dsc.s1 : A.grp_slot_off[g + 1]) - s0;
            const int32_t *colp = A.grp_col + s0 * G + r;
            const double *vp = A.grp_val + s0 * G * ND * ND + lane;
            double accu[U];
#pragma unroll
            for (int u = 0; u < U; ++u) accu[u] = 0.0;
            for (int64_t s = w; s < ns; s += U * WPG) {
                int c[U];
                double v[U][ND];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int64_t su = s + u * WPG;
                    c[u] = su < ns ? colp[su * G] : -1;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const double *vs = vp + (s + u * WPG) * G * ND * ND;
#pragma unroll
                    for (int j = 0; j < ND; ++j)
                        v[u][j] = c[u] >= 0 ? (NT ? __builtin_nontemporal_load(vs + j * G * ND) : vs[j * G * ND]) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (c[u] < 0) continue;
                    const double *xb = a.x + (int64_t)c[u] * ND;
#pragma unroll
                    for (int j = 0; j < ND; ++j) accu[u] = fma(v[u][j], xb[j], accu[u]);
                }
            }
            acc = accu[0];
#pragma unroll
            for (int u = 1; u < U; ++u) acc += accu[u];
        }
        if (WPG > 1) {
            s_acc[par][w][lane] = acc;
            __syncthreads();
            if (w == 0) {
                acc = s_acc[par][0][lane];
#pragma unroll
                for (int k = 1; k < WPG; ++k) acc += s_acc[par][k][lane];
            }
            par ^= 1;
        }
        if (w != 0) continue;  // wave 0 finishes the group
        if (row < 0) continue;
        spmv_out<ND>(A, a, row, i, acc, part);
    }
    if (w != 0 || a.mode == SPMV_PLAIN || a.mode == SPMV_RHS) return;
    wave_sum<2>(part);
    if (lane == 0) {
        a.part[2 * blockIdx.x] = part[0];
        a.part[2 * blockIdx.x + 1] = part[1];
    }
}

// Blocks of more than 32 rows (3-D, p = 4: nd = 35) give one element row per
// group, and the mapping above would leave 29 of 64 lanes idle.  Here the
// (slot, row) pairs of a chunk of the group's blocks are laid end to end and
// each lane takes one pair per step; the chunk is stored trial-index major
// (kWideChunk), so for every trial index j a wavefront's load reads 64
// consecutive doubles.  Each pair's dot product goes to LDS, and lane i of
// wave 0 adds row i's products in slot order, so the result does not depend
// on WPG.
template <int ND, int WPG, bool NT>
__global__ __launch_bounds__(64 * WPG) void k_spmv_wide(DevMatrix A, SpmvArgs a) {
    static_assert(ND >= kWideMinNd, "chunked layout is built for nd >= kWideMinNd only");
    constexpr int CH = kWideChunk;  // slots per chunk (and per LDS pass)
    constexpr int T = CH * ND;
    constexpr int STEPS = (T + 63) / 64;
    __shared__ double s_p[T];
    const SpDesc dsc = A.wg_desc[blockIdx.x];
    const int64_t g_begin = dsc.g_begin, g_end = dsc.g_end;
    if (a.mode == SPMV_PQ) {
        int32_t done;
        if (A.one_sys) done = a.sc[0].done;
        else done = a.sc[dsc.sys].done;
        if (done) return;
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double part[2] = {0.0, 0.0};
    for (int64_t g = g_begin; g < g_end; ++g) {
        const int64_t s0 = g == g_begin ? dsc.s0 : A.grp_slot_off[g];
        const int64_t ns = (g == g_begin ? dsc.s1 : A.grp_slot_off[g + 1]) - s0;
        const int row = (w == 0 && lane < ND) ? A.grp_rows[g] : -1;
        const int32_t *colp = A.grp_col + s0;
        const double *vp = A.grp_val + s0 * ND * ND;
        double acc = 0.0;
        for (int64_t c0 = 0; c0 < ns; c0 += CH) {
            const int nch = (int)(ns - c0 < CH ? ns - c0 : CH);
            const int tn = nch * ND;
            for (int k = w; k < STEPS; k += WPG) {
                const int t = k * 64 + lane;
                if (t >= tn) continue;
                const int sl = t / ND, i = t - sl * ND;
                const int col = colp[c0 + sl];
                double sum = 0.0;
                if (col >= 0) {
                    const double *vs = vp + c0 * ND * ND + t;
                    const double *xb = a.x + (int64_t)col * ND;
                    double v[ND];
#pragma unroll
                    for (int j = 0; j < ND; ++j) v[j] = NT ? __builtin_nontemporal_load(vs + j * tn) : vs[j * tn];
#pragma unroll
                    for (int j = 0; j < ND; ++j) sum = fma(v[j], xb[j], sum);
                }
                s_p[t] = sum;
            }
            __syncthreads();
            if (w == 0 && lane < ND)
                for (int sl = 0; sl < nch; ++sl) acc += s_p[sl * ND + lane];
            __syncthreads();
        }
        if (w != 0 || lane >= ND) continue;
        if (row >= 0) spmv_out<ND>(A, a, row, lane, acc, part);
    }
    if (w != 0 || a.mode == SPMV_PLAIN || a.mode == SPMV_RHS) return;
    wave_sum<2>(part);
    if (lane == 0) {
        a.part[2 * blockIdx.x] = part[0];
        a.part[2 * blockIdx.x + 1] = part[1];
    }
}

// ---------------------------------------------------------------------------
// alpha = (r, z) / (p, q); x += alpha p, r -= alpha q; ||r||^2 and the coarse
// restriction shares of P^T r.  A workgroup owns a contiguous run of update
// chunks (runs of elements inside one coarse element, all of one system):
// it writes one ||r||^2 partial and, per chunk, the chunk's restriction
// share, which the Schwarz kernel adds in chunk order when it gathers r0.
template <int ND, int NQ>
__global__ __launch_bounds__(128) void k_update(UpdateArgs a) {
    const int wg = blockIdx.x;
    // the workgroup's record first (one load): chunks, system, SpMV
    // partials and the first chunk's elements
    const UpdDesc dsc = a.wg_desc[wg];
    const int c_begin = dsc.c_begin, c_end = dsc.c_end;
    const int b = dsc.b;
    DevScalars *sc = a.sc + b;
    constexpr int NV = NQ > 0 ? NQ : 1;
    // The thread's first dof (usually its only one) is read before the
    // reductions below, which do not change it, so the latencies overlap.
    const int f_e0 = dsc.f_e0, f_n = dsc.f_n * ND;
    const bool f_has = (int)threadIdx.x < f_n;
    int64_t f_idx = 0;
    double f_r = 0.0, f_p = 0.0, f_q = 0.0, f_x = 0.0, f_P[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) f_P[k] = 0.0;
    if (f_has) {
        const int le = threadIdx.x / ND, i = threadIdx.x - le * ND;
        f_idx = (int64_t)(dsc.e_first >= 0 ? dsc.e_first + le : a.grp_elems[f_e0 + le]) * ND + i;
        f_r = a.r[f_idx];
        if (!a.init) {
            f_p = a.p[f_idx];
            f_q = a.q[f_idx];
            f_x = a.x[f_idx];
        }
        if (NQ > 0)
#pragma unroll
            for (int j = 0; j < NQ; ++j) f_P[j] = a.P[f_idx * NQ + j];
    }
    // The stop flag, the scalars and this thread's share of the (p, q)
    // partials are requested together with the dof above, before the first
    // barrier.
    const int done = threadIdx.x == 0 ? sc->done : 0;
    const int iters = sc->iters;
    const double rz_even = sc->rz[0], rz_odd = sc->rz[1];
    const double pq_t =
        (a.init || a.pre_pq) ? 0.0 : thread_sum_partials<128>(a.pqpart + 2 * (int64_t)dsc.g0, dsc.g1 - dsc.g0, 2, 0);
    // the owner workgroup may set `done` during this launch
    if (block_bcast<128>(done)) return;
    double alpha = 0.0;
    if (!a.init) {
        const double pq = a.pre_pq ? sc->pq_sum : block_total<128>(pq_t);
        const int j = iters + 1;
        alpha = ((j - 1) & 1 ? rz_odd : rz_even) / pq;
        if (wg == a.rng.upd[b] && threadIdx.x == 0) {
            sc->pq = pq;
            sc->alpha = alpha;
            sc->jcur = j;
            if (a.lanczos && j <= a.lcap) a.lanczos[(int64_t)b * a.lcap + j - 1].x = alpha;
            if (!finite(pq)) {
                sc->status = ST_NONFINITE;
                sc->done = 1;
            } else if (!(pq > 0.0)) {
                sc->status = ST_BREAKDOWN;
                sc->done = 1;
            }
        }
    }
    double rr = 0.0;
    for (int c = c_begin; c < c_end; ++c) {
        const bool first_c = c == c_begin;
        const int e0 = first_c ? f_e0 : a.grp_ptr[c];
        const int ndof = first_c ? f_n : (a.grp_ptr[c + 1] - e0) * ND;
        const int e_first = first_c ? dsc.e_first : -1;
        double v[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = 0.0;
        for (int d = threadIdx.x; d < ndof; d += 128) {
            const bool first = c == c_begin && d == (int)threadIdx.x;
            int64_t idx;
            double rv, pv = 0.0, qv = 0.0, xv = 0.0, Pr[NV];
            if (first) {
                idx = f_idx;
                rv = f_r;
                pv = f_p;
                qv = f_q;
                xv = f_x;
#pragma unroll
                for (int j = 0; j < NV; ++j) Pr[j] = f_P[j];
            } else {
                const int le = d / ND, i = d - le * ND;
                idx = (int64_t)(e_first >= 0 ? e_first + le : a.grp_elems[e0 + le]) * ND + i;
                rv = a.r[idx];
                if (!a.init) {
                    pv = a.p[idx];
                    qv = a.q[idx];
                    xv = a.x[idx];
                }
                if (NQ > 0)
#pragma unroll
                    for (int j = 0; j < NQ; ++j) Pr[j] = a.P[idx * NQ + j];
            }
            if (!a.init) {
                a.x[idx] = fma(alpha, pv, xv);
                rv = fma(-alpha, qv, rv);
                a.r[idx] = rv;
            }
            rr = fma(rv, rv, rr);
            if (NQ > 0) {
#pragma unroll
                for (int j = 0; j < NQ; ++j) v[j] = fma(Pr[j], rv, v[j]);
            }
        }
        if (NQ > 0) {
            if (c + 1 == c_end) {
                // the last chunk's shares and the workgroup's ||r||^2 in one
                // reduction (each component is summed as it would be alone)
                double vv[NV + 1], tot[NV + 1];
#pragma unroll
                for (int j = 0; j < NV; ++j) vv[j] = v[j];
                vv[NV] = rr;
                block_sum<NV + 1, 128>(vv, tot);
                if (threadIdx.x == 0) {
#pragma unroll
                    for (int j = 0; j < NQ; ++j) a.r0part[c * NQ + j] = tot[j];
                    a.rrpart[wg] = tot[NV];
                }
            } else {
                double tot[NV];
                block_sum<NV, 128>(v, tot);
                if (threadIdx.x == 0)
#pragma unroll
                    for (int j = 0; j < NQ; ++j) a.r0part[c * NQ + j] = tot[j];
            }
        }
    }
    if (NQ == 0 || c_begin == c_end) {
        double v1[1] = {rr}, t1[1];
        block_sum<1, 128>(v1, t1);
        if (threadIdx.x == 0) a.rrpart[wg] = t1[0];
    }
}

// ---------------------------------------------------------------------------
// Schwarz apply: z_i = K_i^{-1} r_i for every subdomain and z0 = K_0^{-1} r0.
// Each inverse is symmetric and stored as packed lower-triangular 64x64 tiles
// (row-major inside a tile).  A workgroup (256 threads) owns one work item:
// the stored tiles (I, J), J in [j0, j0 + nj), of one packed tile row I of
// one system; each tile is read once and used for both of its products
// (see schwarz_item).  Each thread loads 16 bytes (8 for BF16) per tile row for RPT rows,
// so every load instruction of a wavefront reads whole contiguous tile rows.
// Items hold ~128 KiB of tiles by default, so the grid is many similar-sized
// workgroups.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename E> struct AccT { using T = float; };
template <> struct AccT<double> { using T = double; };

// Storage type of the row and column partials: FP32 when every item of the
// launch accumulates in FP32 (local and coarse store both below FP64), which
// halves the bytes the apply writes; FP64 otherwise.
template <typename EL, typename EC> struct PartT { using T = double; };
template <> struct PartT<float, float> { using T = float; };
template <> struct PartT<uint16_t, float> { using T = float; };

// Load type per storage type; element c of a loaded vector as the
// accumulation type.
template <typename E> struct Ld;
template <> struct Ld<double> {
    using V = double2;
    static __device__ inline double get(const V &v, int c) { return c == 0 ? v.x : v.y; }
};
template <> struct Ld<float> {
    using V = float4;
    static __device__ inline float get(const V &v, int c) {
        return c == 0 ? v.x : (c == 1 ? v.y : (c == 2 ? v.z : v.w));
    }
};
// BF16 tiles are read 8 bytes (4 columns) per lane: with 16 columns per row
// group the column sums need one shuffle round fewer, and 4 columns instead
// of 8 per round, than with 16-byte loads.
template <> struct Ld<uint16_t> {
    using V = uint2;
    static __device__ inline float get(const V &v, int c) {
        const uint32_t w = (c >> 1) == 0 ? v.x : v.y;
        return __uint_as_float((c & 1) ? (w & 0xffff0000u) : (w << 16));
    }
};

// Bytes one lane loads per tile row piece, and the columns they hold.
template <typename E> struct Piece { static constexpr int bytes = 16; };
template <> struct Piece<uint16_t> { static constexpr int bytes = 8; };
template <typename E> __device__ inline typename Ld<E>::V load_piece(const E *p) {
    using V = typename Ld<E>::V;
    typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
    if constexpr (Piece<E>::bytes == 16)
        return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p)));
    else
        return __builtin_bit_cast(V, __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p)));
}

// Multiply-accumulate of one 64x64 tile held in registers (RPT rows of CW
// columns per thread): tile (I, J) as stored (J <= I) or transposed (J > I).
template <typename E, int CW, int RPT>
__device__ inline void tile_mac(const typename Ld<E>::V (&tv)[RPT], bool stored, const typename AccT<E>::T *xJ,
                                int cg, int rg, typename AccT<E>::T (&accR)[RPT],
                                typename AccT<E>::T (&accC)[CW]) {
    using A = typename AccT<E>::T;
    if (stored) {
        A xb[CW];
#pragma unroll
        for (int c = 0; c < CW; ++c) xb[c] = xJ[cg * CW + c];
#pragma unroll
        for (int k = 0; k < RPT; ++k)
#pragma unroll
            for (int c = 0; c < CW; ++c) accR[k] = fma((A)Ld<E>::get(tv[k], c), xb[c], accR[k]);
    } else {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const A xa = xJ[rg * RPT + k];
#pragma unroll
            for (int c = 0; c < CW; ++c) accC[c] = fma((A)Ld<E>::get(tv[k], c), xa, accC[c]);
        }
    }
}

// Entry gi of the coarse residual of batch system b (coarse element, basis
// index): the sum of the restriction shares of the coarse element's update
// chunks, in chunk order.
__device__ inline double coarse_r0(const SchwarzArgs &a, int b, int gi) {
    const int nq = a.nq0;
    const int cl = gi / nq, j = gi - cl * nq;
    const int cc = a.csys_ce0[b] + cl;
    double v = 0.0;
    for (int ch = a.cchunk_ptr[cc]; ch < a.cchunk_ptr[cc + 1]; ++ch) v += a.r0part[ch * nq + j];
    return v;
}

// Entry gi of the input vector of dense system s (local: r on the
// subdomain's dofs; coarse: r0 of its batch system).
__device__ inline double sys_input(const SchwarzArgs &a, int s, bool coarse, int64_t dof0, int gi) {
    if (coarse) return coarse_r0(a, s - a.n_sub, gi);
    if (dof0 >= 0) return a.r[dof0 + gi];
    const int nd = a.nd;
    const int le = gi / nd, i = gi - le * nd;
    return a.r[(int64_t)a.sub_elems[a.sub_ptr[s] + le] * nd + i];
}

// One work item: stored tiles (I, J), J in [j0, j0 + nj), of packed tile row
// I of system s (J <= I).  Each tile is read once and used twice (the
// diagonal tile (I, I), symmetric, only up to its diagonal: its lower part
// serves the row use and, transposed, the part above the diagonal):
//   row use      y_I += T x_J   (accumulated in registers over the item)
//   column use   y_J  = T^T x_I (J < I; reduced across the row groups inside
//                each wavefront with shuffles; each wavefront leaves its sum in
//                the tile's own LDS slot, and after the last tile one barrier
//                lets wavefront 0 add the four sums of every tile and write the
//                tile's column partial, so tiles need no barrier of their own)
// The first two tiles are requested before x is gathered into LDS so their
// latency overlaps the gather.  Tiles then stream through two register
// buffers A and B in a fixed ping-pong (no register copies, no conditional
// loads in the steady state).  Barriers only wait for LDS traffic, so tile
// loads stay in flight across them.  Outputs: the item's row partial in yout,
// the FP64 input entry of row I in *r_own (threads < 64), and in *dot_col the
// thread's share of sum_J (x_J, column partial of J).
template <typename E, typename P>
__device__ inline void schwarz_item(const SchwarzArgs &a, const E *__restrict__ tiles, const ItemDesc &d,
                                    bool coarse, double *smem, int max_nj, double *yout, double *r_own,
                                    double *dot_col) {
    const int s = d.s, I = d.I, j0 = d.j0, nj = d.nj;
    using A = typename AccT<E>::T;
    using V = typename Ld<E>::V;
    constexpr int CW = Piece<E>::bytes / sizeof(E);  // columns per load
    constexpr int NC = TILE / CW;       // column groups per tile row
    constexpr int RG = 256 / NC;        // row groups
    constexpr int RPT = TILE / RG;      // rows per thread
    const int tid = threadIdx.x, cg = tid % NC, rg = tid / NC, lane = tid & 63, wv = tid >> 6;
    const int n = d.n;
    const int64_t toff = d.toff;
    const int64_t cbase = d.cbase + (int64_t)I * (I + 1) / 2;
    const int64_t dof0 = coarse ? -1 : d.dof0;
    // LDS: x in FP64 (columns, then row I), x in the accumulation type, column exchange
    double *x64 = smem;
    double *xI64 = x64 + max_nj * TILE;
    A *xa = sizeof(A) == 8 ? reinterpret_cast<A *>(x64) : reinterpret_cast<A *>(xI64 + TILE);
    A *xIa = xa + max_nj * TILE;
    A *colx = reinterpret_cast<A *>(smem) + (sizeof(A) == 8 ? 1 : 3) * (max_nj + 1) * TILE;  // [max_nj][4][64]
    auto tile_ptr = [&](int J) -> const E * {
        return tiles + (toff + (int64_t)I * (I + 1) / 2 + J) * (TILE * TILE) + (rg * RPT) * TILE + cg * CW;
    };
    // Tiles are read once per apply and exceed the last-level cache: non-temporal
    // loads keep them from evicting data that is reused (the SpMV matrix).  Of
    // the diagonal tile only the pieces that reach the diagonal are read,
    // and rows past the system's last dof (zero padding) are not read at all.
    const int rows_left = n - I * TILE;
    auto load = [&](V (&buf)[RPT], int J) {
        const E *tp = tile_ptr(J);
        const bool diag = J == I;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int r = rg * RPT + k;
            buf[k] = (r < rows_left && (!diag || cg * CW <= r))
                         ? load_piece<E>(tp + k * TILE)
                         : V{};
        }
    };
    A accR[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) accR[k] = 0;
    V bA[RPT], bB[RPT];
    const int npair = nj >> 1;
    // the first one or two tiles are requested before x is gathered
    load(bA, j0);
    if (nj > 1) load(bB, j0 + 1);
    // BF16 tiles hold the scaled inverse C = D^{-1} K^{-1} D^{-1}: the products
    // run on D x and their results are scaled by D (rows past n have d = 0)
    constexpr bool kScaled = std::is_same<E, uint16_t>::value;
    const float *ds = kScaled ? a.dscale + d.rbase : nullptr;
    // the scales of the item's columns and of row I, kept in LDS after the
    // gather (the epilogue uses them again)
    float *dsl = reinterpret_cast<float *>(colx + (size_t)max_nj * 4 * TILE);
    float *dsI = dsl + (size_t)max_nj * TILE;
    // gather x over the item's tile columns and over tile row I
    const int base = j0 * TILE;
    for (int t = tid; t < nj * TILE; t += 256) {
        const int gi = base + t;
        const double v = gi < n ? sys_input(a, s, coarse, dof0, gi) : 0.0;
        x64[t] = v;
        if constexpr (kScaled) {
            const float dv = ds[gi];
            dsl[t] = dv;
            xa[t] = (A)(v * (double)dv);
        } else if (sizeof(A) != 8) {
            xa[t] = (A)v;
        }
    }
    if (tid < TILE) {
        const int gi = I * TILE + tid;
        const double v = gi < n ? sys_input(a, s, coarse, dof0, gi) : 0.0;
        xI64[tid] = v;
        if constexpr (kScaled) {
            const float dv = ds[gi];
            dsI[tid] = dv;
            xIa[tid] = (A)(v * (double)dv);
        } else if (sizeof(A) != 8) {
            xIa[tid] = (A)v;
        }
        *r_own = v;
    }
    __syncthreads();
    double dcol = 0.0;
    // one tile: row use and column use; on the diagonal tile the row use takes
    // the entries up to the diagonal and the column use those below it
    auto tile_step = [&](const V (&buf)[RPT], int jj) {
        const int J = j0 + jj;
        const A *xJ = (sizeof(A) == 8 ? reinterpret_cast<const A *>(x64) : xa) + jj * TILE;
        const A *xIv = sizeof(A) == 8 ? reinterpret_cast<const A *>(xI64) : xIa;
        A xb[CW], cacc[CW];
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            xb[c] = xJ[cg * CW + c];
            cacc[c] = 0;
        }
        if (J < I) {
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                const A xr = xIv[rg * RPT + k];
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    const A t = (A)Ld<E>::get(buf[k], c);
                    accR[k] = fma(t, xb[c], accR[k]);
                    cacc[c] = fma(t, xr, cacc[c]);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                const int r = rg * RPT + k;
                const A xr = xIv[r];
#pragma unroll
                for (int c = 0; c < CW; ++c) {
                    const int col = cg * CW + c;
                    const A t = (A)Ld<E>::get(buf[k], c);
                    accR[k] = fma(col <= r ? t : (A)0, xb[c], accR[k]);
                    cacc[c] = fma(col < r ? t : (A)0, xr, cacc[c]);
                }
            }
        }
        // sum over the row groups inside the wavefront; the tile's slot keeps
        // the four wavefronts' sums until after the last tile
#pragma unroll
        for (int off = NC; off < 64; off <<= 1)
#pragma unroll
            for (int c = 0; c < CW; ++c) cacc[c] += __shfl_xor(cacc[c], off, 64);
        A *cx = colx + jj * 4 * TILE;
        if (lane < NC)
#pragma unroll
            for (int c = 0; c < CW; ++c) cx[wv * TILE + cg * CW + c] = cacc[c];
    };
    int jj = 0;
    if (npair > 0) {
        for (; jj + 2 < 2 * npair; jj += 2) {
            const int J = j0 + jj;
            // scheduling barriers keep each refill after the multiply that frees its buffer
            tile_step(bA, jj);
            __builtin_amdgcn_sched_barrier(0);
            load(bA, J + 2);
            __builtin_amdgcn_sched_barrier(0);
            tile_step(bB, jj + 1);
            __builtin_amdgcn_sched_barrier(0);
            load(bB, J + 3);
            __builtin_amdgcn_sched_barrier(0);
        }
        // last pair; with an odd count the last tile is requested as soon as
        // buffer A is free, so its latency overlaps the pair's second tile
        tile_step(bA, jj);
        __builtin_amdgcn_sched_barrier(0);
        if (jj + 2 < nj) load(bA, j0 + jj + 2);
        __builtin_amdgcn_sched_barrier(0);
        tile_step(bB, jj + 1);
        jj += 2;
        if (jj < nj) {
            tile_step(bA, jj);
            ++jj;
        }
    } else {  // a single tile
        tile_step(bA, 0);
        jj = 1;
    }
    // column partials of the item's tiles below the diagonal, in tile order;
    // the diagonal tile's belong to this item's own rows
    __syncthreads();
    double diag_add = 0.0;
    if (tid < TILE)
        for (int jj2 = 0; jj2 < nj; ++jj2) {
            const A *cx = colx + jj2 * 4 * TILE;
            double v = (double)cx[tid] + (double)cx[TILE + tid] + (double)cx[2 * TILE + tid] +
                       (double)cx[3 * TILE + tid];
            if (kScaled && j0 + jj2 < I) v *= (double)dsl[jj2 * TILE + tid];
            if (j0 + jj2 < I) {
                // the share of (r, z) takes the partial as stored
                const P vp = (P)v;
                reinterpret_cast<P *>(a.colpart)[(cbase + j0 + jj2) * TILE + tid] = vp;
                dcol = fma(x64[jj2 * TILE + tid], (double)vp, dcol);
            } else {
                diag_add = v;
            }
        }
    *dot_col = dcol;
    __syncthreads();  // the reduction scratch aliases the x buffers
    A *sR = reinterpret_cast<A *>(smem);
#pragma unroll
    for (int k = 0; k < RPT; ++k) sR[(rg * NC + cg) * RPT + k] = accR[k];
    __syncthreads();
    if (tid < TILE) {
        const int ar = tid;
        A y = 0;
        const int arg = ar / RPT, ak = ar % RPT;
        for (int c = 0; c < NC; ++c) y += sR[(arg * NC + c) * RPT + ak];
        yout[ar] = kScaled ? ((double)y + diag_add) * (double)dsI[ar] : (double)y + diag_add;
    }
    __syncthreads();
}

// Minimum waves per SIMD the register allocation must allow.  With FP32
// local and coarse tiles the kernel takes 81 registers unconstrained (5
// workgroups per CU); 80 (6 per CU) costs no spill and hides more of the
// start-up latency of small items.  The BF16 form fits 6 already, and forms
// with an FP64 path keep their allocation (a cap there spills).
template <typename EL, typename EC> struct SchwarzMinWaves { static constexpr int value = 1; };
template <> struct SchwarzMinWaves<float, float> { static constexpr int value = 6; };

// One workgroup per item: a fresh workgroup hides the start-up latency of
// the previous one on its CU (a persistent loop over items does not).
template <typename EL, typename EC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(SchwarzMinWaves<EL, EC>::value)))
void k_schwarz(SchwarzArgs a, int max_nj) {
    const int item = blockIdx.x;
    // the item's descriptor (one 64-byte line) and, in a one-system context,
    // that system's stop flag are read together: one memory round trip before
    // the first tile request (a batch needs the owner first)
    const ItemDesc d = a.item_desc[item];
    if (a.mode != 0) {
        int32_t done;
        if (a.n_sys_one) done = a.sc[0].done;
        else done = a.sc[d.owner].done;
        if (done) return;
    }
    extern __shared__ double smem[];
    __shared__ double yout[TILE];
    const int tid = threadIdx.x;
    const int s = d.s;
    const bool coarse = s >= a.n_sub;
    using P = typename PartT<EL, EC>::T;
    double r_own = 0.0, dcol = 0.0;
    const EL *tl = reinterpret_cast<const EL *>(a.tiles_local);
    const EC *tc = reinterpret_cast<const EC *>(a.tiles_coarse);
    if constexpr (std::is_same<EL, uint16_t>::value) {
        // BF16 local store: systems whose rounded inverse failed the
        // positive-definiteness check are stored in FP32
        if (!coarse && d.f32)
            schwarz_item<float, P>(a, reinterpret_cast<const float *>(a.tiles_fallback), d, false, smem, max_nj,
                                   yout, &r_own, &dcol);
        else if (!coarse)
            schwarz_item<EL, P>(a, tl, d, false, smem, max_nj, yout, &r_own, &dcol);
        else
            schwarz_item<EC, P>(a, tc, d, true, smem, max_nj, yout, &r_own, &dcol);
    } else {
        if (!coarse)
            schwarz_item<EL, P>(a, tl, d, false, smem, max_nj, yout, &r_own, &dcol);
        else
            schwarz_item<EC, P>(a, tc, d, true, smem, max_nj, yout, &r_own, &dcol);
    }
    if (tid < TILE) {
        const P yp = (P)yout[tid];
        const double y = (double)yp;
        reinterpret_cast<P *>(a.part)[(int64_t)item * TILE + tid] = yp;
        if (a.mode != 0) {
            // this item's share of (r, z): row I times the row partial, plus the
            // column partials times their x_J
            double v[1] = {fma(r_own, y, dcol)};
            wave_sum<1>(v);
            if (tid == 0) a.itemdot[item] = v[0];
        }
    }
}

// ---------------------------------------------------------------------------
// z = B r assembled from the Schwarz items (tile rows of the local solves plus
// the prolongation P z0 of the coarse solve), and the search direction
// p = z (+ beta p).  In PCG modes every workgroup first forms (r, z) from the
// items' shares (fixed order) to get beta; workgroup 0 also closes the
// iteration: ||r||^2 from the update chunks, convergence / breakdown flags.
// Where the partials of tile row rt are: its items, its index K inside its
// dense system, the system's tile rows and first tile.
struct TileRow {
    int it0, it1, K, nt;
    int64_t cb;
};

__device__ inline TileRow tile_row(const PupdateArgs &a, int rt) {
    return TileRow{a.rt_item0[rt], a.rt_item0[rt + 1], a.rt_k[rt], a.rt_nt[rt], a.rt_cbase[rt]};
}

__device__ inline TileRow tile_row(const ZSrc &z) {
    return TileRow{z.it0, z.it0 + (z.nl >> 8), z.knt >> 16, z.knt & 0xffff, (int64_t)z.cb};
}

// Entry `lane` of tile row t of z is the sum of the row partials of the tile
// row's items and of the column partials of the stored tiles (I, K), I > K,
// below it.  The first round requests up to 4 item and 16 column partials at
// once (those past the end read nothing); tile_row_rest waits for them, reads
// any further ones (16 per round) and adds all in a fixed order.
constexpr int kTrFirst = 20;

// The partials are loaded in their stored type P (FP32 or FP64) and widened
// to FP64 only where they are added, so all of a round's loads are issued
// before the first wait.
template <typename P>
__device__ inline void tile_row_first(const PupdateArgs &a, const TileRow &t, int lane, P (&w)[kTrFirst]) {
    const P *pp = reinterpret_cast<const P *>(a.part);
    const P *cp = reinterpret_cast<const P *>(a.colpart);
#pragma unroll
    for (int u = 0; u < 4; ++u) w[u] = t.it0 + u < t.it1 ? pp[(int64_t)(t.it0 + u) * TILE + lane] : P(0);
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int I = t.K + 1 + u;
        w[4 + u] = I < t.nt ? cp[(t.cb + (int64_t)I * (I + 1) / 2 + t.K) * TILE + lane] : P(0);
    }
}

template <typename P>
__device__ inline double tile_row_rest(const PupdateArgs &a, const TileRow &t, int lane, const P (&w)[kTrFirst]) {
    const P *pp = reinterpret_cast<const P *>(a.part);
    const P *cp = reinterpret_cast<const P *>(a.colpart);
    double v = ((double)w[0] + (double)w[1]) + ((double)w[2] + (double)w[3]);
    for (int it = t.it0 + 4; it < t.it1; ++it) v += (double)pp[(int64_t)it * TILE + lane];
    const int K = t.K, nt = t.nt;
    const int64_t cb = t.cb;
    double c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) c[u] = (double)w[4 + u] + (double)w[12 + u];
    for (int I0 = K + 17; I0 < nt; I0 += 16) {
        P x[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int I = I0 + u;
            x[u] = I < nt ? cp[(cb + (int64_t)I * (I + 1) / 2 + K) * TILE + lane] : P(0);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) c[u & 7] += (double)x[u];
    }
    return v + (((c[0] + c[1]) + (c[2] + c[3])) + ((c[4] + c[5]) + (c[6] + c[7])));
}

template <typename P>
__device__ inline double tile_row_value(const PupdateArgs &a, const TileRow &t, int lane) {
    P w[kTrFirst];
    tile_row_first<P>(a, t, lane, w);
    return tile_row_rest<P>(a, t, lane, w);
}

template <typename P>
__device__ inline double tile_row_value(const PupdateArgs &a, int rt, int lane) {
    return tile_row_value<P>(a, tile_row(a, rt), lane);
}

// P: the storage type of the Schwarz partials (PupdateArgs::f32part).
template <int NQ, typename P>
__global__ __launch_bounds__(256) void k_pupdate(PupdateArgs a) {
    const int nd = a.nd;
    const int64_t n = a.n_elem * nd;
    const int64_t i0 = (int64_t)blockIdx.x * 256;
    const int64_t idx = i0 + threadIdx.x;
    // The block's record, then everything that depends on it alone at once:
    // this dof's old direction and the record of where its value of z is,
    // the coarse rows the block keeps, the first system's stop flag.  z = B r
    // depends only on the Schwarz partials, not on this launch's reductions,
    // so it is formed first (for every dof of the block, also of systems
    // that turn out to be done; those values are dropped).
    // The records that do not depend on the block's record are requested with it:
    // this dof's source record and old direction, and the source record of the
    // coarse value this thread may keep (the slots past the block's n_c * NQ
    // values exist and are not used).
    constexpr int KMAX = kPupdateKmax;
    constexpr int NV = NQ > 0 ? NQ : 1;
    const bool in = idx < n;
    const PuBlk bk = a.blk[blockIdx.x];
    ZSrc zf{0, 0, 0, 0}, zc{0, 0, 0, 0};
    if (in && !a.r_ident) zf = a.dof_src[idx];
    const double p_old = (in && a.mode == 2) ? a.p[idx] : 0.0;
    if (NQ > 0 && (int)threadIdx.x < KMAX * NV) zc = a.blk_csrc[(int64_t)blockIdx.x * (KMAX * NV) + threadIdx.x];
    const int my = in ? (bk.s_lo == bk.s_hi ? bk.s_lo : a.elem_sys[idx / nd]) : -1;
    const bool fine = my >= 0 && !a.r_ident;
    const int f_lane = zf.nl & 63;
    const TileRow f_tr = tile_row(zf);
    // coarse values z0 of the block's coarse elements, once per block: the
    // block's elements usually lie in one or two coarse elements (numbered
    // contiguously), so the block computes their n_c * NQ values into LDS
    // (the range is planned on the host)
    __shared__ double s_z0[KMAX * NV];
    int c_lo = 0, n_c = KMAX + 1;
    if (NQ > 0) {
        c_lo = bk.c_lo;
        n_c = bk.n_c;
    }
    const bool c_val = NQ > 0 && n_c <= KMAX && (int)threadIdx.x < n_c * NQ;
    const int c_lane = zc.nl & 63;
    const TileRow c_tr = tile_row(zc);
    const int done_lo = (a.mode != 0 && threadIdx.x == 0) ? a.sc[bk.s_lo].done : 0;
    // The first system's iteration index and (r, z) of both parities (the owner
    // block writes only the parity of this iteration, which is not used here),
    // and, for small NQ, this dof's row of P and its coarse element: none
    // depends on this launch's sums, so they are requested before its barriers.
    int j_lo = 0;
    double rz_lo_even = 0.0, rz_lo_odd = 0.0;
    if (a.mode == 2) {
        j_lo = a.sc[bk.s_lo].jcur;
        rz_lo_even = a.sc[bk.s_lo].rz[0];
        rz_lo_odd = a.sc[bk.s_lo].rz[1];
    }
    constexpr bool kEarlyP = NQ > 0 && NQ <= 4;
    double Pe[kEarlyP ? NQ : 1];
    int ce_e = 0;
    if (kEarlyP && in) {
        ce_e = a.elem_coarse[idx / nd];
#pragma unroll
        for (int j = 0; j < (kEarlyP ? NQ : 1); ++j) Pe[j] = a.P[idx * NQ + j];
    }
    // the partials of the fine and the coarse value, requested together
    P wf[kTrFirst], wc[kTrFirst];
    if (fine) tile_row_first<P>(a, f_tr, f_lane, wf);
    if (c_val) tile_row_first<P>(a, c_tr, c_lane, wc);
    // this thread's share of the first system's (r, z) partials
    double rz_t = 0.0;
    if (a.mode != 0 && !a.pre_rz)
        rz_t = a.r_ident ? thread_sum_partials<256>(a.rrpart + bk.u0, bk.u1 - bk.u0, 1, 0)
                         : thread_sum_partials<256>(a.itemdot + bk.it0, bk.it1 - bk.it0, 1, 0);
    double zz = 0.0;
    if (my >= 0) zz = a.r_ident ? a.r_ident[idx] : tile_row_rest<P>(a, f_tr, f_lane, wf);
    if (NQ > 0 && n_c <= KMAX) {
        if (c_val) s_z0[threadIdx.x] = tile_row_rest<P>(a, c_tr, c_lane, wc);
        // more than 256 kept values (NQ = 35): the rest one by one
        for (int t = threadIdx.x + 256; t < n_c * NQ; t += 256) {
            const ZSrc zs = a.blk_csrc[(int64_t)blockIdx.x * (KMAX * NV) + t];
            s_z0[t] = tile_row_value<P>(a, tile_row(zs), zs.nl & 63);
        }
        __syncthreads();
    }
    if (NQ > 0 && my >= 0) {
        const int64_t e = idx / nd;
        const int ce = kEarlyP ? ce_e : a.elem_coarse[e];
        const double *Pr = a.P + idx * NQ;
        if (n_c <= KMAX) {
#pragma unroll
            for (int j = 0; j < NQ; ++j)
                zz = fma(kEarlyP ? Pe[j % (kEarlyP ? NQ : 1)] : Pr[j], s_z0[(ce - c_lo) * NQ + j], zz);
        } else {
            const int g0 = a.coarse_base[ce];
#pragma unroll
            for (int j = 0; j < NQ; ++j) {
                const int gi = g0 + j;
                zz = fma(kEarlyP ? Pe[j % (kEarlyP ? NQ : 1)] : Pr[j], tile_row_value<P>(a, gi >> 6, gi & 63), zz);
            }
        }
    }
    double beta = 0.0;
    bool active = a.mode == 0 && my >= 0;
    if (a.mode != 0) {
        // every system with dofs in this block, in turn
        const int s_lo = bk.s_lo, s_hi = bk.s_hi;
        for (int b = s_lo; b <= s_hi; ++b) {
            DevScalars *sc = a.sc + b;
            const bool first = b == s_lo;
            // the owner block may set `done` during this launch
            if (block_bcast<256>(first ? done_lo : (threadIdx.x == 0 ? sc->done : 0))) continue;
            const int it0 = a.r_ident ? (first ? bk.u0 : a.rng.upd[b]) : (first ? bk.it0 : a.rng.item[b]);
            const int it1 = a.r_ident ? (first ? bk.u1 : a.rng.upd[b + 1]) : (first ? bk.it1 : a.rng.item[b + 1]);
            const double rz =
                a.pre_rz ? sc->rz_sum
                         : block_total<256>(first ? rz_t
                                                  : thread_sum_partials<256>(a.r_ident ? a.rrpart + it0 : a.itemdot + it0,
                                                                             it1 - it0, 1, 0));
            const int j = a.mode == 2 ? (first ? j_lo : sc->jcur) : 0;
            const double bt =
                a.mode == 2 ? rz / (first ? ((j - 1) & 1 ? rz_lo_odd : rz_lo_even) : sc->rz[(j - 1) & 1]) : 0.0;
            if (my == b) {
                beta = bt;
                active = true;
            }
            if (a.rng.owner[b] != (int)blockIdx.x) continue;
            // owner: close iteration j of system b
            const int u0 = first ? bk.u0 : a.rng.upd[b];
            const double rr = block_sum_partials<256>(a.rrpart + u0, (first ? bk.u1 : a.rng.upd[b + 1]) - u0, 1, 0);
            double bb = 0.0;
            if (a.mode == 1) {
                const int g0 = a.rng.spmv[b];
                bb = block_sum_partials<256>(a.bbpart + 2 * (int64_t)g0, a.rng.spmv[b + 1] - g0, 2, 0);
            }
            if (threadIdx.x == 0) {
                if (a.mode == 1) sc->bb = bb;
                bb = sc->bb;
                sc->rr = rr;
                sc->rz[j & 1] = rz;
                sc->beta = bt;
                sc->iters = j;
                if (a.lanczos && a.mode == 2 && j <= a.lcap) a.lanczos[(int64_t)b * a.lcap + j - 1].y = bt;
                if (a.mode == 1 && bb == 0.0) {
                    sc->status = ST_ZERO_RHS;
                    sc->done = 1;
                } else if (!finite(rr) || !finite(bb) || !finite(rz)) {
                    sc->status = ST_NONFINITE;
                    sc->done = 1;
                } else if (rr <= sc->tol2 * bb) {
                    sc->status = ST_CONV;
                    sc->done = 1;
                } else if (!(rz > 0.0)) {
                    sc->status = ST_BREAKDOWN;
                    sc->done = 1;
                } else if (j >= sc->maxit) {
                    sc->status = ST_NOCONV;
                    sc->done = 1;
                }
            }
        }
    }
    if (!active) return;
    if (a.mode == 2) zz = fma(beta, p_old, zz);
    a.p[idx] = zz;
}

// The block size of each sum equals that of the kernel that would otherwise
// form it (update: 128, p-update: 256), so both paths add in the same order
// and give the same bits.
template <int BS>
__global__ __launch_bounds__(BS) void k_reduce(const double *part, const int32_t *ranges, int which,
                                               DevScalars *sc) {
    const int b = blockIdx.x, g0 = ranges[b];
    if (which == 0) {
        const double t = block_sum_partials<BS>(part + 2 * (int64_t)g0, ranges[b + 1] - g0, 2, 0);
        if (threadIdx.x == 0) sc[b].pq_sum = t;
    } else {
        const double t = block_sum_partials<BS>(part + g0, ranges[b + 1] - g0, 1, 0);
        if (threadIdx.x == 0) sc[b].rz_sum = t;
    }
}

// Entries of the Lanczos tridiagonal matrix T_m from the PCG coefficients
// h[j] = (alpha_j, beta_j): T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
// T_{j,j+1}^2 = beta_j / alpha_j^2 (formed as (sqrt(beta_j)/alpha_j)^2).
__device__ inline double lanczos_diag(const double2 *h, int j) {
    return 1.0 / h[j].x + (j > 0 ? h[j - 1].y / h[j - 1].x : 0.0);
}
__device__ inline double lanczos_off2(const double2 *h, int j) {
    const double off = sqrt(h[j].y) / h[j].x;
    return off * off;
}

// T_m held in LDS (short histories) ...
struct TriLds {
    const double *d, *e2;
    __device__ double diag(int j) const { return d[j]; }
    __device__ double off2(int j) const { return e2[j]; }
};
// ... or formed on the fly from the history in global memory (long ones);
// both give the same values.
struct TriHist {
    const double2 *h;
    __device__ double diag(int j) const { return lanczos_diag(h, j); }
    __device__ double off2(int j) const { return lanczos_off2(h, j); }
};

// Number of eigenvalues below x of the symmetric tridiagonal matrix with
// diagonal d and squared off-diagonal e2 (Sturm sequence of the LDL^T pivots).
template <typename Tri>
__device__ inline int sturm_count(const Tri &T, int m, double x, double tiny) {
    int c = 0;
    double q = T.diag(0) - x;
    for (int j = 0;;) {
        if (q < 0.0) ++c;
        if (++j >= m) break;
        if (fabs(q) < tiny) q = q < 0.0 ? -tiny : tiny;
        q = T.diag(j) - x - T.off2(j - 1) / q;
    }
    return c;
}

// Extreme eigenvalues by parallel bisection: each round the 256 threads count
// at 256 interior points of the bracket, which shrinks 257-fold.
template <typename Tri>
__device__ void lanczos_extremes(const Tri &T, int m, DevScalars *sc, int *s_cnt, double *s_lohi) {
    constexpr int NT = 256;
    const int t = threadIdx.x;
    if (t == 0) {  // Gershgorin bracket
        double lo = 1e300, hi = -1e300;
        for (int j = 0; j < m; ++j) {
            const double r = (j > 0 ? sqrt(T.off2(j - 1)) : 0.0) + (j + 1 < m ? sqrt(T.off2(j)) : 0.0);
            lo = fmin(lo, T.diag(j) - r);
            hi = fmax(hi, T.diag(j) + r);
        }
        s_lohi[0] = lo;
        s_lohi[1] = hi;
    }
    __syncthreads();
    const double glo = s_lohi[0], ghi = s_lohi[1];
    const double tiny = 1e-300 + 1e-30 * fmax(fabs(glo), fabs(ghi));
    for (int which = 0; which < 2; ++which) {  // 0: smallest (count >= 1), 1: largest (count >= m)
        const int target = which == 0 ? 1 : m;
        double lo = glo, hi = ghi;
        for (int round = 0; round < 8; ++round) {
            const double x = lo + (hi - lo) * (double)(t + 1) / (double)(NT + 1);
            s_cnt[t] = sturm_count(T, m, x, tiny) >= target;
            __syncthreads();
            if (t == 0) {
                int k = 0;
                while (k < NT && !s_cnt[k]) ++k;  // first point whose count reaches the target
                const double w = (hi - lo) / (double)(NT + 1);
                s_lohi[1] = k < NT ? lo + w * (k + 1) : hi;
                s_lohi[0] = lo + w * k;
            }
            __syncthreads();
            lo = s_lohi[0];
            hi = s_lohi[1];
            __syncthreads();
        }
        if (t == 0) {
            if (which == 0) sc->lmin = 0.5 * (lo + hi);
            else sc->lmax = 0.5 * (lo + hi);
        }
    }
}

__global__ __launch_bounds__(256) void k_lanczos(const double2 *hist, int lcap, DevScalars *sc) {
    constexpr int NT = 256, MAXM = 2048;
    __shared__ double d[MAXM], e2[MAXM];
    __shared__ int s_cnt[NT];
    __shared__ double s_lohi[2];
    const int b = blockIdx.x, t = threadIdx.x;
    const int m = min(sc[b].iters, lcap);
    if (m < 1) {
        if (t == 0) sc[b].lmin = sc[b].lmax = 1.0;
        return;
    }
    const double2 *h = hist + (int64_t)b * lcap;
    if (m <= MAXM) {
        for (int j = t; j < m; j += NT) {
            d[j] = lanczos_diag(h, j);
            if (j + 1 < m) e2[j] = lanczos_off2(h, j);
        }
        __syncthreads();
        lanczos_extremes(TriLds{d, e2}, m, sc + b, s_cnt, s_lohi);
    } else {
        lanczos_extremes(TriHist{h}, m, sc + b, s_cnt, s_lohi);
    }
}

// sc[b].tr = sum of the SpMV partials (slot `slot`) of system b; one block per system.
__global__ __launch_bounds__(256) void k_sum_partials(const double *part, const int32_t *ranges, int slot,
                                                      DevScalars *sc) {
    const int b = blockIdx.x, g0 = ranges[b];
    const double t = block_sum_partials<256>(part + 2 * (int64_t)g0, ranges[b + 1] - g0, 2, slot);
    if (threadIdx.x == 0) sc[b].tr = t;
}

// ---------------------------------------------------------------------------
// Ionic model (Barreto-Cressman-type, five states n, h, K_o, Na_i, Ca_i).
__device__ inline double xexp(double x) {
    return fabs(x) < 1e-4 ? 1.0 + x * 0.5 + x * x / 12.0 : x / (1.0 - exp(-x));
}

// vcl: the chloride reversal potential prm[17] log(prm[15] / prm[16]) (a
// constant of the parameter set).
__device__ inline void ionic_model(double V, const double *y, const double *prm, double vcl, double &f,
                                   double *dy, int &bad) {
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
// I = int f(u~, y^(k+1)) phi with the extrapolated potential
// u~ = ext_now u^k + ext_prev u^(k-1) (2, -1: to t^(k+1); 3/2, -1/2: to the
// Crank-Nicolson mid-point).
template <int DIM, int P>
struct IonicMinWaves { static constexpr int value = NB<DIM, P>::v <= 10 ? 3 : 1; };

template <int DIM, int P>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(IonicMinWaves<DIM, P>::value)))
void k_ionic(IonicArgs a) {
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
    const double vcl = a.prm[17] * log(a.prm[15] / a.prm[16]);
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
            // phi is stored before the model is evaluated, so its registers are free there
#pragma unroll
            for (int k = 0; k < ND; ++k) s_phi[lane][k] = phi[k];
            double f, dy[5];
            ionic_model(u, yv, s_prm, vcl, f, dy, bad);
            const double w = a.qp_w[q];
#pragma unroll
            for (int l = 0; l < 5; ++l) s_w[lane][l] = w * dy[l];
        } else {
#pragma unroll
            for (int l = 0; l < 5; ++l) s_w[lane][l] = 0.0;
#pragma unroll
            for (int k = 0; k < ND; ++k) s_phi[lane][k] = 0.0;
        }
        __syncthreads();
        // the chunk's points (the slots past the last one hold zeros)
        const int nqc = (int)(q1 - c0 < 64 ? q1 - c0 : 64);
#pragma unroll
        for (int t = 0; t < NOUT; ++t) {
            const int o = lane + 64 * t;
            if (o < 5 * ND) {
                const int l = o / ND, k = o - l * ND;
                double s = accG[t];
                for (int qq = 0; qq < nqc; ++qq) s = fma(s_w[qq][l], s_phi[qq][k], s);
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
#pragma unroll
            for (int k = 0; k < ND; ++k) s_phi[lane][k] = phi[k];
            double f;
            ionic_model(a.ext_now * u + a.ext_prev * up, yv, s_prm, vcl, f, nullptr, bad);
            s_w[lane][0] = a.qp_w[q] * f;
        } else {
            s_w[lane][0] = 0.0;
#pragma unroll
            for (int k = 0; k < ND; ++k) s_phi[lane][k] = 0.0;
        }
        __syncthreads();
        const int nqc = (int)(q1 - c0 < 64 ? q1 - c0 : 64);
        if (lane < ND)
            for (int qq = 0; qq < nqc; ++qq) accI = fma(s_w[qq][0], s_phi[qq][lane], accI);
        __syncthreads();
    }
    if (lane < ND) a.I[e * ND + lane] = accI;
    if (bad) s_bad = 1;
    __syncthreads();
    if (lane == 0 && s_bad) *a.bad = 1;
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

// out = x, with the dofs of systems stopped on a zero right-hand side set to 0.
__global__ void k_finish(const double *x, double *out, const int32_t *elem_sys, int nd, int64_t n_elem,
                         const DevScalars *sc) {
    const int64_t n = n_elem * nd;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        out[t] = sc[elem_sys[t / nd]].status == ST_ZERO_RHS ? 0.0 : x[t];
}

// One block per update chunk (inside one system): the system's guess residual
// norm from the SpMV partials, compared with that of u, decides the chunk's
// dofs; the system's first chunk records the decision.
__global__ __launch_bounds__(128) void k_choose(ChooseArgs a) {
    const int c = blockIdx.x, b = a.grp_sys[c];
    DevScalars *sc = a.sc + b;
    const int g0 = a.rng.spmv[b];
    const double rg = block_sum_partials<128>(a.part + 2 * (int64_t)g0, a.rng.spmv[b + 1] - g0, 2, 1);
    const bool use = rg < sc->tr;
    if (c == a.sys_chunk0[b] && threadIdx.x == 0) sc->guess = use ? 1 : 0;
    if (!use) return;
    const int e0 = a.grp_ptr[c], ndof = (a.grp_ptr[c + 1] - e0) * a.nd;
    for (int d = threadIdx.x; d < ndof; d += 128) {
        const int le = d / a.nd, i = d - le * a.nd;
        const int64_t idx = (int64_t)a.grp_elems[e0 + le] * a.nd + i;
        a.x[idx] = a.g[idx];
        a.r[idx] = a.r_g[idx];
    }
}

__global__ void k_extrapolate(const double *u, const double *u1, const double *u2, int order, int64_t n,
                              double *guess) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
        guess[t] = order == 1 ? 2.0 * u[t] - u1[t] : 3.0 * (u[t] - u1[t]) + u2[t];
}

__global__ void k_status_reset(DevScalars *sc, int n_sys, double tol2, int maxit, int reset_ionic) {
    for (int b = blockIdx.x * blockDim.x + threadIdx.x; b < n_sys; b += gridDim.x * blockDim.x) {
        DevScalars &d = sc[b];
        if (reset_ionic) d.ionic_bad = 0;
        d.bb = d.rr = d.pq = d.alpha = d.beta = d.tr = 0.0;
        d.rz[0] = d.rz[1] = 0.0;
        d.tol2 = tol2;
        d.done = 0;
        d.status = ST_RUN;
        d.iters = 0;
        d.jcur = 0;
        d.guess = -1;
        d.maxit = maxit;
    }
}

// ---------------------------------------------------------------------------
// launchers
template <int ND, int WPG>
static hipError_t spmv_nd_w(const DevMatrix &A, const SpmvArgs &a, hipStream_t s) {
    if constexpr (ND >= kWideMinNd) {
        if (A.nt)
            hipLaunchKernelGGL((k_spmv_wide<ND, WPG, true>), dim3((unsigned)A.n_wg), dim3(64 * WPG), 0, s, A, a);
        else
            hipLaunchKernelGGL((k_spmv_wide<ND, WPG, false>), dim3((unsigned)A.n_wg), dim3(64 * WPG), 0, s, A, a);
    } else {
        if (A.nt)
            hipLaunchKernelGGL((k_spmv<ND, WPG, true>), dim3((unsigned)A.n_wg), dim3(64 * WPG), 0, s, A, a);
        else
            hipLaunchKernelGGL((k_spmv<ND, WPG, false>), dim3((unsigned)A.n_wg), dim3(64 * WPG), 0, s, A, a);
    }
    return hipGetLastError();
}

template <int ND>
static hipError_t spmv_nd(const DevMatrix &A, const SpmvArgs &a, hipStream_t s) {
    switch (A.wpg) {
    case 1: return spmv_nd_w<ND, 1>(A, a, s);
    case 2: return spmv_nd_w<ND, 2>(A, a, s);
    case 4: return spmv_nd_w<ND, 4>(A, a, s);
    case 8: return spmv_nd_w<ND, 8>(A, a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_spmv(const DevMatrix &A, const SpmvArgs &a, hipStream_t s) {
    if (A.n_wg <= 0) return hipSuccess;
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

// nq0 = dim P^q of the coarse space: 3, 6, 10, 15 (2-D) or 4, 10, 20, 35 (3-D), 0 without
template <int ND>
static hipError_t update_nd(const UpdateArgs &a, hipStream_t s) {
    const dim3 g(a.n_wg), b(128);
    switch (a.nq0) {
    case 0: hipLaunchKernelGGL((k_update<ND, 0>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_update<ND, 3>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_update<ND, 4>), g, b, 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_update<ND, 6>), g, b, 0, s, a); break;
    case 10: hipLaunchKernelGGL((k_update<ND, 10>), g, b, 0, s, a); break;
    case 15: hipLaunchKernelGGL((k_update<ND, 15>), g, b, 0, s, a); break;
    case 20: hipLaunchKernelGGL((k_update<ND, 20>), g, b, 0, s, a); break;
    case 35: hipLaunchKernelGGL((k_update<ND, 35>), g, b, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_update(const UpdateArgs &a, hipStream_t s) {
    if (a.n_wg <= 0) return hipSuccess;
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
    constexpr int CW = Piece<E>::bytes / sizeof(E), NC = TILE / CW, RG = 256 / NC, RPT = TILE / RG;
    return (size_t)256 * RPT * acc_size<E>();
}

// x (FP64, columns + row I), x in the accumulation type, column exchange
// [2][4][64]; the final row reduction (256 * RPT values) reuses the same space
static size_t lds_need(size_t acc, size_t scratch, int max_nj, bool scaled) {
    size_t b = (size_t)(max_nj + 1) * TILE * 8 + (acc == 8 ? 0 : (size_t)(max_nj + 1) * TILE * acc);
    b = (b + 15) & ~(size_t)15;
    const size_t x_end = (acc == 8 ? 1 : 3) * (size_t)(max_nj + 1) * TILE * acc;  // offset of the exchange area
    if (x_end > b) b = x_end;
    b += (size_t)max_nj * 4 * TILE * acc;  // per-tile column sums of the four wavefronts
    if (scaled) b += (size_t)(max_nj + 1) * TILE * 4;  // BF16 store: column and row scales
    return b > scratch ? b : scratch;
}

template <typename EL, typename EC>
static size_t schwarz_bytes_t(int max_nj) {
    size_t bl = lds_need(acc_size<EL>(), scratch_bytes<EL>(), max_nj, std::is_same<EL, uint16_t>::value);
    const size_t bc = lds_need(acc_size<EC>(), scratch_bytes<EC>(), max_nj, false);
    if (std::is_same<EL, uint16_t>::value) {  // FP32-stored fallback systems
        const size_t bf = lds_need(acc_size<float>(), scratch_bytes<float>(), max_nj, false);
        bl = bl > bf ? bl : bf;
    }
    return bl > bc ? bl : bc;
}

template <typename EL, typename EC>
static hipError_t schwarz_t(const SchwarzArgs &a, int grid, int max_nj, hipStream_t s, hipEvent_t e0,
                            hipEvent_t e1) {
    const size_t lds = schwarz_bytes_t<EL, EC>(max_nj);
    if (e0 || e1)  // the dispatch itself records the start and stop times
        hipExtLaunchKernelGGL(k_schwarz<EL, EC>, dim3(grid), dim3(256), (uint32_t)lds, s, e0, e1, 0u, a, max_nj);
    else
        hipLaunchKernelGGL((k_schwarz<EL, EC>), dim3(grid), dim3(256), lds, s, a, max_nj);
    return hipGetLastError();
}

size_t schwarz_lds_bytes(int local_store, int coarse_store, int max_nj) {
    const size_t l = local_store == STORE_F64 ? schwarz_bytes_t<double, double>(max_nj)
                     : local_store == STORE_F32 ? schwarz_bytes_t<float, float>(max_nj)
                                                : schwarz_bytes_t<uint16_t, float>(max_nj);
    const size_t c = coarse_store == STORE_F64 ? schwarz_bytes_t<double, double>(max_nj)
                                               : schwarz_bytes_t<float, float>(max_nj);
    return l > c ? l : c;
}

hipError_t launch_schwarz(const SchwarzArgs &a, int grid, int local_store, int coarse_store, int max_nj,
                          hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (grid <= 0) return hipSuccess;
    if (coarse_store == STORE_F64) {
        switch (local_store) {
        case STORE_F64: return schwarz_t<double, double>(a, grid, max_nj, s, e0, e1);
        case STORE_F32: return schwarz_t<float, double>(a, grid, max_nj, s, e0, e1);
        case STORE_BF16: return schwarz_t<uint16_t, double>(a, grid, max_nj, s, e0, e1);
        }
    } else {
        switch (local_store) {
        case STORE_F64: return schwarz_t<double, float>(a, grid, max_nj, s, e0, e1);
        case STORE_F32: return schwarz_t<float, float>(a, grid, max_nj, s, e0, e1);
        case STORE_BF16: return schwarz_t<uint16_t, float>(a, grid, max_nj, s, e0, e1);
        }
    }
    return hipErrorInvalidValue;
}

template <typename P>
static hipError_t pupdate_t(const PupdateArgs &a, dim3 g, dim3 b, hipStream_t s) {
    switch (a.nq0) {
    case 0: hipLaunchKernelGGL((k_pupdate<0, P>), g, b, 0, s, a); break;
    case 3: hipLaunchKernelGGL((k_pupdate<3, P>), g, b, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_pupdate<4, P>), g, b, 0, s, a); break;
    case 6: hipLaunchKernelGGL((k_pupdate<6, P>), g, b, 0, s, a); break;
    case 10: hipLaunchKernelGGL((k_pupdate<10, P>), g, b, 0, s, a); break;
    case 15: hipLaunchKernelGGL((k_pupdate<15, P>), g, b, 0, s, a); break;
    case 20: hipLaunchKernelGGL((k_pupdate<20, P>), g, b, 0, s, a); break;
    case 35: hipLaunchKernelGGL((k_pupdate<35, P>), g, b, 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_pupdate(const PupdateArgs &a, hipStream_t s) {
    const int64_t n = a.n_elem * a.nd;
    if (n <= 0) return hipSuccess;
    const dim3 g((unsigned)((n + 255) / 256)), b(256);
    if (a.f32part) return pupdate_t<float>(a, g, b, s);
    return pupdate_t<double>(a, g, b, s);
}

hipError_t launch_sum_partials(const double *part, const int32_t *ranges, int n_sys, int slot, DevScalars *sc,
                               hipStream_t s) {
    if (n_sys <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_partials, dim3(n_sys), dim3(256), 0, s, part, ranges, slot, sc);
    return hipGetLastError();
}

hipError_t launch_reduce(const double *part, const int32_t *ranges, int n_sys, int which, DevScalars *sc,
                         hipStream_t s) {
    if (n_sys <= 0) return hipSuccess;
    if (which == 0)
        hipLaunchKernelGGL(k_reduce<128>, dim3(n_sys), dim3(128), 0, s, part, ranges, which, sc);
    else
        hipLaunchKernelGGL(k_reduce<256>, dim3(n_sys), dim3(256), 0, s, part, ranges, which, sc);
    return hipGetLastError();
}

hipError_t launch_lanczos(const double2 *hist, int lcap, int n_sys, DevScalars *sc, hipStream_t s) {
    if (n_sys <= 0 || !hist) return hipSuccess;
    hipLaunchKernelGGL(k_lanczos, dim3(n_sys), dim3(256), 0, s, hist, lcap, sc);
    return hipGetLastError();
}

hipError_t launch_ionic(const IonicArgs &a, hipStream_t s) {
    if (a.n_elem <= 0) return hipSuccess;
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

static int grid_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

hipError_t launch_project_p0(const double *vals, int ncomp, int64_t n_elem, int nd, const double *norm,
                             double *coeff, hipStream_t s) {
    hipLaunchKernelGGL(k_project_p0, dim3(grid_for((int64_t)ncomp * n_elem * nd)), dim3(256), 0, s, vals, ncomp,
                       n_elem, nd, norm, coeff);
    return hipGetLastError();
}

hipError_t launch_finish(const double *x, double *out, const int32_t *elem_sys, int nd, int64_t n_elem,
                         const DevScalars *sc, hipStream_t s) {
    hipLaunchKernelGGL(k_finish, dim3(grid_for(n_elem * nd)), dim3(256), 0, s, x, out, elem_sys, nd, n_elem, sc);
    return hipGetLastError();
}

hipError_t launch_choose(const ChooseArgs &a, hipStream_t s) {
    if (a.n_grp <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_choose, dim3(a.n_grp), dim3(128), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_extrapolate(const double *u, const double *u1, const double *u2, int order, int64_t n,
                              double *guess, hipStream_t s) {
    hipLaunchKernelGGL(k_extrapolate, dim3(grid_for(n)), dim3(256), 0, s, u, u1, u2, order, n, guess);
    return hipGetLastError();
}

hipError_t launch_status_reset(DevScalars *sc, int n_sys, double tol2, int maxit, int reset_ionic, hipStream_t s) {
    hipLaunchKernelGGL(k_status_reset, dim3(grid_for(n_sys)), dim3(256), 0, s, sc, n_sys, tol2, maxit, reset_ionic);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of the allocation-free preconditioner apply: one array per device,
// held from the library's first use on that device until the process ends.
// In host code `scratch` names a host-side stand-in, not device memory; every
// host use goes through the address hipGetSymbolAddress returns for the
// device that was current at set-up.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_init(int device) {
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device) return hipErrorInvalidDevice;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
    return hipSuccess;
}

void *static_scratch(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace pdg
