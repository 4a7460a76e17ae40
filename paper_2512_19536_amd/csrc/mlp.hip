// Kernels of the learned initial guess: a per-element multilayer perceptron
// trained on trajectories of the method itself, in BF16 with FP32
// accumulation on the gfx950 matrix cores (v_mfma_f32_16x16x32_bf16).
//
// One product kernel serves every layer product of training and inference:
//   forward          H_l  = relu(H_{l-1} W_l^T + b_l)    (NT: A = H_{l-1}, B = W_l)
//   data gradient    dH_l = (dY_{l+1} W_{l+1}) * [H_l > 0]  (NT: B = W_{l+1}^T)
//   weight gradient  dW_l = dY_l^T H_{l-1}               (NT: A = dY_l^T, B = H_{l-1}^T,
//                                                          reduction over samples, split)
// so the kernels keep a transposed copy of every activation and gradient
// they write, and of every weight matrix.  Split products write FP32 partials
// that a second kernel adds in a fixed order: results are deterministic.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "mlp.h"

namespace pdg {
namespace mlp {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// FP32 -> BF16, round to nearest even (NaN stays NaN).
__device__ inline uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline bf16x8 load8(const uint16_t *p) { return __builtin_bit_cast(bf16x8, *(const uint4 *)p); }

// Narrow products (32 output columns): one wavefront per 32 x 32 output tile
// (2 x 2 MFMA tiles of 16 x 16), operands straight from global memory.
// Operand layout of v_mfma_f32_16x16x32_bf16: lane l supplies row l % 16 of
// the A tile and column l % 16 of the B tile at reduction indices
// 8 (l / 16) .. 8 (l / 16) + 7, i.e. one 16-byte load from each operand's row;
// it receives D[4 (l / 16) + v][l % 16], v = 0..3.
__global__ __launch_bounds__(64) void k_gemm_nt(GemmArgs a) {
    const int lane = threadIdx.x;
    const int64_t m0 = (int64_t)blockIdx.x * 32;
    const int n0 = blockIdx.y * 32;
    const int64_t k0 = (int64_t)blockIdx.z * a.k_chunk;
    const int64_t k1 = k0 + a.k_chunk < a.K ? k0 + a.k_chunk : a.K;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    const uint16_t *pa0 = a.A + (m0 + r) * a.lda + kq;
    const uint16_t *pa1 = pa0 + 16 * a.lda;
    const uint16_t *pb0 = a.B + (int64_t)(n0 + r) * a.ldb + kq;
    const uint16_t *pb1 = pb0 + 16 * a.ldb;
    for (int64_t k = k0; k < k1; k += 32) {
        const bf16x8 fa0 = load8(pa0 + k), fa1 = load8(pa1 + k);
        const bf16x8 fb0 = load8(pb0 + k), fb1 = load8(pb1 + k);
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, fb0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa0, fb1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, fb0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa1, fb1, acc[1][1], 0, 0, 0);
    }
    const int rq = (lane >> 4) * 4, c = lane & 15;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int col = n0 + 16 * j + c;
            const int64_t rb = m0 + 16 * i + rq;
            if (a.P) {
                float *P = a.P + (int64_t)blockIdx.z * a.M * a.N;
#pragma unroll
                for (int v = 0; v < 4; ++v) P[(rb + v) * a.N + col] = acc[i][j][v];
                continue;
            }
            uint16_t hv[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = rb + v;
                float x = acc[i][j][v];
                if (a.bias) x += a.bias[col];
                if (a.relu) x = x > 0.f ? x : 0.f;
                if (a.mask && !(bf2f(a.mask[row * a.ldm + col]) > 0.f)) x = 0.f;
                if (a.Cf) a.Cf[row * a.ldcf + col] = x;
                hv[v] = f2bf(x);
                if (a.C) a.C[row * a.ldc + col] = hv[v];
            }
            if (a.CT) {
                uint2 pk;
                pk.x = (uint32_t)hv[0] | ((uint32_t)hv[1] << 16);
                pk.y = (uint32_t)hv[2] | ((uint32_t)hv[3] << 16);
                *reinterpret_cast<uint2 *>(a.CT + (int64_t)col * a.ldct + rb) = pk;
            }
        }
}

// Products with at least 64 output columns: a workgroup of nw wavefronts
// computes a 64 x 32nw tile, each wavefront 64 x 32 (4 x 2 MFMA tiles).  The
// A rows of the tile are staged in LDS per reduction chunk of 256 with
// 16-byte loads (read once instead of once per 32 columns); the wavefront's
// B fragments for the chunk are requested first, so they arrive while A is
// staged.  The epilogue (bias, ReLU) runs in registers, then the tile goes
// through LDS as bf16 so that C, the ReLU mask and CT move in 16-byte pieces.
// Every accumulator receives the same MFMA sequence (k ascending) as in the
// one-wavefront kernel below, so both give the same bits.
constexpr int kGemmKc = 256, kGemmLdsRow = kGemmKc + 8;

__global__ __launch_bounds__(512) void k_gemm_nt_wide(GemmArgs a) {
    __shared__ __attribute__((aligned(16))) uint16_t s_t[64 * kGemmLdsRow];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, nw = blockDim.x >> 6;
    const int64_t m0 = (int64_t)blockIdx.x * 64;
    const int nb = 32 * nw, nb0 = blockIdx.y * nb, n0 = nb0 + 32 * w;
    const int64_t kz0 = (int64_t)blockIdx.z * a.k_chunk;
    const int64_t kz1 = kz0 + a.k_chunk < a.K ? kz0 + a.k_chunk : a.K;
    const int r = lane & 15, kq = (lane >> 4) * 8;
    f32x4 acc[4][2];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t kc0 = kz0; kc0 < kz1; kc0 += kGemmKc) {
        const int kc = (int)(kz1 - kc0 < kGemmKc ? kz1 - kc0 : kGemmKc);
        const int nst = kc >> 5, npr = kc >> 3;
        bf16x8 fb[kGemmKc / 32][2];
        const uint16_t *pb = a.B + (int64_t)(n0 + r) * a.ldb + kc0 + kq;
#pragma unroll
        for (int st = 0; st < kGemmKc / 32; ++st)
            if (st < nst) {
                fb[st][0] = load8(pb + 32 * st);
                fb[st][1] = load8(pb + 16 * a.ldb + 32 * st);
            }
        for (int t = tid; t < 64 * npr; t += blockDim.x) {
            const int row = t / npr, q = t - row * npr;
            uint4 v = {0u, 0u, 0u, 0u};
            if (m0 + row < a.M) v = *(const uint4 *)(a.A + (m0 + row) * a.lda + kc0 + 8 * q);
            *(uint4 *)(s_t + row * kGemmLdsRow + 8 * q) = v;
        }
        __syncthreads();
#pragma unroll
        for (int st = 0; st < kGemmKc / 32; ++st) {
            if (st >= nst) break;
            bf16x8 fa[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) fa[i] = *(const bf16x8 *)(s_t + (16 * i + r) * kGemmLdsRow + 32 * st + kq);
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[i], fb[st][j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }
    const int rq = (lane >> 4) * 4, c = lane & 15;
    if (a.P) {
        float *P = a.P + (int64_t)blockIdx.z * a.M * a.N;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t row = m0 + 16 * i + rq + v;
                    if (row < a.M) P[row * a.N + n0 + 16 * j + c] = acc[i][j][v];
                }
        return;
    }
    const int ldp = nb + 8;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rl = 16 * i + rq + v, cl = 32 * w + 16 * j + c;
                const int64_t row = m0 + rl;
                const int col = nb0 + cl;
                float x = acc[i][j][v];
                if (a.bias) x += a.bias[col];
                if (a.relu) x = x > 0.f ? x : 0.f;
                if (a.Cf && row < a.M) {
                    // (no product here asks for both; kept exact for any caller)
                    const float xm = a.mask && !(bf2f(a.mask[row * a.ldm + col]) > 0.f) ? 0.f : x;
                    a.Cf[row * a.ldcf + col] = xm;
                }
                s_t[rl * ldp + cl] = f2bf(x);
            }
    __syncthreads();
    // row-major pass: the mask (a zero keeps the bits of f2bf(0)) and C
    if (a.mask || a.C)
        for (int t = tid; t < 64 * (nb >> 3); t += blockDim.x) {
            const int rl = t / (nb >> 3), q = t - rl * (nb >> 3);
            const int64_t row = m0 + rl;
            if (row >= a.M) continue;
            uint16_t *sp = s_t + rl * ldp + 8 * q;
            if (a.mask) {
                uint16_t mk[8], hv[8];
                *(uint4 *)mk = *(const uint4 *)(a.mask + row * a.ldm + nb0 + 8 * q);
                *(uint4 *)hv = *(const uint4 *)sp;
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if (!(bf2f(mk[e]) > 0.f)) hv[e] = 0;
                *(uint4 *)sp = *(const uint4 *)hv;
            }
            if (a.C) *(uint4 *)(a.C + row * a.ldc + nb0 + 8 * q) = *(const uint4 *)sp;
        }
    if (a.CT) {
        __syncthreads();
        for (int t = tid; t < nb * 8; t += blockDim.x) {
            const int cl = t >> 3, q = t & 7;
            if (m0 + 8 * q >= a.M) continue;
            uint16_t hv[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) hv[e] = s_t[(8 * q + e) * ldp + cl];
            *(uint4 *)(a.CT + (int64_t)(nb0 + cl) * a.ldct + m0 + 8 * q) = *(const uint4 *)hv;
        }
    }
}

__global__ void k_reduce_splits(const float *P, int splits, int64_t n, float *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        float s = 0.f;
        for (int z = 0; z < splits; ++z) s += P[z * n + i];
        out[i] = s;
    }
}

// One block per output feature: fixed-order sum over the samples, eight
// per 16-byte load (rows and ld are multiples of 32).
__global__ __launch_bounds__(256) void k_bias_grad(const uint16_t *dYT, int64_t rows, int64_t ld, float *db) {
    __shared__ float sh[256];
    const int n = blockIdx.x;
    float s = 0.f;
    for (int64_t m = 8 * (int64_t)threadIdx.x; m < rows; m += 8 * 256) {
        uint16_t h[8];
        *(uint4 *)h = *(const uint4 *)(dYT + n * ld + m);
#pragma unroll
        for (int e = 0; e < 8; ++e) s += bf2f(h[e]);
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) db[n] = sh[0];
}

// Mean-squared error over the first n_valid outputs of the weighted rows.
__global__ __launch_bounds__(256) void k_loss(const float *Y, const float *T, const float *w, int64_t rows, int n_out,
                                              int n_valid, double inv_count, uint16_t *dY, uint16_t *dYT,
                                              double *part) {
    __shared__ double sh[256];
    const int64_t m = (int64_t)blockIdx.x * 256 + threadIdx.x;
    double l = 0.0;
    if (m < rows) {
        const float wm = w[m];
        for (int n = 0; n < n_out; ++n) {
            float g = 0.f;
            if (n < n_valid && wm != 0.f) {
                const float d = Y[m * n_out + n] - T[m * n_out + n];
                g = (float)(2.0 * wm * inv_count) * d;
                l += (double)wm * (double)d * (double)d * inv_count;
            }
            const uint16_t h = f2bf(g);
            dY[m * n_out + n] = h;
            dYT[(int64_t)n * rows + m] = h;
        }
    }
    sh[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void k_sum(const double *part, int n, double *out) {
    __shared__ double sh[256];
    double s = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) s += part[k];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w >= 1; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

__device__ inline void store_weight_copies(const AdamArgs &a, int64_t i, float th) {
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        if (l >= a.n_layers) break;
        const int64_t off = a.w_off[l], cnt = (int64_t)a.w_n[l] * a.w_k[l];
        if (i >= off && i < off + cnt) {
            const int64_t j = i - off;
            const int nn = (int)(j / a.w_k[l]), kk = (int)(j - (int64_t)nn * a.w_k[l]);
            const uint16_t h = f2bf(th);
            a.W[l][j] = h;
            a.Wt[l][(int64_t)kk * a.w_n[l] + nn] = h;
        }
    }
}

// Adam (bias-corrected moments) on the FP32 parameters, then their BF16 copies.
__global__ void k_adam(AdamArgs a) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * blockDim.x) {
        const float g = a.g[i];
        const float m = a.b1 * a.m[i] + (1.f - a.b1) * g;
        const float v = a.b2 * a.v[i] + (1.f - a.b2) * g * g;
        a.m[i] = m;
        a.v[i] = v;
        const float th = a.theta[i] - a.lr * (m * a.c1) / (sqrtf(v * a.c2) + a.eps);
        a.theta[i] = th;
        store_weight_copies(a, i, th);
    }
}

__global__ void k_copy_weights(AdamArgs a) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.n; i += (int64_t)gridDim.x * blockDim.x)
        store_weight_copies(a, i, a.theta[i]);
}

// Feature f of element e: groups of nd coefficients
//   u^n, u^n - u^{n-1}, u^{n-1} - u^{n-2}, u^{n-2} - u^{n-3}, y_1^n .. y_5^n.
__global__ void k_features(FeatArgs a) {
    const int64_t total = (int64_t)a.n_in * a.n_rows;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int f = (int)(t / a.n_rows);
        const int64_t e = t - (int64_t)f * a.n_rows;
        double val = 0.0;
        const bool inside = e < a.n_elem && f < 9 * a.nd;
        if (inside) {
            const int g = f / a.nd, i = f - g * a.nd;
            const int64_t idx = e * a.nd + i;
            switch (g) {
            case 0: val = a.u0[idx]; break;
            case 1: val = a.u0[idx] - a.u1[idx]; break;
            case 2: val = a.u1[idx] - a.u2[idx]; break;
            case 3: val = a.u2[idx] - a.u3[idx]; break;
            default: val = a.ions[(int64_t)(g - 4) * a.n_elem * a.nd + idx]; break;
            }
        }
        if (a.raw) {
            if (e < a.n_elem) a.raw[e * a.n_in + f] = (float)val;
            continue;
        }
        const float x = inside ? (float)((val - (double)a.shift[f]) * (double)a.scale[f]) : 0.f;
        const uint16_t h = f2bf(x);
        a.X[(a.row0 + e) * a.n_in + f] = h;
        a.XT[(int64_t)f * a.ld_t + a.row0 + e] = h;
    }
}

__global__ void k_targets(TargArgs a) {
    const int64_t total = (int64_t)a.n_rows * a.n_out;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = t / a.n_out;
        const int i = (int)(t - e * a.n_out);
        const bool inside = e < a.n_elem && i < a.nd;
        const double val = inside ? a.u_next[e * a.nd + i] - a.u0[e * a.nd + i] : 0.0;
        if (a.raw) {
            if (inside) a.raw[e * a.nd + i] = (float)val;
            continue;
        }
        a.T[(a.row0 + e) * a.n_out + i] = inside ? (float)((val - (double)a.shift[i]) * (double)a.scale[i]) : 0.f;
        if (i == 0) a.w[a.row0 + e] = e < a.n_elem ? 1.f : 0.f;
    }
}

__global__ void k_guess(int64_t n_elem, int nd, int64_t row0, int n_out, const double *u0, const float *Y,
                        const float *shift, const float *scale, double *guess) {
    const int64_t total = n_elem * nd;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = t / nd;
        const int i = (int)(t - e * nd);
        guess[t] = u0[t] + (double)Y[(row0 + e) * n_out + i] / (double)scale[i] + (double)shift[i];
    }
}

// ---------------------------------------------------------------------------
static int grid_for(int64_t n) {
    const int64_t b = (n + 255) / 256;
    return (int)(b < 1 ? 1 : (b > 65536 ? 65536 : b));
}

hipError_t launch_gemm(const GemmArgs &a, int splits, hipStream_t s) {
    if (a.M % 32 || a.N % 32 || a.K % 32 || a.k_chunk % 32 || splits < 1) return hipErrorInvalidValue;
    if ((int64_t)splits * a.k_chunk < a.K) return hipErrorInvalidValue;
    if (a.lda % 8 || a.ldb % 8) return hipErrorInvalidValue;  // 16-byte operand loads
    const bool ld16 = !(a.C && a.ldc % 8) && !(a.mask && a.ldm % 8) && !(a.CT && a.ldct % 8);
    if (a.N >= 64 && ld16) {
        // widest tile of at most 8 wavefronts that divides N
        int nw = 8;
        while ((a.N / 32) % nw) --nw;
        hipLaunchKernelGGL(k_gemm_nt_wide, dim3((unsigned)((a.M + 63) / 64), (unsigned)(a.N / (32 * nw)),
                                                (unsigned)splits),
                           dim3(64 * nw), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_gemm_nt, dim3((unsigned)(a.M / 32), (unsigned)(a.N / 32), (unsigned)splits), dim3(64), 0,
                           s, a);
    }
    return hipGetLastError();
}

hipError_t launch_reduce_splits(const float *P, int splits, int64_t n, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_splits, dim3(grid_for(n)), dim3(256), 0, s, P, splits, n, out);
    return hipGetLastError();
}

hipError_t launch_bias_grad(const uint16_t *dYT, int n_out, int64_t rows, int64_t ld, float *db, hipStream_t s) {
    if (rows % 8 || ld % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_bias_grad, dim3(n_out), dim3(256), 0, s, dYT, rows, ld, db);
    return hipGetLastError();
}

hipError_t launch_loss(const float *Y, const float *T, const float *w, int64_t rows, int n_out, int n_valid,
                       double inv_count, uint16_t *dY, uint16_t *dYT, double *part, int *n_part, hipStream_t s) {
    const int blocks = (int)((rows + 255) / 256);
    *n_part = blocks;
    hipLaunchKernelGGL(k_loss, dim3(blocks), dim3(256), 0, s, Y, T, w, rows, n_out, n_valid, inv_count, dY, dYT,
                       part);
    return hipGetLastError();
}

hipError_t launch_sum(const double *part, int n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(256), 0, s, part, n, out);
    return hipGetLastError();
}

hipError_t launch_adam(const AdamArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3(grid_for(a.n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_copy_weights(const AdamArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_copy_weights, dim3(grid_for(a.n)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_features(const FeatArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_features, dim3(grid_for((int64_t)a.n_in * a.n_rows)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_targets(const TargArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_targets, dim3(grid_for(a.n_rows * a.n_out)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_guess(int64_t n_elem, int nd, int64_t row0, int n_out, const double *u0, const float *Y,
                        const float *shift, const float *scale, double *guess, hipStream_t s) {
    hipLaunchKernelGGL(k_guess, dim3(grid_for(n_elem * nd)), dim3(256), 0, s, n_elem, nd, row0, n_out, u0, Y, shift,
                       scale, guess);
    return hipGetLastError();
}

}  // namespace mlp
}  // namespace pdg
