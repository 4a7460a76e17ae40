// Launch interface of the learned-initial-guess kernels (mlp.hip).
//
// The network is a per-element multilayer perceptron with BF16 weights and
// activations and FP32 accumulation.  Matrices are row-major; "NT" products
// C[M][N] = A[M][K] B[N][K]^T take both operands with the reduction index
// contiguous, so every layer product of training (forward, data gradient,
// weight gradient) is one NT product given the transposed copies the
// kernels keep.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>

namespace pdg {
namespace mlp {

struct GemmArgs {
    const uint16_t *A; int64_t lda;   // [M][K] bf16
    const uint16_t *B; int64_t ldb;   // [N][K] bf16
    int64_t M; int N; int64_t K;      // M, N multiples of 32; K multiple of 32
    int64_t k_chunk;                  // reduction range per blockIdx.z (split products), multiple of 32
    // epilogue (unsplit products)
    const float *bias;                // [N] or null
    int relu;
    const uint16_t *mask; int64_t ldm;// [M][N] bf16 or null: keep entries where mask > 0
    uint16_t *C; int64_t ldc;         // bf16 [M][N] or null
    uint16_t *CT; int64_t ldct;       // bf16 transposed [N][M] or null
    float *Cf; int64_t ldcf;          // fp32 [M][N] or null
    float *P;                         // split products: fp32 partials [splits][M][N] (no epilogue)
};

hipError_t launch_gemm(const GemmArgs &a, int splits, hipStream_t s);
// out[i] = sum_z P[z][i] (fixed order), i < n
hipError_t launch_reduce_splits(const float *P, int splits, int64_t n, float *out, hipStream_t s);
// db[n] = sum_m dYT[n][m], m < rows
hipError_t launch_bias_grad(const uint16_t *dYT, int n_out, int64_t rows, int64_t ld, float *db, hipStream_t s);
// MSE loss on the first n_valid outputs: dY = 2 w (Y - T) * inv_count (bf16, and transposed);
// per-block loss partials
hipError_t launch_loss(const float *Y, const float *T, const float *w, int64_t rows, int n_out, int n_valid,
                       double inv_count, uint16_t *dY, uint16_t *dYT, double *part, int *n_part, hipStream_t s);
hipError_t launch_sum(const double *part, int n, double *out, hipStream_t s);

struct AdamArgs {
    float *theta, *m, *v;
    const float *g;
    int64_t n;
    float lr, b1, b2, eps, c1, c2;   // c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
    // bf16 copies of the weight matrices: layer l occupies theta[w_off[l] .. + N_l K_l)
    int n_layers;
    int64_t w_off[4];
    int w_n[4], w_k[4];
    uint16_t *W[4], *Wt[4];
};
hipError_t launch_adam(const AdamArgs &a, hipStream_t s);
// bf16 copies of the weights from the fp32 parameters (no update)
hipError_t launch_copy_weights(const AdamArgs &a, hipStream_t s);

// Per-element features of rows row0 .. row0 + n_elem (elements), padded with
// zero rows up to row0 + n_rows; normalised to bf16 X [rows][n_in] and XT
// [n_in][ld_t] if raw is null, else raw fp32 values to raw [n_elem][n_in].
struct FeatArgs {
    int64_t n_elem, n_rows, row0;
    int nd, n_in;
    const double *u0, *u1, *u2, *u3, *ions;
    const float *shift, *scale;
    uint16_t *X, *XT; int64_t ld_t;
    float *raw;
};
hipError_t launch_features(const FeatArgs &a, hipStream_t s);

// Targets T[row][i] = ((u_next - u0)[e][i] - shift[i]) * scale[i], i < nd, and
// row weights w (1 for elements, 0 for padding rows); raw mode as above.
struct TargArgs {
    int64_t n_elem, n_rows, row0;
    int nd, n_out;
    const double *u_next, *u0;
    const float *shift, *scale;
    float *T, *w;
    float *raw;
};
hipError_t launch_targets(const TargArgs &a, hipStream_t s);

// guess[e][i] = u0[e][i] + Y[row0 + e][i] / scale[i] + shift[i], i < nd
hipError_t launch_guess(int64_t n_elem, int nd, int64_t row0, int n_out, const double *u0, const float *Y,
                        const float *shift, const float *scale, double *guess, hipStream_t s);

}  // namespace mlp
}  // namespace pdg
