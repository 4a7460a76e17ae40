// C-ABI of the learned initial guess: a per-element multilayer perceptron
// (n_in -> width -> width -> width -> n_out, ReLU between layers) with FP32
// master parameters, BF16 copies for the matrix-core products, Adam, and the
// kernels that turn the method's state into features and predictions into
// an initial guess.  Like the solver context it never allocates device
// memory: all of its device state lives in one caller-bound workspace.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "mlp.h"
#include "pdg_internal.h"

using namespace pdg;
using namespace pdg::mlp;

namespace {

#define HIPCHK(expr)                                                                           \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess)                                                                  \
            throw Error(PDG_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));         \
    } while (0)

constexpr int kLayers = 4;
constexpr int64_t kSplitRows = 1024;   // samples per partial of a weight-gradient product

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

struct pdg_mlp {
    int device = -1;
    hipStream_t stream = nullptr;
    std::string err;
    pdg_mlp_desc d{};
    int N[kLayers] = {}, K[kLayers] = {};
    int64_t off_w[kLayers] = {}, off_b[kLayers] = {};
    int64_t n_params = 0;
    int64_t max_splits = 1;
    bool bound = false, have_params = false, have_norm = false;
    int64_t t = 0;                     // Adam steps taken
    size_t bytes = 0;
    char *ws = nullptr;
    // device slots
    float *theta = nullptr, *m1 = nullptr, *m2 = nullptr, *grad = nullptr;
    uint16_t *W[kLayers] = {}, *Wt[kLayers] = {};
    uint16_t *X = nullptr, *XT = nullptr;
    uint16_t *H[3] = {}, *HT[3] = {};
    uint16_t *dY[kLayers] = {}, *dYT[kLayers] = {};
    float *Y = nullptr, *T = nullptr, *w = nullptr, *P = nullptr;
    float *xs = nullptr, *xk = nullptr, *ts = nullptr, *tk = nullptr;  // normalisation
    double *lpart = nullptr, *loss = nullptr;
    double *loss_host = nullptr;
};

namespace {

template <class F>
pdg_status mguard(pdg_mlp *m, F f) {
    try {
        f();
        if (m) m->err.clear();
        return PDG_OK;
    } catch (Error &e) {
        if (m) m->err = e.what();
        return e.code;
    } catch (std::bad_alloc &) {
        if (m) m->err = "host allocation failed";
        return PDG_ENOMEM;
    } catch (std::exception &e) {
        if (m) m->err = e.what();
        return PDG_EINVAL;
    }
}

void need_bound(const pdg_mlp *m) {
    if (!m) throw Error(PDG_EINVAL, "mlp is NULL");
    if (!m->bound) throw Error(PDG_ESTATE, "workspace not bound");
}

// Carves the workspace (also used with base = nullptr to size it).
size_t carve(pdg_mlp *m, char *base) {
    size_t off = 0;
    auto take = [&](size_t b) {
        char *p = base ? base + off : nullptr;
        off = align256(off + std::max<size_t>(b, 1));
        return p;
    };
    const int64_t R = m->d.max_rows;
    const int64_t np = m->n_params;
    m->theta = (float *)take(np * 4);
    m->m1 = (float *)take(np * 4);
    m->m2 = (float *)take(np * 4);
    m->grad = (float *)take(np * 4);
    for (int l = 0; l < kLayers; ++l) {
        m->W[l] = (uint16_t *)take((size_t)m->N[l] * m->K[l] * 2);
        m->Wt[l] = (uint16_t *)take((size_t)m->N[l] * m->K[l] * 2);
    }
    m->X = (uint16_t *)take((size_t)R * m->d.n_in * 2);
    m->XT = (uint16_t *)take((size_t)R * m->d.n_in * 2);
    for (int l = 0; l < 3; ++l) {
        m->H[l] = (uint16_t *)take((size_t)R * m->d.width * 2);
        m->HT[l] = (uint16_t *)take((size_t)R * m->d.width * 2);
    }
    for (int l = 0; l < kLayers; ++l) {
        m->dY[l] = (uint16_t *)take((size_t)R * m->N[l] * 2);
        m->dYT[l] = (uint16_t *)take((size_t)R * m->N[l] * 2);
    }
    m->Y = (float *)take((size_t)R * m->d.n_out * 4);
    m->T = (float *)take((size_t)R * m->d.n_out * 4);
    m->w = (float *)take((size_t)R * 4);
    int64_t pmax = 0;
    for (int l = 0; l < kLayers; ++l) pmax = std::max<int64_t>(pmax, (int64_t)m->N[l] * m->K[l]);
    m->P = (float *)take((size_t)m->max_splits * pmax * 4);
    m->xs = (float *)take(m->d.n_in * 4);
    m->xk = (float *)take(m->d.n_in * 4);
    m->ts = (float *)take(m->d.n_out * 4);
    m->tk = (float *)take(m->d.n_out * 4);
    m->lpart = (double *)take((size_t)((R + 255) / 256 + 1) * 8);
    m->loss = (double *)take(8);
    return off;
}

AdamArgs adam_args(pdg_mlp *m) {
    AdamArgs a{};
    a.theta = m->theta;
    a.m = m->m1;
    a.v = m->m2;
    a.g = m->grad;
    a.n = m->n_params;
    a.n_layers = kLayers;
    for (int l = 0; l < kLayers; ++l) {
        a.w_off[l] = m->off_w[l];
        a.w_n[l] = m->N[l];
        a.w_k[l] = m->K[l];
        a.W[l] = m->W[l];
        a.Wt[l] = m->Wt[l];
    }
    return a;
}

void check_rows(const pdg_mlp *m, int64_t rows) {
    if (rows < 32 || rows % 32 || rows > m->d.max_rows)
        throw Error(PDG_EINVAL, "rows must be a multiple of 32 in 32..max_rows");
}

// Forward pass over rows [0, rows) of X: H_0..H_2 (bf16, and transposed), Y (fp32).
void forward(pdg_mlp *m, int64_t rows) {
    const int64_t R = m->d.max_rows;
    const uint16_t *in = m->X;
    int64_t ld_in = m->d.n_in;
    for (int l = 0; l < kLayers; ++l) {
        GemmArgs g{};
        g.A = in;
        g.lda = ld_in;
        g.B = m->W[l];
        g.ldb = m->K[l];
        g.M = rows;
        g.N = m->N[l];
        g.K = m->K[l];
        g.k_chunk = m->K[l];
        g.bias = m->theta + m->off_b[l];
        if (l < 3) {
            g.relu = 1;
            g.C = m->H[l];
            g.ldc = m->d.width;
            g.CT = m->HT[l];
            g.ldct = R;
        } else {
            g.Cf = m->Y;
            g.ldcf = m->d.n_out;
        }
        HIPCHK(launch_gemm(g, 1, m->stream));
        if (l < 3) {
            in = m->H[l];
            ld_in = m->d.width;
        }
    }
}

// Loss on Y against T (weights w), then the gradients of every parameter into grad.
void backward(pdg_mlp *m, int64_t rows, int64_t n_valid) {
    const int64_t R = m->d.max_rows;
    hipStream_t s = m->stream;
    int n_part = 0;
    const double inv = 1.0 / ((double)n_valid * m->d.n_out_valid);
    // the loss kernel writes dY / dYT of the last layer with leading dimension `rows`
    HIPCHK(launch_loss(m->Y, m->T, m->w, rows, m->d.n_out, m->d.n_out_valid, inv, m->dY[3], m->dYT[3], m->lpart,
                       &n_part, s));
    HIPCHK(launch_sum(m->lpart, n_part, m->loss, s));
    const int64_t splits = (rows + kSplitRows - 1) / kSplitRows;
    for (int l = kLayers - 1; l >= 0; --l) {
        const int64_t ldyt = (l == kLayers - 1) ? rows : R;
        // weight gradient dW_l = dY_l^T in_l (reduction over samples, split)
        GemmArgs g{};
        g.A = m->dYT[l];
        g.lda = ldyt;
        g.B = l == 0 ? m->XT : m->HT[l - 1];
        g.ldb = R;
        g.M = m->N[l];
        g.N = m->K[l];
        g.K = rows;
        g.k_chunk = kSplitRows;
        g.P = m->P;
        HIPCHK(launch_gemm(g, (int)splits, s));
        HIPCHK(launch_reduce_splits(m->P, (int)splits, (int64_t)m->N[l] * m->K[l], m->grad + m->off_w[l], s));
        HIPCHK(launch_bias_grad(m->dYT[l], m->N[l], rows, ldyt, m->grad + m->off_b[l], s));
        if (l == 0) break;
        // data gradient dY_{l-1} = (dY_l W_l) * [H_{l-1} > 0]
        GemmArgs d{};
        d.A = m->dY[l];
        d.lda = m->N[l];
        d.B = m->Wt[l];
        d.ldb = m->N[l];
        d.M = rows;
        d.N = m->K[l];
        d.K = m->N[l];
        d.k_chunk = m->N[l];
        d.mask = m->H[l - 1];
        d.ldm = m->d.width;
        d.C = m->dY[l - 1];
        d.ldc = m->K[l];
        d.CT = m->dYT[l - 1];
        d.ldct = R;
        HIPCHK(launch_gemm(d, 1, s));
    }
}

}  // namespace

extern "C" {

pdg_status pdg_mlp_create(pdg_mlp **out, int32_t hip_device, void *hip_stream, const pdg_mlp_desc *d) {
    if (!out) return PDG_EINVAL;
    *out = nullptr;
    pdg_mlp *m = nullptr;
    try {
        m = new pdg_mlp();
    } catch (...) {
        return PDG_ENOMEM;
    }
    const pdg_status st = mguard(m, [&] {
        if (!d) throw Error(PDG_EINVAL, "desc is NULL");
        if (hip_device < 0) throw Error(PDG_EINVAL, "a HIP device is required");
        for (int v : {d->n_in, d->width, d->n_out})
            if (v < 32 || v % 32 || v > 1024) throw Error(PDG_EINVAL, "n_in, width, n_out: multiples of 32 in 32..1024");
        if (d->n_out_valid < 1 || d->n_out_valid > d->n_out) throw Error(PDG_EINVAL, "n_out_valid must be in 1..n_out");
        if (d->max_rows < 32 || d->max_rows % 32) throw Error(PDG_EINVAL, "max_rows: a positive multiple of 32");
        int n = 0;
        HIPCHK(hipGetDeviceCount(&n));
        if (hip_device >= n) throw Error(PDG_EINVAL, "no such HIP device");
        HIPCHK(hipSetDevice(hip_device));
        m->device = hip_device;
        m->stream = reinterpret_cast<hipStream_t>(hip_stream);
        m->d = *d;
        const int dims[kLayers + 1] = {d->n_in, d->width, d->width, d->width, d->n_out};
        int64_t off = 0;
        for (int l = 0; l < kLayers; ++l) {
            m->N[l] = dims[l + 1];
            m->K[l] = dims[l];
            m->off_w[l] = off;
            off += (int64_t)m->N[l] * m->K[l];
            m->off_b[l] = off;
            off += m->N[l];
        }
        m->n_params = off;
        m->max_splits = (d->max_rows + kSplitRows - 1) / kSplitRows;
        void *h = nullptr;
        HIPCHK(hipHostMalloc(&h, 8, hipHostMallocDefault));
        m->loss_host = reinterpret_cast<double *>(h);
    });
    if (st != PDG_OK) {
        delete m;
        return st;
    }
    *out = m;
    return PDG_OK;
}

void pdg_mlp_destroy(pdg_mlp *m) {
    if (!m) return;
    if (m->bound) (void)hipStreamSynchronize(m->stream);
    if (m->loss_host) (void)hipHostFree(m->loss_host);
    delete m;
}

const char *pdg_mlp_last_error(const pdg_mlp *m) { return m ? m->err.c_str() : "mlp is NULL"; }

pdg_status pdg_mlp_get_sizes(pdg_mlp *m, int64_t *n_params, size_t *workspace_bytes) {
    return mguard(m, [&] {
        if (!m) throw Error(PDG_EINVAL, "mlp is NULL");
        if (n_params) *n_params = m->n_params;
        if (workspace_bytes) *workspace_bytes = carve(m, nullptr);
    });
}

pdg_status pdg_mlp_bind_workspace(pdg_mlp *m, void *dev_ptr, size_t bytes) {
    return mguard(m, [&] {
        if (!m) throw Error(PDG_EINVAL, "mlp is NULL");
        if (m->bound) throw Error(PDG_ESTATE, "workspace already bound");
        const size_t need = carve(m, nullptr);
        if (!dev_ptr || (reinterpret_cast<uintptr_t>(dev_ptr) & 255)) throw Error(PDG_EINVAL, "workspace must be 256-byte aligned");
        if (bytes < need) throw Error(PDG_ENOMEM, "workspace too small");
        HIPCHK(hipSetDevice(m->device));
        m->ws = reinterpret_cast<char *>(dev_ptr);
        m->bytes = bytes;
        carve(m, m->ws);
        HIPCHK(hipMemsetAsync(m->ws, 0, need, m->stream));
        HIPCHK(hipStreamSynchronize(m->stream));
        m->bound = true;
    });
}

pdg_status pdg_mlp_set_params(pdg_mlp *m, const float *params, int64_t n) {
    return mguard(m, [&] {
        need_bound(m);
        if (!params || n != m->n_params) throw Error(PDG_EINVAL, "params: need n_params floats");
        for (int64_t i = 0; i < n; ++i)
            if (!std::isfinite(params[i])) throw Error(PDG_EINVAL, "parameter not finite");
        HIPCHK(hipMemcpyAsync(m->theta, params, n * 4, hipMemcpyHostToDevice, m->stream));
        HIPCHK(hipMemsetAsync(m->m1, 0, n * 4, m->stream));
        HIPCHK(hipMemsetAsync(m->m2, 0, n * 4, m->stream));
        HIPCHK(launch_copy_weights(adam_args(m), m->stream));
        HIPCHK(hipStreamSynchronize(m->stream));
        m->t = 0;
        m->have_params = true;
    });
}

pdg_status pdg_mlp_get_params(pdg_mlp *m, float *params, int64_t n) {
    return mguard(m, [&] {
        need_bound(m);
        if (!params || n != m->n_params) throw Error(PDG_EINVAL, "params: need n_params floats");
        HIPCHK(hipMemcpyAsync(params, m->theta, n * 4, hipMemcpyDeviceToHost, m->stream));
        HIPCHK(hipStreamSynchronize(m->stream));
    });
}

pdg_status pdg_mlp_set_normalisation(pdg_mlp *m, const float *x_shift, const float *x_scale, const float *t_shift,
                                     const float *t_scale) {
    return mguard(m, [&] {
        need_bound(m);
        if (!x_shift || !x_scale || !t_shift || !t_scale) throw Error(PDG_EINVAL, "NULL array");
        for (int i = 0; i < m->d.n_in; ++i)
            if (!std::isfinite(x_shift[i]) || !(x_scale[i] > 0) || !std::isfinite(x_scale[i]))
                throw Error(PDG_EINVAL, "feature normalisation: finite shifts, positive scales");
        for (int i = 0; i < m->d.n_out; ++i)
            if (!std::isfinite(t_shift[i]) || !(t_scale[i] > 0) || !std::isfinite(t_scale[i]))
                throw Error(PDG_EINVAL, "target normalisation: finite shifts, positive scales");
        HIPCHK(hipMemcpyAsync(m->xs, x_shift, m->d.n_in * 4, hipMemcpyHostToDevice, m->stream));
        HIPCHK(hipMemcpyAsync(m->xk, x_scale, m->d.n_in * 4, hipMemcpyHostToDevice, m->stream));
        HIPCHK(hipMemcpyAsync(m->ts, t_shift, m->d.n_out * 4, hipMemcpyHostToDevice, m->stream));
        HIPCHK(hipMemcpyAsync(m->tk, t_scale, m->d.n_out * 4, hipMemcpyHostToDevice, m->stream));
        HIPCHK(hipStreamSynchronize(m->stream));
        m->have_norm = true;
    });
}

pdg_status pdg_mlp_set_batch(pdg_mlp *m, int64_t rows, const uint16_t *X, const float *T, const float *w) {
    return mguard(m, [&] {
        need_bound(m);
        check_rows(m, rows);
        if (!X || !T || !w) throw Error(PDG_EINVAL, "NULL array");
        const int ni = m->d.n_in;
        std::vector<uint16_t> xt((size_t)ni * m->d.max_rows, 0);
        for (int64_t r = 0; r < rows; ++r)
            for (int f = 0; f < ni; ++f) xt[(size_t)f * m->d.max_rows + r] = X[r * ni + f];
        HIPCHK(hipMemcpyAsync(m->X, X, rows * ni * 2, hipMemcpyHostToDevice, m->stream));
        HIPCHK(hipMemcpyAsync(m->XT, xt.data(), xt.size() * 2, hipMemcpyHostToDevice, m->stream));
        HIPCHK(hipMemcpyAsync(m->T, T, rows * m->d.n_out * 4, hipMemcpyHostToDevice, m->stream));
        HIPCHK(hipMemcpyAsync(m->w, w, rows * 4, hipMemcpyHostToDevice, m->stream));
        HIPCHK(hipStreamSynchronize(m->stream));
    });
}

pdg_status pdg_mlp_features(pdg_mlp *m, int64_t row0, int64_t n_elem, int64_t n_rows, int32_t nd, const double *u0,
                            const double *u1, const double *u2, const double *u3, const double *ions, float *raw) {
    return mguard(m, [&] {
        need_bound(m);
        if (!u0 || !u1 || !u2 || !u3 || !ions) throw Error(PDG_EINVAL, "NULL vector");
        if (nd < 1 || 9 * nd > m->d.n_in) throw Error(PDG_EINVAL, "9 nd features must fit in n_in");
        if (n_elem < 1 || n_rows < n_elem) throw Error(PDG_EINVAL, "need 1 <= n_elem <= n_rows");
        if (!raw) {
            if (!m->have_norm) throw Error(PDG_ESTATE, "normalisation not set");
            if (row0 < 0 || row0 + n_rows > m->d.max_rows) throw Error(PDG_EINVAL, "rows out of range");
        }
        FeatArgs a{};
        a.n_elem = n_elem;
        a.n_rows = raw ? n_elem : n_rows;
        a.row0 = row0;
        a.nd = nd;
        a.n_in = m->d.n_in;
        a.u0 = u0;
        a.u1 = u1;
        a.u2 = u2;
        a.u3 = u3;
        a.ions = ions;
        a.shift = m->xs;
        a.scale = m->xk;
        a.X = m->X;
        a.XT = m->XT;
        a.ld_t = m->d.max_rows;
        a.raw = raw;
        HIPCHK(launch_features(a, m->stream));
    });
}

pdg_status pdg_mlp_targets(pdg_mlp *m, int64_t row0, int64_t n_elem, int64_t n_rows, int32_t nd,
                           const double *u_next, const double *u0, float *raw) {
    return mguard(m, [&] {
        need_bound(m);
        if (!u_next || !u0) throw Error(PDG_EINVAL, "NULL vector");
        if (nd < 1 || nd > m->d.n_out_valid) throw Error(PDG_EINVAL, "nd must be <= n_out_valid");
        if (n_elem < 1 || n_rows < n_elem) throw Error(PDG_EINVAL, "need 1 <= n_elem <= n_rows");
        if (!raw) {
            if (!m->have_norm) throw Error(PDG_ESTATE, "normalisation not set");
            if (row0 < 0 || row0 + n_rows > m->d.max_rows) throw Error(PDG_EINVAL, "rows out of range");
        }
        TargArgs a{};
        a.n_elem = n_elem;
        a.n_rows = raw ? n_elem : n_rows;
        a.row0 = row0;
        a.nd = nd;
        a.n_out = m->d.n_out;
        a.u_next = u_next;
        a.u0 = u0;
        a.shift = m->ts;
        a.scale = m->tk;
        a.T = m->T;
        a.w = m->w;
        a.raw = raw;
        HIPCHK(launch_targets(a, m->stream));
    });
}

pdg_status pdg_mlp_forward(pdg_mlp *m, int64_t rows, float *y_out) {
    return mguard(m, [&] {
        need_bound(m);
        check_rows(m, rows);
        if (!m->have_params) throw Error(PDG_ESTATE, "parameters not set");
        forward(m, rows);
        if (y_out)
            HIPCHK(hipMemcpyAsync(y_out, m->Y, rows * m->d.n_out * 4, hipMemcpyDeviceToDevice, m->stream));
    });
}

pdg_status pdg_mlp_guess(pdg_mlp *m, int64_t row0, int64_t n_elem, int32_t nd, const double *u0, double *guess) {
    return mguard(m, [&] {
        need_bound(m);
        if (!u0 || !guess) throw Error(PDG_EINVAL, "NULL vector");
        if (!m->have_norm) throw Error(PDG_ESTATE, "normalisation not set");
        if (nd < 1 || nd > m->d.n_out_valid || row0 < 0 || n_elem < 1 || row0 + n_elem > m->d.max_rows)
            throw Error(PDG_EINVAL, "rows or nd out of range");
        HIPCHK(launch_guess(n_elem, nd, row0, m->d.n_out, u0, m->Y, m->ts, m->tk, guess, m->stream));
    });
}

pdg_status pdg_mlp_gradients(pdg_mlp *m, int64_t rows, int64_t n_valid, float *grad, double *loss) {
    return mguard(m, [&] {
        need_bound(m);
        check_rows(m, rows);
        if (!m->have_params) throw Error(PDG_ESTATE, "parameters not set");
        if (n_valid < 1) throw Error(PDG_EINVAL, "n_valid < 1");
        forward(m, rows);
        backward(m, rows, n_valid);
        if (grad) HIPCHK(hipMemcpyAsync(grad, m->grad, m->n_params * 4, hipMemcpyDeviceToHost, m->stream));
        HIPCHK(hipMemcpyAsync(m->loss_host, m->loss, 8, hipMemcpyDeviceToHost, m->stream));
        HIPCHK(hipStreamSynchronize(m->stream));
        if (loss) *loss = *m->loss_host;
    });
}

pdg_status pdg_mlp_train_step(pdg_mlp *m, int64_t rows, int64_t n_valid, float lr, float beta1, float beta2,
                              float eps, double *loss) {
    return mguard(m, [&] {
        need_bound(m);
        check_rows(m, rows);
        if (!m->have_params) throw Error(PDG_ESTATE, "parameters not set");
        if (n_valid < 1) throw Error(PDG_EINVAL, "n_valid < 1");
        if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
            throw Error(PDG_EINVAL, "bad Adam hyper-parameters");
        forward(m, rows);
        backward(m, rows, n_valid);
        m->t += 1;
        AdamArgs a = adam_args(m);
        a.lr = lr;
        a.b1 = beta1;
        a.b2 = beta2;
        a.eps = eps;
        a.c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)m->t)));
        a.c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)m->t)));
        HIPCHK(launch_adam(a, m->stream));
        if (loss) {
            HIPCHK(hipMemcpyAsync(m->loss_host, m->loss, 8, hipMemcpyDeviceToHost, m->stream));
            HIPCHK(hipStreamSynchronize(m->stream));
            *loss = *m->loss_host;
        }
    });
}

}  // extern "C"
