// mlp.hip -- BF16 matrix-core (MFMA) training and inference of the
// warm-start surrogate: a fully connected network with GELU hidden layers,
// mean-squared-error loss and Adam (FP32 master weights), mapping the
// control parameters of a run to its mean wall-normal profiles.
//
// Every product is one "NT" GEMM form, C[m][n] = sum_k A[m][k] * Bt[n][k],
// with A and Bt row-major and K-contiguous, computed by
// v_mfma_f32_16x16x32_bf16 (BF16 inputs, FP32 accumulation):
//   forward   Z  = X  * W       : A = X  [B x in],  Bt = Wt [out x in]
//   input grad dX = dZ * W^T    : A = dZ [B x out], Bt = W  [in x out]
//   weight grad dW = X^T * dZ   : A = Xt [in x B],  Bt = dZt [out x B]
// so weights are kept as BF16 in both [in][out] and [out][in] order and
// activations / gradients in both batch-major and feature-major order.  All
// dimensions are padded to multiples of 32 with zeros that stay zero.
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "internal.h"

using namespace nspnp;

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kMaxLayers = 8;

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float x) {
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

enum Epi { EPI_HIDDEN = 0, EPI_OUTPUT = 1, EPI_DX = 2, EPI_DW = 3 };

struct GemmArgs {
    const bf16 *A;   // [M x K]
    const bf16 *Bt;  // [N x K]
    int M, N, K;
    int epi;
    const float *bias;   // HIDDEN, OUTPUT: [N]
    float *Z;            // HIDDEN: pre-activation out [M x N]; DX: pre-activation of the layer below (read)
    bf16 *Y;             // HIDDEN: activation [M x N]; DX: dZ of the layer below [M x N]
    bf16 *Yt;            // HIDDEN / DX: the same, feature-major [N x M]
    float *C;            // OUTPUT: [M x N] FP32 output; DW: [M x N] gradient
};

// One wave per 16 x 16 output tile; 4 waves per block.
__global__ void __launch_bounds__(256) k_gemm_nt(GemmArgs g) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tiles_n = g.N / 16;
    const int tile = blockIdx.x * 4 + wave;
    if (tile >= (g.M / 16) * tiles_n) return;
    const int m0 = (tile / tiles_n) * 16, n0 = (tile % tiles_n) * 16;
    const int r = lane & 15, kc = (lane >> 4) * 8;
    const bf16 *pa = g.A + (size_t)(m0 + r) * g.K + kc;
    const bf16 *pb = g.Bt + (size_t)(n0 + r) * g.K + kc;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < g.K; k0 += 32) {
        const bf16x8 a = *(const bf16x8 *)(pa + k0);
        const bf16x8 b = *(const bf16x8 *)(pb + k0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    // lane holds rows m0 + 4 (lane / 16) + q, column n0 + lane % 16
    const int n = n0 + r;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int m = m0 + (lane >> 4) * 4 + q;
        const float v = acc[q];
        const size_t o = (size_t)m * g.N + n;
        if (g.epi == EPI_HIDDEN) {
            const float z = v + g.bias[n];
            g.Z[o] = z;
            const bf16 y = (bf16)gelu_f(z);
            g.Y[o] = y;
            g.Yt[(size_t)n * g.M + m] = y;
        } else if (g.epi == EPI_OUTPUT) {
            g.C[o] = v + g.bias[n];
        } else if (g.epi == EPI_DX) {
            const bf16 dz = (bf16)(v * gelu_grad_f(g.Z[o]));
            g.Y[o] = dz;
            g.Yt[(size_t)n * g.M + m] = dz;
        } else {
            g.C[o] = v;
        }
    }
}

// Loss and output-layer gradient: mean over the valid rows and outputs of
// (yhat - y)^2; dZ = 2 (yhat - y) / (rows * outs), zero in the padding.
__global__ void __launch_bounds__(256) k_loss(const float *yhat, const float *y, int rows, int outs, int Bp, int Np,
                                              bf16 *dz, bf16 *dzt, float *loss) {
    __shared__ float s[256];
    float acc = 0.f;
    const float scale = 2.0f / ((float)rows * (float)outs);
    for (int e = threadIdx.x; e < Bp * Np; e += blockDim.x) {
        const int m = e / Np, n = e - m * Np;
        float g = 0.f;
        if (m < rows && n < outs) {
            const float d = yhat[e] - y[(size_t)m * outs + n];
            acc += d * d;
            g = scale * d;
        }
        const bf16 gb = (bf16)g;
        dz[e] = gb;
        dzt[(size_t)n * Bp + m] = gb;
    }
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = s[0] / ((float)rows * (float)outs);
}

// bias gradient: column sums of dZ over the batch
__global__ void k_bias_grad(const bf16 *dzt, int Bp, int Np, float *db) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= Np) return;
    float s = 0.f;
    for (int m = 0; m < Bp; ++m) s += (float)dzt[(size_t)n * Bp + m];
    db[n] = s;
}

// Adam on FP32 master weights, then BF16 copies in both orders.
struct AdamArgs {
    float *w, *m, *v;   // master / moments, [in_p x out_p] followed by [out_p] bias
    const float *g;     // gradients in the same layout
    bf16 *wb, *wtb;     // BF16 weights [in_p][out_p] and [out_p][in_p]
    int in_p, out_p;
    float lr, b1, b2, eps, c1, c2;
};

__global__ void __launch_bounds__(256) k_adam(AdamArgs a) {
    const int nW = a.in_p * a.out_p;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nW + a.out_p) return;
    const float g = a.g[e];
    const float m = a.b1 * a.m[e] + (1.f - a.b1) * g;
    const float v = a.b2 * a.v[e] + (1.f - a.b2) * g * g;
    a.m[e] = m;
    a.v[e] = v;
    const float w = a.w[e] - a.lr * (m / a.c1) / (sqrtf(v / a.c2) + a.eps);
    a.w[e] = w;
    if (e < nW) {
        const int i = e / a.out_p, o = e - i * a.out_p;
        const bf16 wb = (bf16)w;
        a.wb[e] = wb;
        a.wtb[(size_t)o * a.in_p + i] = wb;
    }
}

// FP32 rows [rows x cols] -> padded BF16 [Bp x Kp] and [Kp x Bp]
__global__ void k_pack_input(const float *x, int rows, int cols, int Bp, int Kp, bf16 *xb, bf16 *xtb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= Bp * Kp) return;
    const int m = e / Kp, k = e - m * Kp;
    const float v = (m < rows && k < cols) ? x[(size_t)m * cols + k] : 0.f;
    const bf16 b = (bf16)v;
    xb[e] = b;
    xtb[(size_t)k * Bp + m] = b;
}

// copy the valid part of the FP32 output [Bp x Np] to [rows x outs]
__global__ void k_unpack_output(const float *yp, int rows, int outs, int Np, float *y) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * outs) return;
    const int m = e / outs, n = e - m * outs;
    y[e] = yp[(size_t)m * Np + n];
}

__global__ void k_sync_bf16(const float *w, int in_p, int out_p, bf16 *wb, bf16 *wtb) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= in_p * out_p) return;
    const int i = e / out_p, o = e - i * out_p;
    const bf16 b = (bf16)w[e];
    wb[e] = b;
    wtb[(size_t)o * in_p + i] = b;
}

int pad32(int n) { return (n + 31) / 32 * 32; }

}  // namespace

struct nspnp_mlp {
    int nl;                      // number of weight layers
    int sizes[kMaxLayers + 1];   // unpadded widths
    int padded[kMaxLayers + 1];  // padded to 32
    int Bp, Bmax;                // padded batch rows
    hipStream_t stream;
    float *w[kMaxLayers], *m[kMaxLayers], *v[kMaxLayers], *g[kMaxLayers];  // each [in_p*out_p + out_p]
    bf16 *wb[kMaxLayers], *wtb[kMaxLayers];
    bf16 *act[kMaxLayers + 1], *actt[kMaxLayers + 1];  // act[0] = input
    float *z[kMaxLayers];
    float *yhat;
    bf16 *dz[kMaxLayers], *dzt[kMaxLayers];
    float *loss;
    int64_t t;
};

namespace {

size_t mlp_layout(int nl, const int *sizes, int batch, nspnp_mlp *h, char *base) {
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char *p = base ? base + o : nullptr;
        o = (o + bytes + 255) & ~(size_t)255;
        return p;
    };
    int pd[kMaxLayers + 1];
    for (int l = 0; l <= nl; ++l) pd[l] = pad32(sizes[l]);
    const int Bp = pad32(batch);
    for (int l = 0; l < nl; ++l) {
        const size_t np = (size_t)pd[l] * pd[l + 1] + pd[l + 1];
        float *w = (float *)take(np * 4), *m = (float *)take(np * 4), *v = (float *)take(np * 4);
        float *g = (float *)take(np * 4);
        bf16 *wb = (bf16 *)take((size_t)pd[l] * pd[l + 1] * 2), *wtb = (bf16 *)take((size_t)pd[l] * pd[l + 1] * 2);
        if (h) {
            h->w[l] = w; h->m[l] = m; h->v[l] = v; h->g[l] = g; h->wb[l] = wb; h->wtb[l] = wtb;
        }
    }
    for (int l = 0; l <= nl; ++l) {
        bf16 *a = (bf16 *)take((size_t)Bp * pd[l] * 2), *at = (bf16 *)take((size_t)Bp * pd[l] * 2);
        if (h) { h->act[l] = a; h->actt[l] = at; }
    }
    for (int l = 0; l < nl; ++l) {
        float *zz = (float *)take((size_t)Bp * pd[l + 1] * 4);
        bf16 *d = (bf16 *)take((size_t)Bp * pd[l + 1] * 2), *dt = (bf16 *)take((size_t)Bp * pd[l + 1] * 2);
        if (h) { h->z[l] = zz; h->dz[l] = d; h->dzt[l] = dt; }
    }
    float *yh = (float *)take((size_t)Bp * pd[nl] * 4);
    float *ls = (float *)take(256);
    if (h) {
        h->yhat = yh;
        h->loss = ls;
        h->nl = nl;
        h->Bp = Bp;
        h->Bmax = batch;
        for (int l = 0; l <= nl; ++l) { h->sizes[l] = sizes[l]; h->padded[l] = pd[l]; }
    }
    return o;
}

int check_mlp(int nl, const int *sizes, int batch) {
    if (nl < 1 || nl > kMaxLayers || !sizes || batch < 1 || batch > 4096)
        return fail_code(NSPNP_ERR_INVALID, "mlp: 1..8 layers and 1..4096 rows");
    for (int l = 0; l <= nl; ++l)
        if (sizes[l] < 1 || sizes[l] > 8192) return fail_code(NSPNP_ERR_INVALID, "mlp: widths must be 1..8192");
    return NSPNP_OK;
}

#define M_TRY(expr)                                                                                       \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess) return fail_code(NSPNP_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

hipError_t gemm(nspnp_mlp *h, const GemmArgs &g) {
    const int tiles = (g.M / 16) * (g.N / 16);
    k_gemm_nt<<<(tiles + 3) / 4, 256, 0, h->stream>>>(g);
    return hipGetLastError();
}

int pack_input(nspnp_mlp *h, const float *x, int rows) {
    const int n = h->Bp * h->padded[0];
    k_pack_input<<<(n + 255) / 256, 256, 0, h->stream>>>(x, rows, h->sizes[0], h->Bp, h->padded[0], h->act[0],
                                                         h->actt[0]);
    M_TRY(hipGetLastError());
    return NSPNP_OK;
}

int forward(nspnp_mlp *h) {
    for (int l = 0; l < h->nl; ++l) {
        GemmArgs g{};
        g.A = h->act[l];
        g.Bt = h->wtb[l];
        g.M = h->Bp;
        g.N = h->padded[l + 1];
        g.K = h->padded[l];
        g.bias = h->w[l] + (size_t)h->padded[l] * h->padded[l + 1];
        if (l < h->nl - 1) {
            g.epi = EPI_HIDDEN;
            g.Z = h->z[l];
            g.Y = h->act[l + 1];
            g.Yt = h->actt[l + 1];
        } else {
            g.epi = EPI_OUTPUT;
            g.C = h->yhat;
        }
        M_TRY(gemm(h, g));
    }
    return NSPNP_OK;
}

// gradients of the loss for the rows currently packed (requires forward)
int backward(nspnp_mlp *h, const float *y, int rows) {
    const int L = h->nl;
    k_loss<<<1, 256, 0, h->stream>>>(h->yhat, y, rows, h->sizes[L], h->Bp, h->padded[L], h->dz[L - 1],
                                     h->dzt[L - 1], h->loss);
    M_TRY(hipGetLastError());
    for (int l = L - 1; l >= 0; --l) {
        const int in_p = h->padded[l], out_p = h->padded[l + 1];
        GemmArgs gw{};
        gw.A = h->actt[l];
        gw.Bt = h->dzt[l];
        gw.M = in_p;
        gw.N = out_p;
        gw.K = h->Bp;
        gw.epi = EPI_DW;
        gw.C = h->g[l];
        M_TRY(gemm(h, gw));
        k_bias_grad<<<(out_p + 255) / 256, 256, 0, h->stream>>>(h->dzt[l], h->Bp, out_p,
                                                                h->g[l] + (size_t)in_p * out_p);
        M_TRY(hipGetLastError());
        if (l > 0) {
            GemmArgs gx{};
            gx.A = h->dz[l];
            gx.Bt = h->wb[l];
            gx.M = h->Bp;
            gx.N = in_p;
            gx.K = out_p;
            gx.epi = EPI_DX;
            gx.Z = h->z[l - 1];
            gx.Y = h->dz[l - 1];
            gx.Yt = h->dzt[l - 1];
            M_TRY(gemm(h, gx));
        }
    }
    return NSPNP_OK;
}

}  // namespace

extern "C" {

size_t nspnp_mlp_workspace_bytes(int32_t n_layers, const int32_t *sizes, int32_t max_rows) {
    if (check_mlp(n_layers, sizes, max_rows)) return 0;
    return mlp_layout(n_layers, sizes, max_rows, nullptr, nullptr);
}

int nspnp_mlp_init(int32_t n_layers, const int32_t *sizes, int32_t max_rows, const float *host_params,
                   void *dev_workspace, size_t bytes, void *hip_stream, nspnp_mlp **out) {
    if (!out || !host_params) return fail_code(NSPNP_ERR_INVALID, "mlp_init: NULL argument");
    *out = nullptr;
    int rc = check_mlp(n_layers, sizes, max_rows);
    if (rc) return rc;
    const size_t need = mlp_layout(n_layers, sizes, max_rows, nullptr, nullptr);
    if (!dev_workspace || bytes < need || ((uintptr_t)dev_workspace & 255))
        return fail_code(NSPNP_ERR_WORKSPACE, "mlp workspace missing, too small or misaligned");
    nspnp_mlp *h = new nspnp_mlp();
    mlp_layout(n_layers, sizes, max_rows, h, (char *)dev_workspace);
    h->stream = (hipStream_t)hip_stream;
    h->t = 0;
    // zero everything (padding must stay zero), then the parameters
    std::vector<char> zeros(need, 0);
    hipError_t e = hipMemcpyAsync(dev_workspace, zeros.data(), need, hipMemcpyHostToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) {
        delete h;
        return fail_code(NSPNP_ERR_HIP, std::string("mlp init: ") + hipGetErrorString(e));
    }
    *out = h;
    return nspnp_mlp_set_params(h, host_params);
}

// parameters as W_0 [in x out] row-major, b_0 [out], W_1, b_1, ... (FP32)
int nspnp_mlp_set_params(nspnp_mlp *h, const float *host_params) {
    if (!h || !host_params) return fail_code(NSPNP_ERR_INVALID, "mlp_set_params: NULL argument");
    const float *src = host_params;
    for (int l = 0; l < h->nl; ++l) {
        const int in = h->sizes[l], out = h->sizes[l + 1], in_p = h->padded[l], out_p = h->padded[l + 1];
        std::vector<float> buf((size_t)in_p * out_p + out_p, 0.f);
        for (int i = 0; i < in; ++i)
            for (int o = 0; o < out; ++o) buf[(size_t)i * out_p + o] = src[(size_t)i * out + o];
        src += (size_t)in * out;
        for (int o = 0; o < out; ++o) buf[(size_t)in_p * out_p + o] = src[o];
        src += out;
        M_TRY(hipMemcpyAsync(h->w[l], buf.data(), buf.size() * 4, hipMemcpyHostToDevice, h->stream));
        M_TRY(hipStreamSynchronize(h->stream));
        k_sync_bf16<<<(in_p * out_p + 255) / 256, 256, 0, h->stream>>>(h->w[l], in_p, out_p, h->wb[l], h->wtb[l]);
        M_TRY(hipGetLastError());
    }
    M_TRY(hipStreamSynchronize(h->stream));
    return NSPNP_OK;
}

int nspnp_mlp_get_params(nspnp_mlp *h, float *host_params, float *host_grads) {
    if (!h || (!host_params && !host_grads)) return fail_code(NSPNP_ERR_INVALID, "mlp_get_params: NULL argument");
    size_t off = 0;
    for (int l = 0; l < h->nl; ++l) {
        const int in = h->sizes[l], out = h->sizes[l + 1], in_p = h->padded[l], out_p = h->padded[l + 1];
        std::vector<float> buf((size_t)in_p * out_p + out_p);
        for (int which = 0; which < 2; ++which) {
            float *dst = which == 0 ? host_params : host_grads;
            if (!dst) continue;
            M_TRY(hipMemcpyAsync(buf.data(), which == 0 ? h->w[l] : h->g[l], buf.size() * 4, hipMemcpyDeviceToHost,
                                 h->stream));
            M_TRY(hipStreamSynchronize(h->stream));
            for (int i = 0; i < in; ++i)
                for (int o = 0; o < out; ++o) dst[off + (size_t)i * out + o] = buf[(size_t)i * out_p + o];
            for (int o = 0; o < out; ++o) dst[off + (size_t)in * out + o] = buf[(size_t)in_p * out_p + o];
        }
        off += (size_t)in * out + out;
    }
    return NSPNP_OK;
}

int nspnp_mlp_forward(nspnp_mlp *h, const float *dev_x, int32_t rows, float *dev_y) {
    if (!h || !dev_x || !dev_y || rows < 1 || rows > h->Bmax) return fail_code(NSPNP_ERR_INVALID, "mlp_forward: bad rows");
    int rc = pack_input(h, dev_x, rows);
    if (rc || (rc = forward(h))) return rc;
    const int n = rows * h->sizes[h->nl];
    k_unpack_output<<<(n + 255) / 256, 256, 0, h->stream>>>(h->yhat, rows, h->sizes[h->nl], h->padded[h->nl], dev_y);
    M_TRY(hipGetLastError());
    return NSPNP_OK;
}

int nspnp_mlp_gradients(nspnp_mlp *h, const float *dev_x, const float *dev_y, int32_t rows, float *loss) {
    if (!h || !dev_x || !dev_y || rows < 1 || rows > h->Bmax) return fail_code(NSPNP_ERR_INVALID, "mlp_gradients: bad rows");
    int rc = pack_input(h, dev_x, rows);
    if (rc || (rc = forward(h)) || (rc = backward(h, dev_y, rows))) return rc;
    if (loss) {
        M_TRY(hipMemcpyAsync(loss, h->loss, 4, hipMemcpyDeviceToHost, h->stream));
        M_TRY(hipStreamSynchronize(h->stream));
    }
    return NSPNP_OK;
}

int nspnp_mlp_train_step(nspnp_mlp *h, const float *dev_x, const float *dev_y, int32_t rows, float lr,
                         float *dev_loss) {
    if (!h || !dev_x || !dev_y || rows < 1 || rows > h->Bmax) return fail_code(NSPNP_ERR_INVALID, "mlp_train_step: bad rows");
    int rc = pack_input(h, dev_x, rows);
    if (rc || (rc = forward(h)) || (rc = backward(h, dev_y, rows))) return rc;
    h->t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    AdamArgs a{};
    a.lr = lr;
    a.b1 = b1;
    a.b2 = b2;
    a.eps = 1e-8f;
    a.c1 = (float)(1.0 - std::pow(0.9, (double)h->t));
    a.c2 = (float)(1.0 - std::pow(0.999, (double)h->t));
    for (int l = 0; l < h->nl; ++l) {
        a.w = h->w[l]; a.m = h->m[l]; a.v = h->v[l]; a.g = h->g[l];
        a.wb = h->wb[l]; a.wtb = h->wtb[l];
        a.in_p = h->padded[l];
        a.out_p = h->padded[l + 1];
        const int n = a.in_p * a.out_p + a.out_p;
        k_adam<<<(n + 255) / 256, 256, 0, h->stream>>>(a);
        M_TRY(hipGetLastError());
    }
    if (dev_loss) M_TRY(hipMemcpyAsync(dev_loss, h->loss, 4, hipMemcpyDeviceToDevice, h->stream));
    return NSPNP_OK;
}

int nspnp_mlp_sync(nspnp_mlp *h) {
    if (!h) return fail_code(NSPNP_ERR_INVALID, "mlp is NULL");
    M_TRY(hipStreamSynchronize(h->stream));
    return NSPNP_OK;
}

void nspnp_mlp_destroy(nspnp_mlp *h) { delete h; }

}  // extern "C"
