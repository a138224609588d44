// Multilayer perceptron for the learned warm start of the batched sweep: dense layers with tanh
// on every hidden layer and a linear output, FP32, trained with mean-squared error and Adam,
// forward and backward passes as HIP kernels.  The layers are small (a few hundred units), so
// each output element is one thread with a loop over the inputs; every reduction (gradients
// over the batch, the loss) runs in a fixed order, so training is deterministic.

#include <hip/hip_runtime.h>

#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "../../include/pplbm.h"

namespace {

// Y[b][o] = act(sum_i X[b][i] W[o][i] + bias[o])
__global__ void dense_forward(const float *__restrict__ X, const float *__restrict__ W,
                              const float *__restrict__ bias, float *__restrict__ Y, int B,
                              int in, int out, int tanh_act) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (o >= out || b >= B) return;
    const float *x = X + (size_t)b * in;
    const float *w = W + (size_t)o * in;
    float acc = bias[o];
    for (int i = 0; i < in; ++i) acc = fmaf(x[i], w[i], acc);
    Y[(size_t)b * out + o] = tanh_act ? tanhf(acc) : acc;
}

// dZ = dY * (1 - Y^2) for a tanh layer (in place on dY).
__global__ void tanh_backward(float *__restrict__ dY, const float *__restrict__ Y, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dY[i] *= 1.0f - Y[i] * Y[i];
}

// dX[b][i] = sum_o dZ[b][o] W[o][i]
__global__ void dense_backward_input(const float *__restrict__ dZ, const float *__restrict__ W,
                                     float *__restrict__ dX, int B, int in, int out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = blockIdx.y;
    if (i >= in || b >= B) return;
    const float *dz = dZ + (size_t)b * out;
    float acc = 0.0f;
    for (int o = 0; o < out; ++o) acc = fmaf(dz[o], W[(size_t)o * in + i], acc);
    dX[(size_t)b * in + i] = acc;
}

// dW[o][i] = sum_b dZ[b][o] X[b][i]; dbias[o] = sum_b dZ[b][o] (threads i == in do the bias).
__global__ void dense_backward_weights(const float *__restrict__ dZ, const float *__restrict__ X,
                                       float *__restrict__ dW, float *__restrict__ dbias, int B,
                                       int in, int out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int o = blockIdx.y;
    if (i > in || o >= out) return;
    float acc = 0.0f;
    if (i < in) {
        for (int b = 0; b < B; ++b) acc = fmaf(dZ[(size_t)b * out + o], X[(size_t)b * in + i], acc);
        dW[(size_t)o * in + i] = acc;
    } else {
        for (int b = 0; b < B; ++b) acc += dZ[(size_t)b * out + o];
        dbias[o] = acc;
    }
}

// Mean-squared error over B x n outputs: dY = 2 (Y - T) / (B n); per-block partial sums of
// (Y - T)^2 in a fixed tree.
__global__ void __launch_bounds__(256) mse_grad(const float *__restrict__ Y, const float *__restrict__ T,
                                                float *__restrict__ dY, size_t n_all,
                                                float *__restrict__ partial) {
    __shared__ float sh[256];
    const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
    float d = 0.0f;
    if (i < n_all) {
        d = Y[i] - T[i];
        dY[i] = 2.0f * d / (float)n_all;
    }
    sh[threadIdx.x] = d * d;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void sum_partials(const float *__restrict__ partial, int n, float scale,
                             float *__restrict__ out) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double acc = 0.0;
        for (int i = 0; i < n; ++i) acc += partial[i];
        out[0] = (float)(acc * scale);
    }
}

// Adam (Kingma & Ba) with bias correction folded into the step size.
__global__ void adam_update(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, size_t n, float lr_t, float b1, float b2,
                            float eps) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr_t * mi / (sqrtf(vi) + eps);
}

}  // namespace

struct lbm_mlp {
    std::vector<int> dims;
    size_t nparam = 0;
    std::vector<size_t> woff, boff;  // offsets of W_l and b_l in the flat parameter vector
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    std::vector<float *> act;        // activations per layer (act[0] unused: input is external)
    float *dbuf[2] = {nullptr, nullptr};
    float *partial = nullptr, *loss = nullptr;
    int cap = 0;                     // batch capacity of the activation buffers
    long long t = 0;                 // Adam step count
    std::string err;
};

namespace {

int mfail(lbm_mlp *n, int code, const std::string &m) {
    if (n) n->err = m;
    return code;
}

#define MHIP(n, call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) return mfail(n, LBM_EHIP, std::string(#call ": ") + hipGetErrorString(e_)); \
    } while (0)

int widest(const lbm_mlp *n) {
    int w = 0;
    for (int d : n->dims) w = d > w ? d : w;
    return w;
}

int ensure_cap(lbm_mlp *n, int B) {
    if (B <= n->cap) return LBM_OK;
    for (float *p : n->act)
        if (p) (void)hipFree(p);
    for (float *&p : n->dbuf)
        if (p) (void)hipFree(p), p = nullptr;
    if (n->partial) (void)hipFree(n->partial);
    n->act.assign(n->dims.size(), nullptr);
    const size_t w = widest(n);
    bool ok = true;
    for (size_t l = 1; l < n->dims.size() && ok; ++l)
        ok = hipMalloc(&n->act[l], (size_t)B * n->dims[l] * sizeof(float)) == hipSuccess;
    ok = ok && hipMalloc(&n->dbuf[0], (size_t)B * w * sizeof(float)) == hipSuccess &&
         hipMalloc(&n->dbuf[1], (size_t)B * w * sizeof(float)) == hipSuccess &&
         hipMalloc(&n->partial, ((size_t)B * n->dims.back() + 255) / 256 * sizeof(float)) == hipSuccess;
    if (!ok) {
        (void)hipGetLastError();
        n->cap = 0;
        return mfail(n, LBM_ENOMEM, "activation buffers");
    }
    n->cap = B;
    return LBM_OK;
}

int forward(lbm_mlp *n, const float *x, int B, hipStream_t s) {
    const int L = (int)n->dims.size() - 1;
    const float *in = x;
    for (int l = 0; l < L; ++l) {
        const int di = n->dims[l], dout = n->dims[l + 1];
        hipLaunchKernelGGL(dense_forward, dim3((dout + 63) / 64, B), dim3(64), 0, s, in,
                           n->params + n->woff[l], n->params + n->boff[l], n->act[l + 1], B, di,
                           dout, l + 1 < L ? 1 : 0);
        MHIP(n, hipGetLastError());
        in = n->act[l + 1];
    }
    return LBM_OK;
}

// Gradient of sum(dy * y) with respect to every parameter into n->grads; dy is consumed.
int backward(lbm_mlp *n, const float *x, const float *dy, int B, hipStream_t s) {
    const int L = (int)n->dims.size() - 1;
    const size_t nout = (size_t)B * n->dims[L];
    MHIP(n, hipMemcpyAsync(n->dbuf[0], dy, nout * sizeof(float), hipMemcpyDeviceToDevice, s));
    int cur = 0;
    for (int l = L - 1; l >= 0; --l) {
        const int di = n->dims[l], dout = n->dims[l + 1];
        float *dz = n->dbuf[cur];
        if (l + 1 < L) {  // hidden layer: through tanh
            const size_t cnt = (size_t)B * dout;
            hipLaunchKernelGGL(tanh_backward, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, dz,
                               n->act[l + 1], cnt);
            MHIP(n, hipGetLastError());
        }
        const float *xin = l == 0 ? x : n->act[l];
        hipLaunchKernelGGL(dense_backward_weights, dim3((di + 1 + 63) / 64, dout), dim3(64), 0, s, dz,
                           xin, n->grads + n->woff[l], n->grads + n->boff[l], B, di, dout);
        MHIP(n, hipGetLastError());
        if (l > 0) {
            hipLaunchKernelGGL(dense_backward_input, dim3((di + 63) / 64, B), dim3(64), 0, s, dz,
                               n->params + n->woff[l], n->dbuf[1 - cur], B, di, dout);
            MHIP(n, hipGetLastError());
            cur = 1 - cur;
        }
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_mlp_create(int nlayers, const int *dims, lbm_mlp_t **out) {
    if (!out || nlayers < 1 || !dims) return LBM_EINVAL;
    *out = nullptr;
    for (int l = 0; l <= nlayers; ++l)
        if (dims[l] < 1 || dims[l] > 4096) return LBM_EINVAL;
    lbm_mlp *n = new (std::nothrow) lbm_mlp();
    if (!n) return LBM_ENOMEM;
    n->dims.assign(dims, dims + nlayers + 1);
    for (int l = 0; l < nlayers; ++l) {
        n->woff.push_back(n->nparam);
        n->nparam += (size_t)dims[l] * dims[l + 1];
        n->boff.push_back(n->nparam);
        n->nparam += dims[l + 1];
    }
    const size_t bytes = n->nparam * sizeof(float);
    if (hipMalloc(&n->params, bytes) != hipSuccess || hipMalloc(&n->grads, bytes) != hipSuccess ||
        hipMalloc(&n->m, bytes) != hipSuccess || hipMalloc(&n->v, bytes) != hipSuccess ||
        hipMalloc(&n->loss, sizeof(float)) != hipSuccess ||
        hipMemset(n->params, 0, bytes) != hipSuccess || hipMemset(n->m, 0, bytes) != hipSuccess ||
        hipMemset(n->v, 0, bytes) != hipSuccess) {
        (void)hipGetLastError();
        lbm_mlp_destroy(n);
        return LBM_ENOMEM;
    }
    *out = n;
    return LBM_OK;
}

void lbm_mlp_destroy(lbm_mlp_t *n) {
    if (!n) return;
    (void)hipDeviceSynchronize();
    for (float *p : {n->params, n->grads, n->m, n->v, n->loss, n->partial, n->dbuf[0], n->dbuf[1]})
        if (p) (void)hipFree(p);
    for (float *p : n->act)
        if (p) (void)hipFree(p);
    delete n;
}

size_t lbm_mlp_param_count(const lbm_mlp_t *n) { return n ? n->nparam : 0; }

int lbm_mlp_set_params(lbm_mlp_t *n, const float *host) {
    if (!n || !host) return LBM_EINVAL;
    MHIP(n, hipMemcpy(n->params, host, n->nparam * sizeof(float), hipMemcpyHostToDevice));
    MHIP(n, hipMemset(n->m, 0, n->nparam * sizeof(float)));
    MHIP(n, hipMemset(n->v, 0, n->nparam * sizeof(float)));
    n->t = 0;
    return LBM_OK;
}

int lbm_mlp_get_params(lbm_mlp_t *n, float *host) {
    if (!n || !host) return LBM_EINVAL;
    MHIP(n, hipMemcpy(host, n->params, n->nparam * sizeof(float), hipMemcpyDeviceToHost));
    return LBM_OK;
}

int lbm_mlp_forward(lbm_mlp_t *n, const float *x, int batch, float *y, void *stream) {
    if (!n || !x || !y || batch < 1) return LBM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int rc = ensure_cap(n, batch);
    if (rc) return rc;
    rc = forward(n, x, batch, s);
    if (rc) return rc;
    MHIP(n, hipMemcpyAsync(y, n->act.back(), (size_t)batch * n->dims.back() * sizeof(float),
                           hipMemcpyDeviceToDevice, s));
    return LBM_OK;
}

int lbm_mlp_gradient(lbm_mlp_t *n, const float *x, const float *dy, int batch, float *grad,
                     void *stream) {
    if (!n || !x || !dy || !grad || batch < 1) return LBM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int rc = ensure_cap(n, batch);
    if (rc) return rc;
    rc = forward(n, x, batch, s);
    if (rc) return rc;
    rc = backward(n, x, dy, batch, s);
    if (rc) return rc;
    MHIP(n, hipMemcpyAsync(grad, n->grads, n->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
    return LBM_OK;
}

int lbm_mlp_train_step(lbm_mlp_t *n, const float *x, const float *target, int batch, float lr,
                       float *loss_out, void *stream) {
    if (!n || !x || !target || batch < 1 || !(lr > 0)) return LBM_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int rc = ensure_cap(n, batch);
    if (rc) return rc;
    rc = forward(n, x, batch, s);
    if (rc) return rc;
    const size_t nout = (size_t)batch * n->dims.back();
    const int nb = (int)((nout + 255) / 256);
    // dbuf[0] would be overwritten by backward's copy; compute dY into dbuf[1], then copy.
    hipLaunchKernelGGL(mse_grad, dim3(nb), dim3(256), 0, s, n->act.back(), target, n->dbuf[1], nout,
                       n->partial);
    MHIP(n, hipGetLastError());
    hipLaunchKernelGGL(sum_partials, dim3(1), dim3(64), 0, s, n->partial, nb, 1.0f / (float)nout, n->loss);
    MHIP(n, hipGetLastError());
    rc = backward(n, x, n->dbuf[1], batch, s);
    if (rc) return rc;
    ++n->t;
    const float b1 = 0.9f, b2 = 0.999f;
    const float lr_t = lr * (float)(std::sqrt(1.0 - std::pow(b2, (double)n->t)) / (1.0 - std::pow(b1, (double)n->t)));
    hipLaunchKernelGGL(adam_update, dim3((unsigned)((n->nparam + 255) / 256)), dim3(256), 0, s, n->params,
                       n->grads, n->m, n->v, n->nparam, lr_t, b1, b2, 1e-8f);
    MHIP(n, hipGetLastError());
    if (loss_out) {
        MHIP(n, hipMemcpyAsync(loss_out, n->loss, sizeof(float), hipMemcpyDeviceToHost, s));
        MHIP(n, hipStreamSynchronize(s));
    }
    return LBM_OK;
}

const char *lbm_mlp_last_error(const lbm_mlp_t *n) { return n ? n->err.c_str() : ""; }

}  // extern "C"
