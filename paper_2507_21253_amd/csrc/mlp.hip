// The learned path selector and nnz predictor: a 32-64-64-5 multilayer
// perceptron in float32, trained on the GPU.  Forward pass, back-propagation
// and Adam are plain kernels: the network is tiny (6,597 parameters), so each
// sample gets one 64-lane block for the forward and delta passes, and each
// parameter one lane that sums its gradient over the batch in sample order
// (deterministic).
//
//   x_n = (x - mu) / sd;  h1 = relu(W1 x_n + b1);  h2 = relu(W2 h1 + b2);
//   z = W3 h2 + b3, z[0..3] path logits, z[4] log compression ratio;
//   loss = mean(-log softmax(z[0..3])[y]) + lam * mean((z[4] - t)^2).
#include "internal.h"

namespace hcsp {

constexpr int kIn = HCSP_MLP_NIN, kH = HCSP_MLP_NH, kOut = HCSP_MLP_NOUT, kCls = HCSP_MLP_NCLS;
constexpr int oW1 = 0, oB1 = oW1 + kH * kIn, oW2 = oB1 + kH, oB2 = oW2 + kH * kH, oW3 = oB2 + kH,
              oB3 = oW3 + kOut * kH, kParams = oB3 + kOut;
static_assert(kParams == HCSP_MLP_NPARAMS, "parameter layout");
constexpr int aXN = 0, aA1 = kIn, aA2 = kIn + kH, kAct = kIn + 2 * kH;  // per-sample activations
constexpr int dZ = 0, dA2 = kOut, dA1 = kOut + kH, kDelta = kOut + 2 * kH;
static_assert(kAct == HCSP_MLP_NACT && kDelta == HCSP_MLP_NDELTA, "activation layout");

// one block of 64 lanes per sample
__global__ void __launch_bounds__(64) k_mlp_forward(const float *__restrict__ P, const float *__restrict__ norm,
                                                    const float *__restrict__ X, int B, float *__restrict__ Z,
                                                    float *__restrict__ act)
{
    __shared__ float xn[kIn], h1[kH], h2[kH];
    const int b = blockIdx.x, u = threadIdx.x;
    if (b >= B) return;
    if (u < kIn) xn[u] = (X[(int64_t)b * kIn + u] - norm[u]) / norm[kIn + u];
    __syncthreads();
    float s = P[oB1 + u];
    for (int i = 0; i < kIn; ++i) s = __fmaf_rn(P[oW1 + u * kIn + i], xn[i], s);
    h1[u] = fmaxf(s, 0.0f);
    if (act) {
        if (u < kIn) act[(int64_t)b * kAct + aXN + u] = xn[u];
        act[(int64_t)b * kAct + aA1 + u] = s;
    }
    __syncthreads();
    float s2 = P[oB2 + u];
    for (int v = 0; v < kH; ++v) s2 = __fmaf_rn(P[oW2 + u * kH + v], h1[v], s2);
    h2[u] = fmaxf(s2, 0.0f);
    if (act) act[(int64_t)b * kAct + aA2 + u] = s2;
    __syncthreads();
    if (u < kOut) {
        float z = P[oB3 + u];
        for (int v = 0; v < kH; ++v) z = __fmaf_rn(P[oW3 + u * kH + v], h2[v], z);
        Z[(int64_t)b * kOut + u] = z;
    }
}

// Per-sample loss and deltas: dz = d loss / dz, then back through both
// hidden layers (da = d loss / d pre-activation).
__global__ void __launch_bounds__(64) k_mlp_delta(const float *__restrict__ P, const float *__restrict__ act,
                                                  const float *__restrict__ Z, const int32_t *__restrict__ y,
                                                  const float *__restrict__ t, int B, float lam,
                                                  float *__restrict__ delta, float *__restrict__ loss)
{
    __shared__ float dz[kOut], da2[kH];
    const int b = blockIdx.x, u = threadIdx.x;
    if (b >= B) return;
    const float *z = Z + (int64_t)b * kOut;
    float *d = delta + (int64_t)b * kDelta;
    if (u == 0) {
        float m = z[0];
        for (int c = 1; c < kCls; ++c) m = fmaxf(m, z[c]);
        float se = 0.0f;
        for (int c = 0; c < kCls; ++c) se += expf(z[c] - m);
        const int yc = y[b];
        for (int c = 0; c < kCls; ++c) dz[c] = (expf(z[c] - m) / se - (c == yc ? 1.0f : 0.0f)) / (float)B;
        const float r = z[kCls] - t[b];
        dz[kCls] = 2.0f * lam * r / (float)B;
        loss[b] = (m + logf(se) - z[yc]) + lam * r * r;
        for (int o = 0; o < kOut; ++o) d[dZ + o] = dz[o];
    }
    __syncthreads();
    float g = 0.0f;
    for (int o = 0; o < kOut; ++o) g = __fmaf_rn(P[oW3 + o * kH + u], dz[o], g);
    const float a2 = act[(int64_t)b * kAct + aA2 + u];
    da2[u] = a2 > 0.0f ? g : 0.0f;
    d[dA2 + u] = da2[u];
    __syncthreads();
    float g1 = 0.0f;
    for (int v = 0; v < kH; ++v) g1 = __fmaf_rn(P[oW2 + v * kH + u], da2[v], g1);
    const float a1 = act[(int64_t)b * kAct + aA1 + u];
    d[dA1 + u] = a1 > 0.0f ? g1 : 0.0f;
}

// One lane per parameter: its gradient summed over the batch in sample order.
__global__ void __launch_bounds__(256) k_mlp_param_grad(const float *__restrict__ act,
                                                        const float *__restrict__ delta, int B,
                                                        float *__restrict__ grad)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kParams) return;
    float s = 0.0f;
    if (k < oB1) {                      // W1[u][i] : da1[u] * xn[i]
        const int u = (k - oW1) / kIn, i = (k - oW1) % kIn;
        for (int b = 0; b < B; ++b)
            s = __fmaf_rn(delta[(int64_t)b * kDelta + dA1 + u], act[(int64_t)b * kAct + aXN + i], s);
    } else if (k < oW2) {               // b1[u] : da1[u]
        const int u = k - oB1;
        for (int b = 0; b < B; ++b) s += delta[(int64_t)b * kDelta + dA1 + u];
    } else if (k < oB2) {               // W2[u][v] : da2[u] * relu(a1[v])
        const int u = (k - oW2) / kH, v = (k - oW2) % kH;
        for (int b = 0; b < B; ++b)
            s = __fmaf_rn(delta[(int64_t)b * kDelta + dA2 + u], fmaxf(act[(int64_t)b * kAct + aA1 + v], 0.0f), s);
    } else if (k < oW3) {               // b2[u] : da2[u]
        const int u = k - oB2;
        for (int b = 0; b < B; ++b) s += delta[(int64_t)b * kDelta + dA2 + u];
    } else if (k < oB3) {               // W3[o][v] : dz[o] * relu(a2[v])
        const int o = (k - oW3) / kH, v = (k - oW3) % kH;
        for (int b = 0; b < B; ++b)
            s = __fmaf_rn(delta[(int64_t)b * kDelta + dZ + o], fmaxf(act[(int64_t)b * kAct + aA2 + v], 0.0f), s);
    } else {                            // b3[o] : dz[o]
        const int o = k - oB3;
        for (int b = 0; b < B; ++b) s += delta[(int64_t)b * kDelta + dZ + o];
    }
    grad[k] = s;
}

__global__ void __launch_bounds__(256) k_mlp_adam(float *__restrict__ P, const float *__restrict__ g,
                                                  float *__restrict__ m, float *__restrict__ v, float lr,
                                                  float b1, float b2, float eps, float c1, float c2)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kParams) return;
    const float gk = g[k];
    const float mk = b1 * m[k] + (1.0f - b1) * gk;
    const float vk = b2 * v[k] + (1.0f - b2) * gk * gk;
    m[k] = mk;
    v[k] = vk;
    P[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
}

}  // namespace hcsp

using namespace hcsp;

extern "C" {

int hcsp_mlp_forward(const float *params_d, const float *norm_d, const float *X_d, int32_t B, float *Z_d,
                     float *act_d, void *stream)
{
    clear_error();
    if (B < 0 || (B > 0 && (!params_d || !norm_d || !X_d || !Z_d))) return fail(HCSP_E_INVALID, "bad arguments");
    if (B == 0) return HCSP_OK;
    hipLaunchKernelGGL(k_mlp_forward, dim3(B), dim3(64), 0, (hipStream_t)stream, params_d, norm_d, X_d, B, Z_d,
                       act_d);
    HCSP_HIP(hipGetLastError());
    return HCSP_OK;
}

int hcsp_mlp_backward(const float *params_d, const float *act_d, const float *Z_d, const int32_t *y_d,
                      const float *t_d, int32_t B, float lam, float *delta_d, float *loss_d, float *grad_d,
                      void *stream)
{
    clear_error();
    if (B <= 0 || !params_d || !act_d || !Z_d || !y_d || !t_d || !delta_d || !loss_d || !grad_d)
        return fail(HCSP_E_INVALID, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    hipLaunchKernelGGL(k_mlp_delta, dim3(B), dim3(64), 0, s, params_d, act_d, Z_d, y_d, t_d, B, lam, delta_d, loss_d);
    HCSP_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_mlp_param_grad, dim3((kParams + 255) / 256), dim3(256), 0, s, act_d, delta_d, B, grad_d);
    HCSP_HIP(hipGetLastError());
    return HCSP_OK;
}

int hcsp_mlp_adam(float *params_d, const float *grad_d, float *m_d, float *v_d, int32_t step, float lr, float beta1,
                  float beta2, float eps, void *stream)
{
    clear_error();
    if (!params_d || !grad_d || !m_d || !v_d || step < 1) return fail(HCSP_E_INVALID, "bad arguments");
    const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + 255) / 256), dim3(256), 0, (hipStream_t)stream, params_d, grad_d,
                       m_d, v_d, lr, beta1, beta2, eps, c1, c2);
    HCSP_HIP(hipGetLastError());
    return HCSP_OK;
}

}  // extern "C"
