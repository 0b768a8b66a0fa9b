// Learned iteration schedule: a small multilayer perceptron with its own forward,
// backward and optimizer kernels (FP32).
//
//   x[16] -> z1 = W1 x + b1 -> h1 = silu(z1) -> z2 = W2 h1 + b2 -> h2 = silu(z2)
//         -> y = W3 h2 + b3          (hidden width 64, nout <= 4 outputs)
//
// Forward: one sample per thread, parameters broadcast from LDS.
// Backward: a workgroup takes 64 samples, forms the per-sample vectors
// (h1, h2, dz1, dz2) in LDS, and every thread then sums a fixed subset of the
// parameter gradients over those samples; per-workgroup partial gradients are
// summed over workgroups in index order by a second kernel, so the gradient is
// bitwise reproducible.
#include "common.h"

namespace nolsm {

constexpr int NIN = NOLSM_NFEAT;
constexpr int NH = NOLSM_MLP_HIDDEN;
constexpr int MAXOUT = NOLSM_MLP_MAXOUT;
constexpr int OFF_W1 = 0, OFF_B1 = NH * NIN, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH,
              OFF_W3 = OFF_B2 + NH;
constexpr int BWD_SAMPLES = 64;

__host__ __device__ constexpr int mlp_params(int nout) { return OFF_W3 + nout * NH + nout; }

__device__ __forceinline__ float sigmoidf_(float z) { return 1.0f / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu(float z) { return z * sigmoidf_(z); }
__device__ __forceinline__ float dsilu(float z) {
  const float s = sigmoidf_(z);
  return s * (1.0f + z * (1.0f - s));
}

__global__ __launch_bounds__(256) void mlp_forward_kernel(const float *__restrict__ prm, int nout,
                                                          const float *__restrict__ x,
                                                          int64_t B, float *__restrict__ y,
                                                          float *__restrict__ act) {
  __shared__ float sp[mlp_params(MAXOUT)];
  const int P = mlp_params(nout);
  for (int i = threadIdx.x; i < P; i += 256) sp[i] = prm[i];
  __syncthreads();
  const int64_t s = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (s >= B) return;
  float xi[NIN], h1[NH];
#pragma unroll
  for (int i = 0; i < NIN; ++i) xi[i] = x[s * NIN + i];
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    float z = sp[OFF_B1 + j];
#pragma unroll
    for (int i = 0; i < NIN; ++i) z += sp[OFF_W1 + j * NIN + i] * xi[i];
    if (act) act[s * 2 * NH + j] = z;
    h1[j] = silu(z);
  }
  float out[MAXOUT];
#pragma unroll
  for (int o = 0; o < MAXOUT; ++o) out[o] = (o < nout) ? sp[OFF_W3 + nout * NH + o] : 0.0f;
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    float z = sp[OFF_B2 + j];
#pragma unroll
    for (int i = 0; i < NH; ++i) z += sp[OFF_W2 + j * NH + i] * h1[i];
    if (act) act[s * 2 * NH + NH + j] = z;
    const float h = silu(z);
#pragma unroll
    for (int o = 0; o < MAXOUT; ++o)
      if (o < nout) out[o] += sp[OFF_W3 + o * NH + j] * h;
  }
#pragma unroll
  for (int o = 0; o < MAXOUT; ++o)
    if (o < nout) y[s * nout + o] = out[o];
}

__global__ __launch_bounds__(256) void mlp_backward_kernel(
    const float *__restrict__ prm, int nout, const float *__restrict__ x,
    const float *__restrict__ act, const float *__restrict__ dy, int64_t B,
    float *__restrict__ partial) {
  __shared__ float sp[mlp_params(MAXOUT)];
  __shared__ float sx[BWD_SAMPLES][NIN];
  __shared__ float sh1[BWD_SAMPLES][NH + 1];
  __shared__ float sh2[BWD_SAMPLES][NH + 1];
  __shared__ float sd1[BWD_SAMPLES][NH + 1];
  __shared__ float sd2[BWD_SAMPLES][NH + 1];
  __shared__ float sdy[BWD_SAMPLES][MAXOUT];
  const int P = mlp_params(nout);
  for (int i = threadIdx.x; i < P; i += 256) sp[i] = prm[i];
  const int64_t s0 = (int64_t)blockIdx.x * BWD_SAMPLES;
  __syncthreads();
  if (threadIdx.x < BWD_SAMPLES) {
    const int t = threadIdx.x;
    const int64_t s = s0 + t;
    const bool ok = s < B;
    float d2[NH];
#pragma unroll
    for (int i = 0; i < NIN; ++i) sx[t][i] = ok ? x[s * NIN + i] : 0.0f;
#pragma unroll
    for (int o = 0; o < MAXOUT; ++o) sdy[t][o] = (ok && o < nout) ? dy[s * nout + o] : 0.0f;
#pragma unroll
    for (int j = 0; j < NH; ++j) {
      const float z1 = ok ? act[s * 2 * NH + j] : 0.0f;
      const float z2 = ok ? act[s * 2 * NH + NH + j] : 0.0f;
      sh1[t][j] = ok ? silu(z1) : 0.0f;
      sh2[t][j] = ok ? silu(z2) : 0.0f;
      float g = 0.0f;
#pragma unroll
      for (int o = 0; o < MAXOUT; ++o)
        if (o < nout) g += sp[OFF_W3 + o * NH + j] * sdy[t][o];
      d2[j] = g * dsilu(z2);
      sd2[t][j] = d2[j];
    }
#pragma unroll
    for (int i = 0; i < NH; ++i) {
      float g = 0.0f;
#pragma unroll
      for (int j = 0; j < NH; ++j) g += sp[OFF_W2 + j * NH + i] * d2[j];
      const float z1 = ok ? act[s * 2 * NH + i] : 0.0f;
      sd1[t][i] = g * dsilu(z1);
    }
  }
  __syncthreads();
  float *out = partial + (int64_t)blockIdx.x * P;
  for (int p = threadIdx.x; p < P; p += 256) {
    float g = 0.0f;
    if (p < OFF_B1) {                       // W1[j][i]
      const int j = p / NIN, i = p % NIN;
      for (int t = 0; t < BWD_SAMPLES; ++t) g += sd1[t][j] * sx[t][i];
    } else if (p < OFF_W2) {                // b1[j]
      const int j = p - OFF_B1;
      for (int t = 0; t < BWD_SAMPLES; ++t) g += sd1[t][j];
    } else if (p < OFF_B2) {                // W2[j][i]
      const int q = p - OFF_W2, j = q / NH, i = q % NH;
      for (int t = 0; t < BWD_SAMPLES; ++t) g += sd2[t][j] * sh1[t][i];
    } else if (p < OFF_W3) {                // b2[j]
      const int j = p - OFF_B2;
      for (int t = 0; t < BWD_SAMPLES; ++t) g += sd2[t][j];
    } else if (p < OFF_W3 + nout * NH) {    // W3[o][j]
      const int q = p - OFF_W3, o = q / NH, j = q % NH;
      for (int t = 0; t < BWD_SAMPLES; ++t) g += sdy[t][o] * sh2[t][j];
    } else {                                // b3[o]
      const int o = p - OFF_W3 - nout * NH;
      for (int t = 0; t < BWD_SAMPLES; ++t) g += sdy[t][o];
    }
    out[p] = g;
  }
}

// grad[p] = sum over workgroups (in index order) of partial[wg][p]
__global__ __launch_bounds__(256) void sum_partials_kernel(const float *__restrict__ partial,
                                                           int64_t nparts, int P,
                                                           float *__restrict__ out) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= P) return;
  float g = 0.0f;
  for (int64_t w = 0; w < nparts; ++w) g += partial[w * P + p];
  out[p] = g;
}

__global__ __launch_bounds__(256) void mse_kernel(const float *__restrict__ y,
                                                  const float *__restrict__ t, int64_t total,
                                                  float scale, float *__restrict__ dy,
                                                  float *__restrict__ partial) {
  __shared__ float red[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float e2 = 0.0f;
  if (i < total) {
    const float e = y[i] - t[i];
    dy[i] = 2.0f * scale * e;
    e2 = e * e;
  }
  const float s = block_sum256(e2, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ prm,
                                                   const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ v,
                                                   int64_t P, float lr, float b1, float b2,
                                                   float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= P) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  prm[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void scale_copy_kernel(const float *__restrict__ src, float sc, float *__restrict__ dst) {
  dst[0] = src[0] * sc;
}

static inline int64_t nbwd(int64_t B) { return (B + BWD_SAMPLES - 1) / BWD_SAMPLES; }
static inline int64_t nmse(int64_t total) { return (total + 255) / 256; }

}  // namespace nolsm

using namespace nolsm;

static nolsm_status launch_status(void) {
  return hipGetLastError() == hipSuccess ? NOLSM_OK : NOLSM_EHIP;
}

extern "C" {

int64_t nolsm_mlp_param_count(int32_t nout) {
  return (nout < 1 || nout > MAXOUT) ? -1 : (int64_t)mlp_params(nout);
}

int64_t nolsm_mlp_scratch_floats(int64_t B, int32_t nout) {
  if (B < 0 || nout < 1 || nout > MAXOUT) return -1;
  const int64_t a = nbwd(B) * mlp_params(nout);
  const int64_t b = nmse(B * nout) + 1;
  return a > b ? a : b;
}

nolsm_status nolsm_mlp_forward(const float *params, int32_t nout, const float *x, int64_t B,
                               float *y, float *act, hipStream_t s) {
  if (!params || !x || !y || B < 0 || nout < 1 || nout > MAXOUT) return NOLSM_EINVAL;
  if (B == 0) return NOLSM_OK;
  mlp_forward_kernel<<<(unsigned)((B + 255) / 256), 256, 0, s>>>(params, nout, x, B, y, act);
  return launch_status();
}

nolsm_status nolsm_mlp_backward(const float *params, int32_t nout, const float *x,
                                const float *act, const float *dy, int64_t B, float *grad,
                                float *scratch, hipStream_t s) {
  if (!params || !x || !act || !dy || !grad || !scratch || B < 1 || nout < 1 || nout > MAXOUT)
    return NOLSM_EINVAL;
  const int64_t nw = nbwd(B);
  const int P = mlp_params(nout);
  mlp_backward_kernel<<<(unsigned)nw, 256, 0, s>>>(params, nout, x, act, dy, B, scratch);
  sum_partials_kernel<<<(P + 255) / 256, 256, 0, s>>>(scratch, nw, P, grad);
  return launch_status();
}

nolsm_status nolsm_mlp_mse(const float *y, const float *t, int64_t B, int32_t nout, float *dy,
                           float *loss, float *scratch, hipStream_t s) {
  if (!y || !t || !dy || !loss || !scratch || B < 1 || nout < 1 || nout > MAXOUT)
    return NOLSM_EINVAL;
  const int64_t total = B * nout;
  const int64_t nb = nmse(total);
  const float scale = 1.0f / (float)total;
  mse_kernel<<<(unsigned)nb, 256, 0, s>>>(y, t, total, scale, dy, scratch);
  // loss = scale * sum of the block partials, summed in index order
  sum_partials_kernel<<<1, 256, 0, s>>>(scratch, nb, 1, scratch + nb);
  scale_copy_kernel<<<1, 1, 0, s>>>(scratch + nb, scale, loss);
  return launch_status();
}

nolsm_status nolsm_mlp_adam(float *params, const float *grad, float *m, float *v, int64_t P,
                            float lr, float beta1, float beta2, float eps, int32_t step,
                            hipStream_t s) {
  if (!params || !grad || !m || !v || P < 1 || step < 1) return NOLSM_EINVAL;
  const float c1 = 1.0f - powf(beta1, (float)step);
  const float c2 = 1.0f - powf(beta2, (float)step);
  adam_kernel<<<(unsigned)((P + 255) / 256), 256, 0, s>>>(params, grad, m, v, P, lr, beta1, beta2,
                                                         eps, c1, c2);
  return launch_status();
}

}  // extern "C"
