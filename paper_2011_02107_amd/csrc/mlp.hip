// The learned window's regression network on the GPU: a multilayer perceptron (tanh hidden
// layers, linear output, loss 0.5 mean |y - t|^2) with its own forward, backward and Adam
// kernels in FP32.  It maps coupling statistics of a Hamiltonian to the spectral bound and the
// central density of states, which set the filter order and the window (Sec. II.A, Sec. III
// parameter settings); the Lanczos / kernel-polynomial estimates stay the fallback.
//
// Parameters are one flat vector, layer by layer: W (n_out x n_in, row-major), then b.
// k_mlp_pass is a single workgroup: the networks and mini-batches are small (a few thousand
// multiply-adds per sample and layer), and one workgroup keeps every reduction in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <random>
#include <vector>

#include "internal.h"

struct dacp_mlp_s {
  int device = 0;
  int n_in = 0, hidden = 0, layers = 0, n_out = 0;
  int nparams = 0;
  int64_t t = 0;  // Adam steps taken
  dacp::DevBuf params, m, v, grad, loss, act, dlt, xs, ys, idx;
  size_t cap_batch = 0;
  bool scaled = false;
  std::vector<double> x_mean, x_std, y_mean, y_std;
};

namespace dacp {
namespace {

constexpr int kMT = 256;

__device__ __forceinline__ int width(int l, int n_in, int hidden, int layers, int n_out) {
  return l == 0 ? n_in : (l <= layers ? hidden : n_out);
}

// Forward pass over nb samples (rows idx[s] of X, or s when idx is null); with T, the loss and
// the output-layer deltas; with grad, the backward pass and the parameter gradient.
__global__ __launch_bounds__(kMT) void k_mlp_pass(const float *P, int n_in, int hidden, int layers, int n_out,
                                                  const float *X, const float *T, const int *idx, int nb, float *act,
                                                  float *dlt, float *grad, float *loss) {
  __shared__ float red[kMT / 64];
  const int nl = layers + 1;
  auto W = [&](int l) { return width(l, n_in, hidden, layers, n_out); };
  auto poff = [&](int l) {  // offset of layer l's W in P
    int o = 0;
    for (int j = 1; j < l; ++j) o += W(j) * W(j - 1) + W(j);
    return o;
  };
  auto aoff = [&](int l) {  // offset of layer l's activations (l >= 1) in act / dlt
    int o = 0;
    for (int j = 1; j < l; ++j) o += nb * W(j);
    return o;
  };
  auto a_in = [&](int l, int s, int k) -> float {  // activation k of sample s feeding layer l
    if (l == 1) return X[static_cast<int64_t>(idx ? idx[s] : s) * n_in + k];
    return act[aoff(l - 1) + s * W(l - 1) + k];
  };
  for (int l = 1; l <= nl; ++l) {
    const int wo = W(l), wi = W(l - 1), po = poff(l), ao = aoff(l);
    for (int e = threadIdx.x; e < nb * wo; e += kMT) {
      const int s = e / wo, j = e - s * wo;
      float z = P[po + wo * wi + j];
      for (int k = 0; k < wi; ++k) z += P[po + j * wi + k] * a_in(l, s, k);
      act[ao + e] = (l < nl) ? tanhf(z) : z;
    }
    __syncthreads();
  }
  if (!T) return;
  {
    const int ao = aoff(nl);
    float part = 0.0f;
    for (int e = threadIdx.x; e < nb * n_out; e += kMT) {
      const int s = e / n_out, j = e - s * n_out;
      const float r = act[ao + e] - T[static_cast<int64_t>(idx ? idx[s] : s) * n_out + j];
      dlt[ao + e] = r / static_cast<float>(nb);
      part += r * r;
    }
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
      float tot = 0.0f;
      for (int w = 0; w < kMT / 64; ++w) tot += red[w];
      loss[0] = 0.5f * tot / static_cast<float>(nb);
    }
  }
  if (!grad) return;
  for (int l = nl; l >= 2; --l) {  // delta of layer l - 1 from layer l, through tanh
    const int wo = W(l), wi = W(l - 1), po = poff(l), ao = aoff(l), ai = aoff(l - 1);
    for (int e = threadIdx.x; e < nb * wi; e += kMT) {
      const int s = e / wi, k = e - s * wi;
      float g = 0.0f;
      for (int j = 0; j < wo; ++j) g += P[po + j * wi + k] * dlt[ao + s * wo + j];
      const float a = act[ai + e];
      dlt[ai + e] = g * (1.0f - a * a);
    }
    __syncthreads();
  }
  for (int l = 1; l <= nl; ++l) {  // dL/dW_l = delta_l^T a_(l-1), dL/db_l = sum_s delta_l (fixed order)
    const int wo = W(l), wi = W(l - 1), po = poff(l), ao = aoff(l);
    for (int q = threadIdx.x; q < wo * wi + wo; q += kMT) {
      float g = 0.0f;
      if (q < wo * wi) {
        const int j = q / wi, k = q - j * wi;
        for (int s = 0; s < nb; ++s) g += dlt[ao + s * wo + j] * a_in(l, s, k);
      } else {
        const int j = q - wo * wi;
        for (int s = 0; s < nb; ++s) g += dlt[ao + s * wo + j];
      }
      grad[po + q] = g;
    }
  }
}

// Adam (Kingma & Ba): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
// p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
__global__ void k_adam(float *p, const float *g, float *m, float *v, int n, float lr, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

dacp_status ensure_batch(dacp_ctx ctx, dacp_mlp mm, size_t nb) {
  if (nb <= mm->cap_batch) return DACP_OK;
  const size_t per = static_cast<size_t>(mm->layers) * mm->hidden + mm->n_out;
  DACP_HIP(ctx, mm->act.alloc(nb * per * sizeof(float)));
  DACP_HIP(ctx, mm->dlt.alloc(nb * per * sizeof(float)));
  mm->cap_batch = nb;
  return DACP_OK;
}

dacp_status launch_pass(dacp_ctx ctx, dacp_mlp mm, const float *X, const float *T, const int *idx, int nb, bool grad) {
  DACP_TRY(ensure_batch(ctx, mm, static_cast<size_t>(nb)));
  hipLaunchKernelGGL(k_mlp_pass, dim3(1), dim3(kMT), 0, ctx->stream, mm->params.as<float>(), mm->n_in, mm->hidden,
                     mm->layers, mm->n_out, X, T, idx, nb, mm->act.as<float>(), mm->dlt.as<float>(),
                     grad ? mm->grad.as<float>() : nullptr, mm->loss.as<float>());
  DACP_HIP(ctx, hipGetLastError());
  return DACP_OK;
}

}  // namespace
}  // namespace dacp

using dacp::DevBuf;

extern "C" {

dacp_status dacp_mlp_create(dacp_ctx ctx, int n_in, int hidden, int layers, int n_out, uint64_t seed, dacp_mlp *out) {
  if (!ctx || !out) return DACP_E_INVALID;
  *out = nullptr;
  if (n_in < 1 || n_in > 64 || hidden < 0 || hidden > 256 || layers < 0 || layers > 8 || n_out < 1 || n_out > 16 ||
      (layers > 0 && hidden < 1))
    return dacp::set_err(ctx, DACP_E_INVALID, "mlp: n_in 1..64, hidden 1..256, layers 0..8, n_out 1..16");
  dacp_mlp mm = new (std::nothrow) dacp_mlp_s();
  if (!mm) return DACP_E_NOMEM;
  mm->device = ctx->device;
  mm->n_in = n_in;
  mm->hidden = hidden;
  mm->layers = layers;
  mm->n_out = n_out;
  // Glorot-uniform weights, zero biases
  std::mt19937_64 rng(seed);
  std::vector<float> p;
  int prev = n_in;
  for (int l = 1; l <= layers + 1; ++l) {
    const int wo = l <= layers ? hidden : n_out;
    const double lim = std::sqrt(6.0 / (prev + wo));
    std::uniform_real_distribution<double> u(-lim, lim);
    for (int q = 0; q < wo * prev; ++q) p.push_back(static_cast<float>(u(rng)));
    for (int q = 0; q < wo; ++q) p.push_back(0.0f);
    prev = wo;
  }
  mm->nparams = static_cast<int>(p.size());
  const size_t bytes = p.size() * sizeof(float);
  hipError_t e;
  if ((e = mm->params.alloc(bytes)) != hipSuccess || (e = mm->m.alloc(bytes)) != hipSuccess ||
      (e = mm->v.alloc(bytes)) != hipSuccess || (e = mm->grad.alloc(bytes)) != hipSuccess ||
      (e = mm->loss.alloc(sizeof(float))) != hipSuccess) {
    delete mm;
    return dacp::hip_err(ctx, e, "mlp alloc");
  }
  dacp_status st = dacp::to_device(ctx, mm->params.p, p.data(), bytes);
  std::vector<float> zero(p.size(), 0.0f);
  if (!st) st = dacp::to_device(ctx, mm->m.p, zero.data(), bytes);
  if (!st) st = dacp::to_device(ctx, mm->v.p, zero.data(), bytes);
  if (st) {
    delete mm;
    return st;
  }
  *out = mm;
  return DACP_OK;
}

void dacp_mlp_free(dacp_mlp m) {
  if (!m) return;
  (void)hipSetDevice(m->device);
  delete m;
}

dacp_status dacp_mlp_params(dacp_ctx ctx, dacp_mlp m, float *get, const float *set, int *n_params) {
  if (!ctx || !m) return DACP_E_INVALID;
  if (n_params) *n_params = m->nparams;
  const size_t bytes = static_cast<size_t>(m->nparams) * sizeof(float);
  if (get) DACP_TRY(dacp::to_host(ctx, get, m->params.p, bytes));
  if (set) {
    DACP_TRY(dacp::to_device(ctx, m->params.p, set, bytes));
    std::vector<float> zero(m->nparams, 0.0f);
    DACP_TRY(dacp::to_device(ctx, m->m.p, zero.data(), bytes));
    DACP_TRY(dacp::to_device(ctx, m->v.p, zero.data(), bytes));
    m->t = 0;
  }
  return DACP_OK;
}

dacp_status dacp_mlp_loss_grad(dacp_ctx ctx, dacp_mlp m, int n, const double *X, const double *T, double *loss,
                               double *grad) {
  if (!ctx || !m || n < 1 || !X || !T) return DACP_E_INVALID;
  std::vector<float> xf(static_cast<size_t>(n) * m->n_in), tf(static_cast<size_t>(n) * m->n_out);
  for (size_t i = 0; i < xf.size(); ++i) xf[i] = static_cast<float>(X[i]);
  for (size_t i = 0; i < tf.size(); ++i) tf[i] = static_cast<float>(T[i]);
  DevBuf dx, dt;
  DACP_HIP(ctx, dx.alloc(xf.size() * sizeof(float)));
  DACP_HIP(ctx, dt.alloc(tf.size() * sizeof(float)));
  DACP_TRY(dacp::to_device(ctx, dx.p, xf.data(), xf.size() * sizeof(float)));
  DACP_TRY(dacp::to_device(ctx, dt.p, tf.data(), tf.size() * sizeof(float)));
  DACP_TRY(dacp::launch_pass(ctx, m, dx.as<float>(), dt.as<float>(), nullptr, n, grad != nullptr));
  float lf = 0.0f;
  DACP_TRY(dacp::to_host(ctx, &lf, m->loss.p, sizeof(float)));
  if (loss) *loss = lf;
  if (grad) {
    std::vector<float> g(m->nparams);
    DACP_TRY(dacp::to_host(ctx, g.data(), m->grad.p, g.size() * sizeof(float)));
    for (int i = 0; i < m->nparams; ++i) grad[i] = g[i];
  }
  return DACP_OK;
}

dacp_status dacp_mlp_train(dacp_ctx ctx, dacp_mlp m, int n, const double *X, const double *Y, int epochs, int batch,
                           double lr, uint64_t seed, double *final_loss) {
  if (!ctx || !m || n < 1 || !X || !Y || epochs < 0 || batch < 1 || !(lr > 0.0))
    return dacp::set_err(ctx, DACP_E_INVALID, "mlp_train: need n >= 1, epochs >= 0, batch >= 1, lr > 0");
  // per-column standardisation, fixed by the first training set
  if (!m->scaled) {
    auto stats = [&](const double *A, int cols, std::vector<double> &mu, std::vector<double> &sd) {
      mu.assign(cols, 0.0);
      sd.assign(cols, 0.0);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < cols; ++j) mu[j] += A[static_cast<size_t>(i) * cols + j];
      for (int j = 0; j < cols; ++j) mu[j] /= n;
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < cols; ++j) {
          const double d = A[static_cast<size_t>(i) * cols + j] - mu[j];
          sd[j] += d * d;
        }
      for (int j = 0; j < cols; ++j) {
        sd[j] = std::sqrt(sd[j] / n);
        if (!(sd[j] > 1e-12)) sd[j] = 1.0;
      }
    };
    stats(X, m->n_in, m->x_mean, m->x_std);
    stats(Y, m->n_out, m->y_mean, m->y_std);
    m->scaled = true;
  }
  std::vector<float> xf(static_cast<size_t>(n) * m->n_in), yf(static_cast<size_t>(n) * m->n_out);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < m->n_in; ++j)
      xf[static_cast<size_t>(i) * m->n_in + j] =
          static_cast<float>((X[static_cast<size_t>(i) * m->n_in + j] - m->x_mean[j]) / m->x_std[j]);
    for (int j = 0; j < m->n_out; ++j)
      yf[static_cast<size_t>(i) * m->n_out + j] =
          static_cast<float>((Y[static_cast<size_t>(i) * m->n_out + j] - m->y_mean[j]) / m->y_std[j]);
  }
  DACP_HIP(ctx, m->xs.alloc(xf.size() * sizeof(float)));
  DACP_HIP(ctx, m->ys.alloc(yf.size() * sizeof(float)));
  DACP_HIP(ctx, m->idx.alloc(static_cast<size_t>(n) * sizeof(int)));
  DACP_TRY(dacp::to_device(ctx, m->xs.p, xf.data(), xf.size() * sizeof(float)));
  DACP_TRY(dacp::to_device(ctx, m->ys.p, yf.data(), yf.size() * sizeof(float)));
  std::mt19937_64 rng(seed);
  std::vector<int> perm(n);
  const int nb_max = std::min(batch, n);
  for (int ep = 0; ep < epochs; ++ep) {
    std::iota(perm.begin(), perm.end(), 0);
    std::shuffle(perm.begin(), perm.end(), rng);
    DACP_TRY(dacp::to_device(ctx, m->idx.p, perm.data(), perm.size() * sizeof(int)));
    for (int b0 = 0; b0 < n; b0 += nb_max) {
      const int nb = std::min(nb_max, n - b0);
      DACP_TRY(dacp::launch_pass(ctx, m, m->xs.as<float>(), m->ys.as<float>(), m->idx.as<int>() + b0, nb, true));
      ++m->t;
      const float c1 = static_cast<float>(1.0 - std::pow(0.9, static_cast<double>(m->t)));
      const float c2 = static_cast<float>(1.0 - std::pow(0.999, static_cast<double>(m->t)));
      hipLaunchKernelGGL(dacp::k_adam, dim3((m->nparams + 255) / 256), dim3(256), 0, ctx->stream, m->params.as<float>(),
                         m->grad.as<float>(), m->m.as<float>(), m->v.as<float>(), m->nparams, static_cast<float>(lr), c1,
                         c2);
      DACP_HIP(ctx, hipGetLastError());
    }
  }
  // loss of the standardised targets over the whole set
  DACP_TRY(dacp::launch_pass(ctx, m, m->xs.as<float>(), m->ys.as<float>(), nullptr, n, false));
  float lf = 0.0f;
  DACP_TRY(dacp::to_host(ctx, &lf, m->loss.p, sizeof(float)));
  if (final_loss) *final_loss = lf;
  return DACP_OK;
}

dacp_status dacp_mlp_predict(dacp_ctx ctx, dacp_mlp m, int n, const double *X, double *Y) {
  if (!ctx || !m || n < 1 || !X || !Y) return DACP_E_INVALID;
  if (!m->scaled) return dacp::set_err(ctx, DACP_E_INVALID, "mlp_predict: the network has not been trained");
  std::vector<float> xf(static_cast<size_t>(n) * m->n_in);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m->n_in; ++j)
      xf[static_cast<size_t>(i) * m->n_in + j] =
          static_cast<float>((X[static_cast<size_t>(i) * m->n_in + j] - m->x_mean[j]) / m->x_std[j]);
  DevBuf dx;
  DACP_HIP(ctx, dx.alloc(xf.size() * sizeof(float)));
  DACP_TRY(dacp::to_device(ctx, dx.p, xf.data(), xf.size() * sizeof(float)));
  DACP_TRY(dacp::launch_pass(ctx, m, dx.as<float>(), nullptr, nullptr, n, false));
  // outputs are the last activation block
  const size_t off = static_cast<size_t>(n) * m->layers * m->hidden;
  std::vector<float> yf(static_cast<size_t>(n) * m->n_out);
  DACP_TRY(dacp::to_host(ctx, yf.data(), m->act.as<float>() + off, yf.size() * sizeof(float)));
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < m->n_out; ++j)
      Y[static_cast<size_t>(i) * m->n_out + j] = yf[static_cast<size_t>(i) * m->n_out + j] * m->y_std[j] + m->y_mean[j];
  return DACP_OK;
}

}  // extern "C"
