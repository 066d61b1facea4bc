// Batched dense symmetric eigensolver for many small subspace problems (App. C, one workgroup per
// matrix).  The per-problem solver of eig.hip issues several kernels per column and is bound by
// launches at n of a few hundred; here one launch covers every problem of a batch:
//   1. Householder tridiagonalisation in place (one column per step, the step's vectors in LDS);
//   2. implicit symmetric QR with a Wilkinson shift on (d, e): thread 0 chases the bulge and
//      records the sweep's Givens pairs in LDS, then every thread applies them to one column of
//      Zr (rows = eigenvectors of the tridiagonal, starting from I);
//   3. Q = H_0 H_1 ... H_(n-3) formed explicitly, one thread per column.
// The host then sorts the eigenvalues and forms the eigenvectors of A as rows of Zr Q^T.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "internal.h"

namespace dacp {

namespace {

constexpr int kBT = 1024;       // threads per problem
constexpr int kBWaves = kBT / 64;

// Sum over the workgroup, the same value returned to every thread (fixed order: lanes by
// butterfly, then the waves in index order).  red holds kBWaves doubles.
__device__ double block_sum(double s, double *red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int w = 0; w < kBWaves; ++w) t += red[w];
  __syncthreads();
  return t;
}

// Givens pair with c x - s z = r and s x + c z = 0 (the stable Golub-Van Loan formulas).
__device__ void givens_pair(double x, double z, double &c, double &s) {
  if (z == 0.0) {
    c = 1.0;
    s = 0.0;
  } else if (fabs(z) > fabs(x)) {
    const double tau = -x / z;
    s = 1.0 / sqrt(1.0 + tau * tau);
    c = s * tau;
  } else {
    const double tau = -z / x;
    c = 1.0 / sqrt(1.0 + tau * tau);
    s = c * tau;
  }
}

// LDS: v, w (n each), cs (2n), d, e (n each), then the reduction slots and control words.
__global__ __launch_bounds__(kBT) void k_batch_syev(const BatchEigProblem *probs) {
  extern __shared__ double sm[];
  const BatchEigProblem pb = probs[blockIdx.x];
  const int n = pb.n;
  double *vsh = sm, *wsh = sm + n, *cs = sm + 2 * n, *d = sm + 4 * n, *e = sm + 5 * n, *red = sm + 6 * n;
  int *ctl = reinterpret_cast<int *>(red + kBWaves);  // p, q, go
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double *A = pb.A;
  double *betas = pb.beta;
  if (n == 1) {
    if (tid == 0) {
      pb.w[0] = A[0];
      pb.Zr[0] = 1.0;
      pb.Q[0] = 1.0;
      *pb.status = 0;
    }
    return;
  }
  // ---- 1. tridiagonalise
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    const double *x = A + static_cast<int64_t>(k) * n + k + 1;
    double s = 0.0;
    for (int i = 1 + tid; i < m; i += kBT) s += x[i] * x[i];
    const double sigma = block_sum(s, red);
    const double x0 = x[0];
    double alpha = x0, v0 = 0.0, beta = 0.0;
    if (sigma > 0.0) {
      const double mu = sqrt(x0 * x0 + sigma);
      alpha = (x0 >= 0.0) ? -mu : mu;
      v0 = x0 - alpha;
      beta = 2.0 / (v0 * v0 + sigma);
    }
    for (int i = tid; i < m; i += kBT) vsh[i] = (i == 0) ? v0 : x[i];
    if (tid == 0) {
      d[k] = A[static_cast<int64_t>(k) * n + k];
      e[k] = alpha;
      betas[k] = beta;
      A[static_cast<int64_t>(k) * n + k + 1] = v0;  // row k keeps v for forming Q
    }
    __syncthreads();
    if (beta == 0.0) continue;
    double *a22 = A + static_cast<int64_t>(k + 1) * n + k + 1;
    // p = beta A22 v, one wave per row
    for (int i = wave; i < m; i += kBWaves) {
      const double *row = a22 + static_cast<int64_t>(i) * n;
      double t = 0.0;
      for (int j = lane; j < m; j += 64) t += row[j] * vsh[j];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
      if (lane == 0) wsh[i] = beta * t;
    }
    __syncthreads();
    // w = p - (beta p^T v / 2) v
    double pv = 0.0;
    for (int i = tid; i < m; i += kBT) pv += wsh[i] * vsh[i];
    const double half = 0.5 * beta * block_sum(pv, red);
    for (int i = tid; i < m; i += kBT) wsh[i] -= half * vsh[i];
    __syncthreads();
    // A22 -= v w^T + w v^T
    for (int i = 0; i < m; ++i) {
      const double vi = vsh[i], wi = wsh[i];
      double *row = a22 + static_cast<int64_t>(i) * n;
      for (int j = tid; j < m; j += kBT) row[j] -= vi * wsh[j] + wi * vsh[j];
    }
    __syncthreads();
  }
  if (tid == 0) {
    d[n - 2] = A[static_cast<int64_t>(n - 2) * n + n - 2];
    e[n - 2] = A[static_cast<int64_t>(n - 2) * n + n - 1];
    d[n - 1] = A[static_cast<int64_t>(n - 1) * n + n - 1];
    e[n - 1] = 0.0;
  }
  // Zr = I
  for (int64_t idx = tid; idx < static_cast<int64_t>(n) * n; idx += kBT)
    pb.Zr[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
  __syncthreads();
  // ---- 2. implicit symmetric QR on (d, e): thread 0 steers, everyone rotates Zr's rows p..q
  int q = n - 1;  // thread 0's working state
  long iters = 0;
  const long max_iters = 40L * n + 100;
  const double eps = 2.220446049250313e-16;
  while (true) {
    if (tid == 0) {
      int go = 0;
      while (q > 0) {
        if (e[q - 1] == 0.0 || fabs(e[q - 1]) <= eps * (fabs(d[q - 1]) + fabs(d[q]))) {
          e[q - 1] = 0.0;
          --q;
          continue;
        }
        int p = q - 1;
        while (p > 0 && !(fabs(e[p - 1]) <= eps * (fabs(d[p - 1]) + fabs(d[p])))) --p;
        if (p > 0) e[p - 1] = 0.0;
        if (++iters > max_iters) {
          *pb.status = 1;
          break;
        }
        // Wilkinson shift from the trailing 2 x 2 block, then the bulge chase from p to q
        const double a = d[q - 1], bb = e[q - 1], cc = d[q];
        const double delta = 0.5 * (a - cc);
        const double den = delta + (delta >= 0.0 ? 1.0 : -1.0) * hypot(delta, bb);
        const double mu = (den != 0.0) ? cc - bb * bb / den : cc;
        double xx = d[p] - mu, zz = e[p];
        for (int kk = p; kk < q; ++kk) {
          double c, sn;
          givens_pair(xx, zz, c, sn);
          if (kk > p) e[kk - 1] = c * xx - sn * zz;
          const double dk = d[kk], dk1 = d[kk + 1], ek = e[kk];
          d[kk] = c * c * dk - 2.0 * c * sn * ek + sn * sn * dk1;
          d[kk + 1] = sn * sn * dk + 2.0 * c * sn * ek + c * c * dk1;
          e[kk] = c * sn * (dk - dk1) + (c * c - sn * sn) * ek;
          if (kk < q - 1) {
            xx = e[kk];
            zz = -sn * e[kk + 1];
            e[kk + 1] = c * e[kk + 1];
          }
          cs[2 * (kk - p)] = c;
          cs[2 * (kk - p) + 1] = sn;
        }
        ctl[0] = p;
        ctl[1] = q;
        go = 1;
        break;
      }
      ctl[2] = go;
    }
    __syncthreads();
    if (!ctl[2]) break;
    const int p = ctl[0], qq = ctl[1];
    for (int col = tid; col < n; col += kBT) {
      double carry = pb.Zr[static_cast<int64_t>(p) * n + col];
      for (int kk = p; kk < qq; ++kk) {
        const double c = cs[2 * (kk - p)], sn = cs[2 * (kk - p) + 1];
        double *zk1 = pb.Zr + static_cast<int64_t>(kk + 1) * n + col;
        const double zn = *zk1;
        pb.Zr[static_cast<int64_t>(kk) * n + col] = c * carry - sn * zn;
        carry = sn * carry + c * zn;
      }
      pb.Zr[static_cast<int64_t>(qq) * n + col] = carry;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += kBT) pb.w[i] = d[i];
  if (tid == 0 && *pb.status != 1) *pb.status = 0;
  // ---- 3. Q = H_0 H_1 ... H_(n-3): apply H_k from k = n-3 down to 0 onto I; H_k touches rows
  // and columns k+1.. only, so columns <= k of the product stay those of I
  for (int64_t idx = tid; idx < static_cast<int64_t>(n) * n; idx += kBT)
    pb.Q[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
  __syncthreads();
  for (int k = n - 3; k >= 0; --k) {
    const double beta = betas[k];
    if (beta == 0.0) continue;
    const int m = n - k - 1;
    for (int i = tid; i < m; i += kBT) vsh[i] = A[static_cast<int64_t>(k) * n + k + 1 + i];
    __syncthreads();
    double *qk = pb.Q + static_cast<int64_t>(k + 1) * n;
    for (int col = k + 1 + tid; col < n; col += kBT) {
      double t = 0.0;
      for (int r = 0; r < m; ++r) t += vsh[r] * qk[static_cast<int64_t>(r) * n + col];
      t *= beta;
      for (int r = 0; r < m; ++r) qk[static_cast<int64_t>(r) * n + col] -= t * vsh[r];
    }
    __syncthreads();
  }
}

}  // namespace

size_t batch_syev_lds(int max_n) { return (6 * static_cast<size_t>(max_n) + kBWaves) * sizeof(double) + 4 * sizeof(int); }

hipError_t launch_batch_syev(const BatchEigProblem *probs, int count, int max_n, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (max_n < 1 || max_n > kBatchEigMaxN) return hipErrorInvalidValue;
  const size_t lds = batch_syev_lds(max_n);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_batch_syev),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_syev, dim3(count), dim3(kBT), lds, s, probs);
  return hipGetLastError();
}

// Host side, first half: one launch over `count` matrices A[i] (device, n[i] x n[i], ld n[i],
// destroyed); Zr[i], Q[i] (device, n x n) receive the tridiagonal's eigenvectors (rows, unsorted)
// and the Householder product, w[i] (host) the eigenvalues in the same unsorted order.
dacp_status batch_syev_raw(dacp_ctx ctx, int count, const int *n, double *const *A, double *const *Zr,
                           double *const *Q, double *const *w) {
  if (count <= 0) return DACP_OK;
  hipStream_t st = ctx->stream;
  int max_n = 0;
  size_t total = 0;
  std::vector<size_t> off(count);
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > kBatchEigMaxN) return set_err(ctx, DACP_E_INVALID, "batch_syev: 1 <= n <= 2048");
    max_n = std::max(max_n, n[i]);
    off[i] = total;
    total += 2 * static_cast<size_t>(n[i]);  // w, beta
  }
  DevBuf work, dprobs, dstat;
  DACP_HIP(ctx, work.alloc(total * sizeof(double)));
  DACP_HIP(ctx, dstat.alloc(sizeof(int) * count));
  DACP_HIP(ctx, hipMemsetAsync(dstat.p, 0, sizeof(int) * count, st));
  std::vector<BatchEigProblem> probs(count);
  for (int i = 0; i < count; ++i) {
    double *base = work.as<double>() + off[i];
    probs[i].A = A[i];
    probs[i].Zr = Zr[i];
    probs[i].Q = Q[i];
    probs[i].w = base;
    probs[i].beta = base + n[i];
    probs[i].status = dstat.as<int>() + i;
    probs[i].n = n[i];
  }
  DACP_HIP(ctx, dprobs.alloc(sizeof(BatchEigProblem) * count));
  DACP_TRY(to_device(ctx, dprobs.p, probs.data(), sizeof(BatchEigProblem) * count));
  DACP_HIP(ctx, launch_batch_syev(dprobs.as<BatchEigProblem>(), count, max_n, st));
  std::vector<int> status(count);
  DACP_TRY(to_host(ctx, status.data(), dstat.p, sizeof(int) * count));
  for (int i = 0; i < count; ++i)
    if (status[i] != 0) return set_err(ctx, DACP_E_CONVERGENCE, "batch_syev: QR iteration did not converge");
  std::vector<double> all(total);
  DACP_TRY(to_host(ctx, all.data(), work.p, total * sizeof(double)));
  for (int i = 0; i < count; ++i) std::copy(all.begin() + off[i], all.begin() + off[i] + n[i], w[i]);
  return DACP_OK;
}

// Second half, for one matrix on the caller's stream: eigenvalues ascending into w_out and, if
// Zrows is set, the eigenvectors of A as its rows: Y = Zr Q^T (written over the destroyed A), then
// the rows of Y in ascending order of the eigenvalues.
dacp_status batch_syev_finish(dacp_ctx ctx, int n, const double *w_raw, double *A, const double *Zr, const double *Q,
                              double *w_out, double *Zrows) {
  hipStream_t st = ctx->stream;
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return w_raw[a] < w_raw[b]; });
  for (int j = 0; j < n; ++j) w_out[j] = w_raw[perm[j]];
  if (!Zrows) return DACP_OK;
  DevBuf dperm;
  DACP_HIP(ctx, dperm.alloc(sizeof(int) * n));
  DACP_TRY(to_device(ctx, dperm.p, perm.data(), sizeof(int) * n));
  DACP_HIP(ctx, launch_dgemm(0, 1, n, n, n, 1.0, Zr, n, Q, n, 0.0, A, n, 0, st));
  DACP_HIP(ctx, launch_gather_rows(A, n, Zrows, n, dperm.as<int>(), nullptr, n, n, st));
  DACP_HIP(ctx, hipStreamSynchronize(st));  // dperm is released on return
  return DACP_OK;
}

// Both halves: eigen-decompositions of `count` symmetric matrices A[i] (device, n[i] x n[i], ld n[i],
// destroyed) in one launch.  w[i] (host) ascending; Zrows[i] (device, n x n) row j = eigenvector j.
dacp_status batch_syev(dacp_ctx ctx, int count, const int *n, double *const *A, double *const *w,
                       double *const *Zrows) {
  if (count <= 0) return DACP_OK;
  size_t total = 0;
  std::vector<size_t> off(count);
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > kBatchEigMaxN) return set_err(ctx, DACP_E_INVALID, "batch_syev: 1 <= n <= 2048");
    off[i] = total;
    total += 2 * static_cast<size_t>(n[i]) * n[i];
  }
  DevBuf scratch;
  DACP_HIP(ctx, scratch.alloc(total * sizeof(double)));
  std::vector<double *> zr(count), q(count), wr(count);
  std::vector<std::vector<double>> wraw(count);
  for (int i = 0; i < count; ++i) {
    zr[i] = scratch.as<double>() + off[i];
    q[i] = zr[i] + static_cast<size_t>(n[i]) * n[i];
    wraw[i].resize(n[i]);
    wr[i] = wraw[i].data();
  }
  DACP_TRY(batch_syev_raw(ctx, count, n, A, zr.data(), q.data(), wr.data()));
  for (int i = 0; i < count; ++i)
    DACP_TRY(batch_syev_finish(ctx, n[i], wr[i], A[i], zr[i], q[i], w[i], Zrows[i]));
  return DACP_OK;
}

}  // namespace dacp
