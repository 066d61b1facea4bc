// Dense symmetric eigen-decomposition for the subspace problem (App. C):
// Householder tridiagonalisation on the GPU, implicit symmetric QR with a
// Wilkinson shift on the host (O(n^2) scalar work), and the QR rotations
// replayed on the GPU onto the Householder Q.  Eigenvectors are returned as
// rows (row j = eigenvector j), the layout in which the rotations of one QR
// sweep stream through memory with every lane owning one column.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "internal.h"

namespace dacp {

// ----------------------------------------------------------- tridiagonalise
// Step k reduces row k: x = A[k][k+1..n-1], v = x - alpha e1 with
// alpha = -sign(x0) ||x||, beta = 2 / v^T v; v is written back over x (it is
// never read again by the reduction) and kept for forming Q.
__global__ __launch_bounds__(1024) void k_house(double *A, int64_t ld, int n, int k, double *v, double *dd,
                                                double *ee, double *betas) {
  __shared__ double red[1024];
  const int m = n - k - 1;
  const double *x = A + static_cast<int64_t>(k) * ld + k + 1;
  double s = 0.0;
  for (int i = 1 + threadIdx.x; i < m; i += blockDim.x) s += x[i] * x[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double sigma = red[0];
  const double x0 = x[0];
  double beta = 0.0, alpha = x0, v0 = 0.0;
  if (sigma > 0.0) {
    const double mu = sqrt(x0 * x0 + sigma);
    alpha = (x0 >= 0.0) ? -mu : mu;
    v0 = x0 - alpha;
    beta = 2.0 / (v0 * v0 + sigma);
  }
  for (int i = threadIdx.x; i < m; i += blockDim.x) v[i] = (i == 0) ? v0 : (sigma > 0.0 ? x[i] : 0.0);
  __syncthreads();
  if (threadIdx.x == 0) {
    dd[k] = A[static_cast<int64_t>(k) * ld + k];
    ee[k] = alpha;
    betas[k] = beta;
    A[static_cast<int64_t>(k) * ld + k + 1] = v0;
  }
}

// p[i] = beta * sum_j A[k+1+i][k+1+j] v[j]; one wave per row.
__global__ __launch_bounds__(256) void k_symv(const double *A, int64_t ld, int n, int k, const double *v,
                                              const double *betas, double *p) {
  const double beta = betas[k];
  const int m = n - k - 1;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= m || beta == 0.0) return;
  const double *a = A + static_cast<int64_t>(k + 1 + row) * ld + k + 1;
  // four independent 64-wide strips in flight per wave
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int j = lane;
  for (; j + 192 < m; j += 256) {
    s0 += a[j] * v[j];
    s1 += a[j + 64] * v[j + 64];
    s2 += a[j + 128] * v[j + 128];
    s3 += a[j + 192] * v[j + 192];
  }
  for (; j < m; j += 64) s0 += a[j] * v[j];
  double s = (s0 + s1) + (s2 + s3);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) p[row] = beta * s;
}

// w = p - (beta p^T v / 2) v, in place over p.
__global__ __launch_bounds__(1024) void k_wvec(double *p, const double *v, const double *betas, int n, int k) {
  __shared__ double red[1024];
  const double beta = betas[k];
  const int m = n - k - 1;
  if (beta == 0.0) return;
  double s = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) s += p[i] * v[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double half = 0.5 * beta * red[0];
  for (int i = threadIdx.x; i < m; i += blockDim.x) p[i] -= half * v[i];
}

// A22 -= v w^T + w v^T.
__global__ __launch_bounds__(256) void k_syr2(double *A, int64_t ld, int n, int k, const double *v, const double *w,
                                              const double *betas) {
  if (betas[k] == 0.0) return;
  const int m = n - k - 1;
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int i = blockIdx.y;
  if (j >= m || i >= m) return;
  double *a = A + static_cast<int64_t>(k + 1 + i) * ld + k + 1;
  a[j] -= v[i] * w[j] + w[i] * v[j];
}

// Q^T <- Q^T P_k on rows i > k: Qc[i] -= beta (Qc[i] . v) v^T, v = A[k][k+1..].
__global__ __launch_bounds__(256) void k_qupdate(double *Qc, int64_t ldq, const double *A, int64_t ld, int n, int k,
                                                 const double *betas) {
  const double beta = betas[k];
  const int row = k + 1 + blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n || beta == 0.0) return;
  const double *v = A + static_cast<int64_t>(k) * ld;
  double *q = Qc + static_cast<int64_t>(row) * ldq;
  double s = 0.0;
  for (int j = k + 1 + lane; j < n; j += 64) s += q[j] * v[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  s *= beta;
  for (int j = k + 1 + lane; j < n; j += 64) q[j] -= s * v[j];
}

// ---- panel (blocked) tridiagonalisation: the rank-2 updates of a panel of kTB reflectors are
// deferred and applied to the trailing matrix as two GEMMs at the panel's end.  Within the panel,
// row k is brought up to date before its reflector is formed, and the matrix-vector product uses
// the trailing matrix as of the panel start, corrected by the panel's V and W:
//   p = beta (A v - V (W^T v) - W (V^T v)).
// V and W are n x kTB row-major (row = global index, column = reflector within the panel).
constexpr int kTB = 32;

// A[k][c] -= sum_(i<j) V[k][i] W[c][i] + W[k][i] V[c][i]  for c >= k.
__global__ __launch_bounds__(256) void k_panel_row(double *A, int64_t ld, int n, int k, const double *V,
                                                   const double *W, int j) {
  const int c = k + blockIdx.x * 256 + threadIdx.x;
  if (c >= n || j == 0) return;
  const double *vk = V + static_cast<int64_t>(k) * kTB, *wk = W + static_cast<int64_t>(k) * kTB;
  const double *vc = V + static_cast<int64_t>(c) * kTB, *wc = W + static_cast<int64_t>(c) * kTB;
  double s = 0.0;
  for (int i = 0; i < j; ++i) s += vk[i] * wc[i] + wk[i] * vc[i];
  A[static_cast<int64_t>(k) * ld + c] -= s;
}

// xy[i] = sum_r W[k+1+r][i] v[r], xy[kTB + i] = sum_r V[k+1+r][i] v[r]  (i < j); one block per i.
__global__ __launch_bounds__(256) void k_panel_dots(const double *V, const double *W, int n, int k, int j,
                                                    const double *v, double *xy) {
  __shared__ double red[256];
  const int i = blockIdx.x % kTB, which = blockIdx.x / kTB;
  if (i >= j) return;
  const double *P = which == 0 ? W : V;
  const int m = n - k - 1;
  double s = 0.0;
  for (int r = threadIdx.x; r < m; r += 256) s += P[static_cast<int64_t>(k + 1 + r) * kTB + i] * v[r];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) xy[which * kTB + i] = red[0];
}

// p[r] -= beta sum_(i<j) (V[k+1+r][i] x_i + W[k+1+r][i] y_i)
__global__ __launch_bounds__(256) void k_panel_corr(double *p, const double *V, const double *W, int n, int k, int j,
                                                    const double *xy, const double *betas) {
  const int r = blockIdx.x * 256 + threadIdx.x;
  const int m = n - k - 1;
  const double beta = betas[k];
  if (r >= m || j == 0 || beta == 0.0) return;
  const double *vr = V + static_cast<int64_t>(k + 1 + r) * kTB, *wr = W + static_cast<int64_t>(k + 1 + r) * kTB;
  double s = 0.0;
  for (int i = 0; i < j; ++i) s += vr[i] * xy[i] + wr[i] * xy[kTB + i];
  p[r] -= beta * s;
}

// V[:, j] = (0 .. 0, v), W[:, j] = (0 .. 0, w) with v, w starting at global index k + 1.
__global__ __launch_bounds__(256) void k_panel_store(double *V, double *W, int n, int k, int j, const double *v,
                                                     const double *w, const double *betas) {
  const int row = blockIdx.x * 256 + threadIdx.x;
  if (row >= n) return;
  const bool in = row > k && betas[k] != 0.0;
  V[static_cast<int64_t>(row) * kTB + j] = in ? v[row - k - 1] : 0.0;
  W[static_cast<int64_t>(row) * kTB + j] = in ? w[row - k - 1] : 0.0;
}

// Rows of V^T for reflectors k0 .. k0 + kb - 1: vt[j][c] = v_(k0+j)[c] (stored in A[k0 + j][c] for
// c > k0 + j), zero elsewhere.
__global__ void k_build_vt(const double *A, int64_t ld, int n, int k0, int kb, double *vt) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(kb) * n) return;
  const int j = static_cast<int>(e / n), c = static_cast<int>(e - static_cast<int64_t>(j) * n);
  const int k = k0 + j;
  vt[e] = (c > k) ? A[static_cast<int64_t>(k) * ld + c] : 0.0;
}

__global__ void k_set_identity(double *Q, int64_t ldq, int n) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(n) * n) return;
  const int64_t i = e / n, j = e - i * n;
  Q[i * ldq + j] = (i == j) ? 1.0 : 0.0;
}

// Replay of implicit-QR sweeps onto the rows of Qc.  Sweep i rotates, for
// k = p_i..q_i-1:  Qc[k] <- c Qc[k] - s Qc[k+1],  Qc[k+1] <- s Qc[k] + c Qc[k+1].
//
// A batch of NSW consecutive sweeps is applied in one pass as a wavefront:
// at time tau, sweep i applies its rotation k = tau - 2i.  Sweep i+1 touches
// rows k, k+1 only after sweep i has finished row k+1 (its rotation k+1 ran
// at tau - 1), and the sweeps active at one tau touch disjoint row pairs.
// Each lane owns one column and keeps the last W = 2 NSW rows in registers:
// row tau + 1 is loaded into the slot that row tau + 1 - W (final for every
// sweep of the batch) is stored from, so each row is read and written once
// per batch instead of once per sweep.
constexpr int NSW = 16;
constexpr int WIN = 2 * NSW;

struct SweepBatch {
  int p[NSW], q[NSW];
  int64_t off[NSW];  // offset (in rotation pairs) of each sweep's rotations
  int count;
  int rmin, rmax;    // rows touched by the batch
};

__global__ __launch_bounds__(64) void k_rot_batch(double *Qc, int64_t ldq, int ncols, SweepBatch sb,
                                                  const double *cs) {
  const int col = blockIdx.x * 64 + threadIdx.x;
  if (col >= ncols) return;
  double *base = Qc + col;
  double win[WIN];
#pragma unroll
  for (int u = 0; u < WIN; ++u) win[u] = 0.0;
  // tau runs from rmin - 1 (load row rmin) to rmax + WIN - 1 (store row rmax); aligned so that
  // slot (row mod WIN) is static inside the unrolled body.
  const int tau_beg = sb.rmin - 1;
  const int tau_end = sb.rmax + WIN - 1;
  const int t0_beg = tau_beg - (((tau_beg % WIN) + WIN) % WIN);
  for (int t0 = t0_beg; t0 <= tau_end; t0 += WIN) {
#pragma unroll
    for (int u = 0; u < WIN; ++u) {
      const int tau = t0 + u;
      const int slot = (u + 1) % WIN;  // slot of rows tau + 1 and tau + 1 - WIN
      const int r_out = tau + 1 - WIN;
      if (r_out >= sb.rmin && r_out <= sb.rmax) base[static_cast<int64_t>(r_out) * ldq] = win[slot];
      const int r_in = tau + 1;
      if (r_in >= sb.rmin && r_in <= sb.rmax) win[slot] = base[static_cast<int64_t>(r_in) * ldq];
#pragma unroll
      for (int i = 0; i < NSW; ++i) {
        const int k = tau - 2 * i;
        if (i < sb.count && k >= sb.p[i] && k < sb.q[i]) {
          const int64_t o = sb.off[i] + (k - sb.p[i]);
          const double c = cs[2 * o], s = cs[2 * o + 1];
          const int sk = ((u - 2 * i) % WIN + WIN) % WIN;
          const int sk1 = (sk + 1) % WIN;
          const double xk = win[sk], xk1 = win[sk1];
          win[sk] = c * xk - s * xk1;
          win[sk1] = s * xk + c * xk1;
        }
      }
    }
  }
}

__global__ void k_gather_rows(const double *src, int64_t lds, double *dst, int64_t ldd, const int *perm,
                              const double *scale, int rows, int cols) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(rows) * cols) return;
  const int64_t i = e / cols, j = e - i * cols;
  const double sc = scale ? scale[i] : 1.0;
  dst[i * ldd + j] = sc * src[static_cast<int64_t>(perm[i]) * lds + j];
}

// ---------------------------------------------------- host implicit QR

namespace {

struct Sweep {
  int p, q;
  size_t off;  // offset (in pairs) into the rotation buffer
};

// Givens pair for the rotation row_k' = c row_k - s row_{k+1},
// row_{k+1}' = s row_k + c row_{k+1}: chosen so that c x - s z = r and
// s x + c z = 0 (Golub & Van Loan's stable formulas).
inline void givens(double x, double z, double &c, double &s) {
  if (z == 0.0) {
    c = 1.0;
    s = 0.0;
  } else if (std::fabs(z) > std::fabs(x)) {
    const double tau = -x / z;
    s = 1.0 / std::sqrt(1.0 + tau * tau);
    c = s * tau;
  } else {
    const double tau = -z / x;
    c = 1.0 / std::sqrt(1.0 + tau * tau);
    s = c * tau;
  }
}

// Implicit symmetric QR with a Wilkinson shift (Golub & Van Loan), deflating
// from the bottom.  d (n), e (n, e[i] couples i and i+1) are overwritten by
// the eigenvalues (unsorted).  Every sweep over the unreduced block [p, q]
// calls sink(p, q, cs) with the q - p rotations (c, s) in order k = p..q-1.
template <typename Sink>
bool tridiag_qr(std::vector<double> &d, std::vector<double> &e, int n, Sink &&sink) {
  const double eps = 2.220446049250313e-16;
  std::vector<double> cs(2 * static_cast<size_t>(n));
  int q = n - 1;
  long iters = 0;
  const long max_iters = 40L * n + 100;
  while (q > 0) {
    if (e[q - 1] == 0.0 || std::fabs(e[q - 1]) <= eps * (std::fabs(d[q - 1]) + std::fabs(d[q]))) {
      e[q - 1] = 0.0;
      --q;
      continue;
    }
    int p = q - 1;
    while (p > 0 && !(std::fabs(e[p - 1]) <= eps * (std::fabs(d[p - 1]) + std::fabs(d[p])))) --p;
    if (p > 0) e[p - 1] = 0.0;
    if (++iters > max_iters) return false;
    const double a = d[q - 1], bb = e[q - 1], cc = d[q];
    const double delta = 0.5 * (a - cc);
    const double den = delta + (delta >= 0.0 ? 1.0 : -1.0) * std::hypot(delta, bb);
    const double mu = (den != 0.0) ? cc - bb * bb / den : cc;
    double x = d[p] - mu, z = e[p];
    for (int k = p; k < q; ++k) {
      double c, s;
      givens(x, z, c, s);
      if (k > p) e[k - 1] = c * x - s * z;
      const double dk = d[k], dk1 = d[k + 1], ek = e[k];
      d[k] = c * c * dk - 2.0 * c * s * ek + s * s * dk1;
      d[k + 1] = s * s * dk + 2.0 * c * s * ek + c * c * dk1;
      e[k] = c * s * (dk - dk1) + (c * c - s * s) * ek;
      if (k < q - 1) {
        x = e[k];
        z = -s * e[k + 1];
        e[k + 1] = c * e[k + 1];
      }
      cs[2 * (k - p)] = c;
      cs[2 * (k - p) + 1] = s;
    }
    sink(p, q, cs.data());
  }
  return true;
}

}  // namespace

// Small symmetric tridiagonal eigenproblem on the host (Lanczos matrices):
// w ascending; Z (n x n row-major, may be null) column j = eigenvector j.
bool host_tridiag_eig(const double *diag, const double *off, int n, double *w, double *Z) {
  std::vector<double> d(diag, diag + n), e(n, 0.0);
  for (int i = 0; i + 1 < n; ++i) e[i] = off[i];
  std::vector<double> Zr;  // rows = eigenvectors while iterating
  if (Z) {
    Zr.assign(static_cast<size_t>(n) * n, 0.0);
    for (int i = 0; i < n; ++i) Zr[static_cast<size_t>(i) * n + i] = 1.0;
  }
  auto sink = [&](int p, int q, const double *cs) {
    if (!Z) return;
    for (int col = 0; col < n; ++col) {
      double carry = Zr[static_cast<size_t>(p) * n + col];
      for (int k = p; k < q; ++k) {
        const double c = cs[2 * (k - p)], s = cs[2 * (k - p) + 1];
        const double zn = Zr[static_cast<size_t>(k + 1) * n + col];
        Zr[static_cast<size_t>(k) * n + col] = c * carry - s * zn;
        carry = s * carry + c * zn;
      }
      Zr[static_cast<size_t>(q) * n + col] = carry;
    }
  };
  if (!tridiag_qr(d, e, n, sink)) return false;
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int i, int j) { return d[i] < d[j]; });
  for (int j = 0; j < n; ++j) {
    w[j] = d[perm[j]];
    if (Z)
      for (int i = 0; i < n; ++i) Z[static_cast<size_t>(i) * n + j] = Zr[static_cast<size_t>(perm[j]) * n + i];
  }
  return true;
}

// Eigen-decomposition of the symmetric n x n device matrix A (row-major, ld,
// destroyed).  w (host) ascending; Zrows (device, n x n, ld n) row j =
// eigenvector j, or nullptr for eigenvalues only.
static double wall_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

dacp_status gpu_syev(dacp_ctx ctx, int n, double *A, int64_t ld, double *w, double *Zrows) {
  hipStream_t st = ctx->stream;
  const double t_begin = wall_ms();
  if (n <= 0) return DACP_OK;
  if (n == 1) {
    DACP_TRY(to_host(ctx, w, A, sizeof(double)));
    DACP_HIP(ctx, hipStreamSynchronize(st));
    if (Zrows) {
      const double one = 1.0;
      DACP_TRY(to_device(ctx, Zrows, &one, sizeof(double)));
      DACP_HIP(ctx, hipStreamSynchronize(st));
    }
    return DACP_OK;
  }
  double *dv = nullptr, *dp = nullptr, *dd = nullptr, *de = nullptr, *db = nullptr;
  DACP_HIP(ctx, hipMalloc(&dv, sizeof(double) * n));
  DACP_HIP(ctx, hipMalloc(&dp, sizeof(double) * n));
  DACP_HIP(ctx, hipMalloc(&dd, sizeof(double) * n));
  DACP_HIP(ctx, hipMalloc(&de, sizeof(double) * n));
  DACP_HIP(ctx, hipMalloc(&db, sizeof(double) * n));
  DACP_HIP(ctx, hipMemsetAsync(db, 0, sizeof(double) * n, st));
  const int report_every = std::max(1, n / 4);
  const bool blocked = ctx->blocked_min_n > 0 && n >= std::max(ctx->blocked_min_n, 8 * kTB);
  if (blocked) {
    DevBuf pv, pw, pxy;
    DACP_HIP(ctx, pv.alloc(sizeof(double) * n * kTB));
    DACP_HIP(ctx, pw.alloc(sizeof(double) * n * kTB));
    DACP_HIP(ctx, pxy.alloc(sizeof(double) * 2 * kTB));
    double *V = pv.as<double>(), *W = pw.as<double>();
    const int nred = n - 2;
    for (int p0 = 0; p0 < nred; p0 += kTB) {
      const int nbp = std::min(kTB, nred - p0);
      if (verbose() && p0 > 0 && (p0 / kTB) % std::max(1, report_every / kTB) == 0) {
        (void)hipStreamSynchronize(st);
        vlog("eigensolver n=%d: tridiagonalised %d columns (panels)", n, p0);
      }
      for (int j = 0; j < nbp; ++j) {
        const int k = p0 + j;
        const int m = n - k - 1;
        hipLaunchKernelGGL(k_panel_row, dim3((n - k + 255) / 256), dim3(256), 0, st, A, ld, n, k, V, W, j);
        hipLaunchKernelGGL(k_house, dim3(1), dim3(1024), 0, st, A, ld, n, k, dv, dd, de, db);
        hipLaunchKernelGGL(k_symv, dim3((m + 3) / 4), dim3(256), 0, st, A, ld, n, k, dv, db, dp);
        if (j > 0) {
          hipLaunchKernelGGL(k_panel_dots, dim3(2 * kTB), dim3(256), 0, st, V, W, n, k, j, dv, pxy.as<double>());
          hipLaunchKernelGGL(k_panel_corr, dim3((m + 255) / 256), dim3(256), 0, st, dp, V, W, n, k, j,
                             pxy.as<double>(), db);
        }
        hipLaunchKernelGGL(k_wvec, dim3(1), dim3(1024), 0, st, dp, dv, db, n, k);
        hipLaunchKernelGGL(k_panel_store, dim3((n + 255) / 256), dim3(256), 0, st, V, W, n, k, j, dv, dp, db);
      }
      // trailing matrix after the panel: A22 -= V W^T + W V^T on rows / columns >= t
      const int t = p0 + nbp;
      const int mt = n - t;
      if (mt > 0) {
        double *a22 = A + static_cast<int64_t>(t) * ld + t;
        const double *Vt = V + static_cast<int64_t>(t) * kTB, *Wt = W + static_cast<int64_t>(t) * kTB;
        DACP_HIP(ctx, launch_dgemm(0, 1, mt, mt, nbp, -1.0, Vt, kTB, Wt, kTB, 1.0, a22, ld, 0, st));
        DACP_HIP(ctx, launch_dgemm(0, 1, mt, mt, nbp, -1.0, Wt, kTB, Vt, kTB, 1.0, a22, ld, 0, st));
      }
    }
    DACP_HIP(ctx, hipGetLastError());
    DACP_HIP(ctx, hipStreamSynchronize(st));  // the panel buffers are released at scope end
  }
  for (int k = blocked ? n - 2 : 0; k < n - 2; ++k) {
    const int m = n - k - 1;
    if (verbose() && k > 0 && k % report_every == 0) {
      (void)hipStreamSynchronize(st);
      vlog("eigensolver n=%d: tridiagonalised %d columns", n, k);
    }
    hipLaunchKernelGGL(k_house, dim3(1), dim3(1024), 0, st, A, ld, n, k, dv, dd, de, db);
    hipLaunchKernelGGL(k_symv, dim3((m + 3) / 4), dim3(256), 0, st, A, ld, n, k, dv, db, dp);
    hipLaunchKernelGGL(k_wvec, dim3(1), dim3(1024), 0, st, dp, dv, db, n, k);
    hipLaunchKernelGGL(k_syr2, dim3((m + 255) / 256, m), dim3(256), 0, st, A, ld, n, k, dv, dp, db);
  }
  DACP_HIP(ctx, hipGetLastError());
  std::vector<double> d(n), e(n, 0.0);
  double tail[4];
  if (n > 2) {
    DACP_TRY(to_host(ctx, d.data(), dd, sizeof(double) * (n - 2)));
    DACP_TRY(to_host(ctx, e.data(), de, sizeof(double) * (n - 2)));
  }
  DACP_TRY(to_host_2d(ctx, tail, A + static_cast<int64_t>(n - 2) * ld + (n - 2), ld, 2, 2));
  DACP_HIP(ctx, hipStreamSynchronize(st));
  d[n - 2] = tail[0];
  e[n - 2] = tail[2];
  d[n - 1] = tail[3];
  e[n - 1] = 0.0;
  const double t_tri = wall_ms();

  if (Zrows) {
    const int64_t nn = static_cast<int64_t>(n) * n;
    hipLaunchKernelGGL(k_set_identity, dim3((nn + 255) / 256), dim3(256), 0, st, Zrows, (int64_t)n, n);
    constexpr int kQB = 64;  // reflectors per compact-WY block
    if (ctx->blocked_min_n > 0 && n >= std::max(ctx->blocked_min_n, 4 * kQB)) {
      // Qc <- Qc P_k for k = n-3 .. 0, a block of reflectors at a time (last block first):
      // P_k0 ... P_(k0+kb-1) = I - V T V^T (T upper triangular, T_jj = beta_j,
      // T[0:j, j] = -beta_j T[0:j, 0:j] (V[:, 0:j]^T v_j)), so Qc <- Qc - (Qc V) T^T V^T on the rows and
      // columns after k0 (the others are untouched identity rows / zero columns of V).
      const int nref = n - 2;
      std::vector<double> beta(n), g(kQB * kQB), T(kQB * kQB);
      DACP_TRY(to_host(ctx, beta.data(), db, sizeof(double) * n));
      DevBuf vt, gd, td, w1, w2;
      DACP_HIP(ctx, vt.alloc(sizeof(double) * kQB * n));
      DACP_HIP(ctx, gd.alloc(sizeof(double) * kQB * kQB));
      DACP_HIP(ctx, td.alloc(sizeof(double) * kQB * kQB));
      DACP_HIP(ctx, w1.alloc(sizeof(double) * kQB * n));
      DACP_HIP(ctx, w2.alloc(sizeof(double) * kQB * n));
      for (int k0 = ((nref - 1) / kQB) * kQB; k0 >= 0; k0 -= kQB) {
        const int kb = std::min(kQB, nref - k0);
        const int c0 = k0 + 1, R = n - c0;
        hipLaunchKernelGGL(k_build_vt, dim3(static_cast<unsigned>((static_cast<int64_t>(kb) * n + 255) / 256)),
                           dim3(256), 0, st, A, ld, n, k0, kb, vt.as<double>());
        DACP_HIP(ctx, hipGetLastError());
        // G = V^T V over the columns after k0
        DACP_HIP(ctx, launch_dgemm(0, 1, kb, kb, R, 1.0, vt.as<double>() + c0, n, vt.as<double>() + c0, n, 0.0,
                                   gd.as<double>(), kb, 0, st));
        DACP_TRY(to_host(ctx, g.data(), gd.p, sizeof(double) * kb * kb));
        std::fill(T.begin(), T.end(), 0.0);
        for (int j = 0; j < kb; ++j) {
          const double bj = beta[k0 + j];
          for (int i = 0; i < j; ++i) {
            double acc = 0.0;
            for (int q = i; q < j; ++q) acc += T[i * kb + q] * g[q * kb + j];
            T[i * kb + j] = -bj * acc;
          }
          T[j * kb + j] = bj;
        }
        DACP_TRY(to_device(ctx, td.p, T.data(), sizeof(double) * kb * kb));
        double *qs = Zrows + static_cast<int64_t>(c0) * n + c0;
        // W1 = Qc_sub V_sub (R x kb), W2 = W1 T^T, Qc_sub -= W2 V_sub^T
        DACP_HIP(ctx, launch_dgemm(0, 1, R, kb, R, 1.0, qs, n, vt.as<double>() + c0, n, 0.0, w1.as<double>(), kb, 0,
                                   st));
        DACP_HIP(ctx, launch_dgemm(0, 1, R, kb, kb, 1.0, w1.as<double>(), kb, td.as<double>(), kb, 0.0,
                                   w2.as<double>(), kb, 0, st));
        DACP_HIP(ctx, launch_dgemm(0, 0, R, R, kb, -1.0, w2.as<double>(), kb, vt.as<double>() + c0, n, 1.0, qs, n,
                                   0, st));
      }
      DACP_HIP(ctx, hipStreamSynchronize(st));  // vt, w1, w2 are released at scope end
    } else {
      for (int k = n - 3; k >= 0; --k) {
        const int rows = n - k - 1;
        hipLaunchKernelGGL(k_qupdate, dim3((rows + 3) / 4), dim3(256), 0, st, Zrows, (int64_t)n, A, ld, n, k, db);
      }
    }
    DACP_HIP(ctx, hipGetLastError());
    if (verbose()) (void)hipStreamSynchronize(st);
  }
  const double t_q = wall_ms();

  if (Zrows && ctx->dc_min_n > 0 && n >= ctx->dc_min_n) {
    // Eigenvectors of T by divide and conquer, then rows of (Q Y)^T = Y^T Q^T = Zt * Qc.
    DevBuf zt, qc;
    DACP_HIP(ctx, zt.alloc(static_cast<size_t>(n) * n * sizeof(double)));
    DACP_HIP(ctx, qc.alloc(static_cast<size_t>(n) * n * sizeof(double)));
    DACP_HIP(ctx, hipMemcpyAsync(qc.p, Zrows, static_cast<size_t>(n) * n * sizeof(double), hipMemcpyDeviceToDevice, st));
    DACP_HIP(ctx, hipStreamSynchronize(st));  // the Q-formation kernels read db and A
    (void)hipFree(dv);
    (void)hipFree(dp);
    (void)hipFree(dd);
    (void)hipFree(de);
    (void)hipFree(db);
    dacp_status drc = dc_tridiag(ctx, n, d.data(), e.data(), w, zt.as<double>());
    if (drc) return drc;
    const double t_dc = wall_ms();
    DACP_HIP(ctx, launch_dgemm(0, 0, n, n, n, 1.0, zt.as<double>(), n, qc.as<double>(), n, 0.0, Zrows, n, 0, st));
    DACP_HIP(ctx, hipStreamSynchronize(st));
    vlog("eigensolver n=%d timing: tridiagonalise %.0f ms, form Q %.0f ms, divide and conquer %.0f ms, back-transform "
         "%.0f ms", n, t_tri - t_begin, t_q - t_tri, t_dc - t_q, wall_ms() - t_dc);
    return DACP_OK;
  }

  // QR on the host; rotations batched into pinned memory and replayed on the GPU.
  const size_t flush_pairs = size_t(1) << 24;
  const size_t cap_pairs = flush_pairs + static_cast<size_t>(n);
  std::vector<double> rot;
  std::vector<Sweep> sweeps;
  double *pinned = nullptr, *drot = nullptr;
  dacp_status frc = DACP_OK;
  if (Zrows) {
    rot.reserve(2 * cap_pairs);
    DACP_HIP(ctx, hipMalloc(&drot, cap_pairs * 2 * sizeof(double)));
    DACP_HIP(ctx, hipHostMalloc(&pinned, cap_pairs * 2 * sizeof(double), hipHostMallocDefault));
  }
  auto flush = [&]() {
    if (sweeps.empty() || frc != DACP_OK) return;
    hipError_t he = hipStreamSynchronize(st);  // the previous batch no longer reads the buffers
    if (he == hipSuccess) {
      std::memcpy(pinned, rot.data(), rot.size() * sizeof(double));
      he = hipMemcpyAsync(drot, pinned, rot.size() * sizeof(double), hipMemcpyHostToDevice, st);
    }
    if (he == hipSuccess) {
      for (size_t s0 = 0; s0 < sweeps.size(); s0 += NSW) {
        SweepBatch sb;
        sb.count = static_cast<int>(std::min<size_t>(NSW, sweeps.size() - s0));
        sb.rmin = n;
        sb.rmax = -1;
        for (int i = 0; i < NSW; ++i) {
          if (i < sb.count) {
            const Sweep &sw = sweeps[s0 + i];
            sb.p[i] = sw.p;
            sb.q[i] = sw.q;
            sb.off[i] = static_cast<int64_t>(sw.off);
            sb.rmin = std::min(sb.rmin, sw.p);
            sb.rmax = std::max(sb.rmax, sw.q);
          } else {
            sb.p[i] = 0;
            sb.q[i] = 0;
            sb.off[i] = 0;
          }
        }
        hipLaunchKernelGGL(k_rot_batch, dim3((n + 63) / 64), dim3(64), 0, st, Zrows, (int64_t)n, n, sb, drot);
      }
      he = hipGetLastError();
    }
    if (he != hipSuccess) frc = hip_err(ctx, he, "rotation replay");
    rot.clear();
    sweeps.clear();
  };
  auto sink = [&](int p, int q, const double *cs) {
    if (!Zrows) return;
    if (rot.size() / 2 + static_cast<size_t>(q - p) > cap_pairs) flush();
    sweeps.push_back(Sweep{p, q, rot.size() / 2});
    rot.insert(rot.end(), cs, cs + 2 * static_cast<size_t>(q - p));
  };
  vlog("eigensolver n=%d: tridiagonal form ready, QR iteration%s", n, Zrows ? " with vectors" : "");
  const bool ok = tridiag_qr(d, e, n, sink);
  const double t_qr = wall_ms();
  vlog("eigensolver n=%d: QR done", n);
  if (ok && Zrows) flush();
  hipError_t he = hipStreamSynchronize(st);
  if (drot) (void)hipFree(drot);
  if (pinned) (void)hipHostFree(pinned);
  (void)hipFree(dv);
  (void)hipFree(dp);
  (void)hipFree(dd);
  (void)hipFree(de);
  (void)hipFree(db);
  const double t_replay = wall_ms();
  vlog("eigensolver n=%d timing: tridiagonalise %.0f ms, form Q %.0f ms, QR (host, overlapping replay) %.0f ms, "
       "replay tail %.0f ms", n, t_tri - t_begin, t_q - t_tri, t_qr - t_q, t_replay - t_qr);
  if (frc != DACP_OK) return frc;
  if (he != hipSuccess) return hip_err(ctx, he, "eigensolver");
  dacp_status rc = ok ? DACP_OK : DACP_E_CONVERGENCE;
  if (rc != DACP_OK) return set_err(ctx, rc, "symmetric QR did not converge");

  // sort ascending, permuting eigenvector rows
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int i, int j) { return d[i] < d[j]; });
  for (int i = 0; i < n; ++i) w[i] = d[perm[i]];
  if (Zrows) {
    double *tmp = nullptr;
    int *dperm = nullptr;
    const int64_t nn = static_cast<int64_t>(n) * n;
    DACP_HIP(ctx, hipMalloc(&tmp, sizeof(double) * nn));
    DACP_HIP(ctx, hipMalloc(&dperm, sizeof(int) * n));
    DACP_TRY(to_device(ctx, dperm, perm.data(), sizeof(int) * n));
    DACP_HIP(ctx, hipMemcpyAsync(tmp, Zrows, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_gather_rows, dim3((nn + 255) / 256), dim3(256), 0, st, tmp, (int64_t)n, Zrows, (int64_t)n,
                       dperm, nullptr, n, n);
    DACP_HIP(ctx, hipGetLastError());
    DACP_HIP(ctx, hipStreamSynchronize(st));
    (void)hipFree(tmp);
    (void)hipFree(dperm);
  }
  return DACP_OK;
}

hipError_t launch_gather_rows(const double *src, int64_t lds, double *dst, int64_t ldd, const int *perm,
                              const double *scale, int rows, int cols, hipStream_t s) {
  const int64_t nn = static_cast<int64_t>(rows) * cols;
  if (nn == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3((nn + 255) / 256), dim3(256), 0, s, src, lds, dst, ldd, perm, scale, rows,
                     cols);
  return hipGetLastError();
}

}  // namespace dacp
