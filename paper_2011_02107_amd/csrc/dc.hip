// Divide-and-conquer eigen-decomposition of a symmetric tridiagonal matrix
// (Cuppen's tear, deflation and the secular equation; eigenvectors of each
// rank-one update from the Gu-Eisenstat recomputed z so they stay orthogonal
// to working precision).  The host keeps the O(n) bookkeeping; the secular
// roots, the eigenvector matrices of the rank-one problems and their products
// with the child eigenvectors (FP64 MFMA GEMMs) run on the GPU.
//
// Eigenvectors are kept as rows: Zc[lo + j][lo + i] = component i of
// eigenvector j of the block [lo, hi).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "host_rules.h"
#include "internal.h"

namespace dacp {

namespace {

constexpr int kLeaf = 32;

// Root j of f(lam) = 1 + rho sum_i z_i^2 / (d_i - lam) in (d_j, d_{j+1}) (or
// (d_{k-1}, d_{k-1} + rho |z|^2] for the last one), stored as origin index
// org[j] and offset tau[j] from d[org[j]] so that d_i - lam = (d_i - d_org) - tau
// keeps full relative accuracy near the pole.
__global__ void k_secular(const double *d, const double *z, int k, double rho, int *org, double *tau) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  double zz = 0.0;
  for (int i = 0; i < k; ++i) zz += z[i] * z[i];
  const double hi_gap = (j + 1 < k) ? d[j + 1] - d[j] : rho * zz;
  // f at the middle of the interval decides the nearer pole
  int o = j;
  {
    const double mid = 0.5 * hi_gap;
    double f = 1.0;
    for (int i = 0; i < k; ++i) f += rho * z[i] * z[i] / ((d[i] - d[j]) - mid);
    if (j + 1 < k && f <= 0.0) o = j + 1;
  }
  const double base = d[o] - d[j];  // 0 or hi_gap
  // bracket for tau relative to d[o]
  double lo, hi;
  if (o == j) {
    lo = 0.0;
    hi = (j + 1 < k) ? 0.5 * hi_gap : hi_gap;
  } else {
    lo = -0.5 * hi_gap;
    hi = 0.0;
  }
  auto feval = [&](double t, double &fp) {
    double f = 1.0;
    fp = 0.0;
    for (int i = 0; i < k; ++i) {
      const double del = (d[i] - d[o]) - t;
      const double q = z[i] / del;
      f += rho * z[i] * q;
      fp += rho * q * q;
    }
    return f;
  };
  double t = 0.5 * (lo + hi);
  for (int it = 0; it < 70; ++it) {
    double fp;
    const double f = feval(t, fp);
    if (f > 0.0) hi = t;
    else lo = t;
    const double tn = 0.5 * (lo + hi);
    if (tn == t) break;
    t = tn;
  }
  for (int it = 0; it < 4; ++it) {  // Newton polish inside the bracket
    double fp;
    const double f = feval(t, fp);
    if (!(fp > 0.0)) break;
    double tn = t - f / fp;
    if (!(tn > lo && tn < hi)) break;
    t = tn;
  }
  (void)base;
  org[j] = o;
  tau[j] = t;
}

// zhat_i = sign(z_i) sqrt(prod_j (lam_j - d_i) / (rho prod_{j != i} (d_j - d_i)))  (Gu-Eisenstat)
__global__ void k_zhat(const double *d, const double *z, int k, double rho, const int *org, const double *tau,
                       double *zh) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  // (lam_i - d_i) first, then the ratios (lam_j - d_i)/(d_j - d_i), each of moderate size
  double p = -((d[i] - d[org[i]]) - tau[i]);
  for (int j = 0; j < k; ++j) {
    if (j == i) continue;
    const double lmd = -((d[i] - d[org[j]]) - tau[j]);  // lam_j - d_i
    p *= lmd / (d[j] - d[i]);
  }
  p /= rho;
  const double v = sqrt(fabs(p));
  zh[i] = (z[i] >= 0.0) ? v : -v;
}

// U[j][i] = zhat_i / (d_i - lam_j), rows normalised afterwards.
__global__ void k_form_u(const double *d, const double *zh, int k, const int *org, const double *tau, double *U) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(k) * k) return;
  const int j = static_cast<int>(e / k), i = static_cast<int>(e - static_cast<int64_t>(j) * k);
  U[e] = zh[i] / ((d[i] - d[org[j]]) - tau[j]);
}

__global__ void k_normalise_rows(double *U, int k, int64_t ld, int ncols) {
  __shared__ double red[256];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int i = threadIdx.x; i < ncols; i += blockDim.x) s += U[j * ld + i] * U[j * ld + i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  const double inv = 1.0 / sqrt(red[0]);
  for (int i = threadIdx.x; i < ncols; i += blockDim.x) U[j * ld + i] *= inv;
  (void)k;
}

// Sequential list of plane rotations on row pairs (p, q): row_p <- c row_p - s row_q,
// row_q <- s row_p + c row_q; every lane owns one column.
__global__ void k_row_rotations(double *Z, int64_t ld, int col0, int ncols, const int *pq, const double *cs, int nrot) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= ncols) return;
  double *zc = Z + col0 + col;
  for (int r = 0; r < nrot; ++r) {
    const int p = pq[2 * r], q = pq[2 * r + 1];
    const double c = cs[2 * r], s = cs[2 * r + 1];
    const double a = zc[static_cast<int64_t>(p) * ld], b = zc[static_cast<int64_t>(q) * ld];
    zc[static_cast<int64_t>(p) * ld] = c * a - s * b;
    zc[static_cast<int64_t>(q) * ld] = s * a + c * b;
  }
}

// dst[r][c] = src[rows[r]][col0 + c]
__global__ void k_gather_block(const double *src, int64_t lds, const int *rows, int col0, int nrows, int ncols,
                               double *dst, int64_t ldd) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(nrows) * ncols) return;
  const int r = static_cast<int>(e / ncols), c = static_cast<int>(e - static_cast<int64_t>(r) * ncols);
  dst[r * ldd + c] = src[static_cast<int64_t>(rows[r]) * lds + col0 + c];
}

// dst[rows[r]][col0 + c] = src[r][c]
__global__ void k_scatter_block(const double *src, int64_t lds, const int *rows, int col0, int nrows, int ncols,
                                double *dst, int64_t ldd) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(nrows) * ncols) return;
  const int r = static_cast<int>(e / ncols), c = static_cast<int>(e - static_cast<int64_t>(r) * ncols);
  dst[static_cast<int64_t>(rows[r]) * ldd + col0 + c] = src[r * lds + c];
}

inline unsigned nblk(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

struct DcWork {
  dacp_ctx ctx;
  int n;
  double *Z;  // n x n device, rows = eigenvectors
  std::vector<double> w;  // eigenvalues of solved blocks (ascending within each block)
  // device scratch, grown on demand
  DevBuf dd, dz, dtau, dzh, dU, dA, dB, dcs;
  DevBuf dorg, drows, dpq;
};

dacp_status ensure(dacp_ctx ctx, DevBuf &b, size_t bytes) {
  if (b.bytes >= bytes) return DACP_OK;
  DACP_HIP(ctx, b.alloc(bytes));
  return DACP_OK;
}

dacp_status solve(DcWork &W, std::vector<double> &d, std::vector<double> &e, int lo, int hi);

// Merge the solved halves [lo, m) and [m, hi), torn with rho = |beta|.
dacp_status merge(DcWork &W, int lo, int m, int hi, double beta) {
  dacp_ctx ctx = W.ctx;
  hipStream_t st = ctx->stream;
  const int n = hi - lo;
  const int n1 = m - lo;
  {
    // every scratch buffer of this merge sized for the whole block before any kernel uses it
    const size_t nn = static_cast<size_t>(n) * n;
    dacp_status s0 = DACP_OK;
    if ((s0 = ensure(ctx, W.dA, nn * sizeof(double)))) return s0;
    if ((s0 = ensure(ctx, W.dB, nn * sizeof(double)))) return s0;
    if ((s0 = ensure(ctx, W.dU, nn * sizeof(double)))) return s0;
    if ((s0 = ensure(ctx, W.dd, n * sizeof(double)))) return s0;
    if ((s0 = ensure(ctx, W.dz, n * sizeof(double)))) return s0;
    if ((s0 = ensure(ctx, W.dtau, n * sizeof(double)))) return s0;
    if ((s0 = ensure(ctx, W.dzh, n * sizeof(double)))) return s0;
    if ((s0 = ensure(ctx, W.dorg, n * sizeof(int)))) return s0;
    if ((s0 = ensure(ctx, W.drows, n * sizeof(int)))) return s0;
    if ((s0 = ensure(ctx, W.dpq, 2 * n * sizeof(int)))) return s0;
    if ((s0 = ensure(ctx, W.dcs, 2 * n * sizeof(double)))) return s0;
  }
  const double sgn = beta >= 0.0 ? 1.0 : -1.0;
  double rho = std::fabs(beta);
  // z = [sgn * last row of Q1; first row of Q2]: component m-1 of the first half's
  // eigenvectors, component m of the second half's.
  std::vector<double> z(n);
  {
    // both strided columns gathered into the merge's own z buffer, then one copy to the host
    std::vector<double> col(n);
    DACP_HIP(ctx, launch_copy_cols(W.Z + static_cast<int64_t>(lo) * W.n + (m - 1), W.n, W.dz.as<double>(), 1, n1, 1,
                                   st));
    DACP_HIP(ctx, launch_copy_cols(W.Z + static_cast<int64_t>(m) * W.n + m, W.n, W.dz.as<double>() + n1, 1, n - n1, 1,
                                   st));
    DACP_TRY(to_host(ctx, col.data(), W.dz.p, static_cast<size_t>(n) * sizeof(double)));
    for (int i = 0; i < n1; ++i) z[i] = sgn * col[i];
    for (int i = n1; i < n; ++i) z[i] = col[i];
  }
  std::vector<double> dv(W.w.begin() + lo, W.w.begin() + hi);
  // normalise z (rho absorbs |z|^2)
  double zn = 0.0;
  for (double v : z) zn += v * v;
  zn = std::sqrt(zn);
  for (double &v : z) v /= zn;
  rho *= zn * zn;
  // sort, deflate and list the secular problem (host bookkeeping, host_rules.cpp)
  rules::DcDeflation df = rules::dc_deflate(dv, z, rho, lo);
  const std::vector<double> &ds = df.ds, &zs = df.zs;
  const std::vector<int> &rowid = df.rowid, &rot_pq = df.rot_pq, &nd = df.nd;
  const std::vector<double> &rot_cs = df.rot_cs;
  const std::vector<char> &defl = df.defl;
  if (!rot_pq.empty()) {
    const int nr = static_cast<int>(rot_cs.size() / 2);
    DACP_TRY(to_device(ctx, W.dpq.p, rot_pq.data(), rot_pq.size() * sizeof(int)));
    DACP_TRY(to_device(ctx, W.dcs.p, rot_cs.data(), rot_cs.size() * sizeof(double)));
    hipLaunchKernelGGL(k_row_rotations, dim3(nblk(n, 64)), dim3(64), 0, st, W.Z, (int64_t)W.n, lo, n,
                       W.dpq.as<int>(), W.dcs.as<double>(), nr);
    DACP_HIP(ctx, hipGetLastError());
  }
  // non-deflated problem
  const int k = static_cast<int>(nd.size());
  // final eigenvalue list: (value, kind, index) kind 0 = deflated (rowid), 1 = secular root (nd index)
  std::vector<rules::DcEntry> ents;
  for (int j = 0; j < n; ++j)
    if (defl[j]) ents.push_back({ds[j], 0, rowid[j]});
  if (k > 0) {
    std::vector<double> dk(k), zk(k);
    std::vector<int> rk(k);
    for (int q = 0; q < k; ++q) {
      dk[q] = ds[nd[q]];
      zk[q] = zs[nd[q]];
      rk[q] = rowid[nd[q]];
    }
    const size_t kk = static_cast<size_t>(k) * k;
    DACP_TRY(to_device(ctx, W.dd.p, dk.data(), k * sizeof(double)));
    DACP_TRY(to_device(ctx, W.dz.p, zk.data(), k * sizeof(double)));
    hipLaunchKernelGGL(k_secular, dim3(nblk(k, 64)), dim3(64), 0, st, W.dd.as<double>(), W.dz.as<double>(), k, rho,
                       W.dorg.as<int>(), W.dtau.as<double>());
    hipLaunchKernelGGL(k_zhat, dim3(nblk(k, 64)), dim3(64), 0, st, W.dd.as<double>(), W.dz.as<double>(), k, rho,
                       W.dorg.as<int>(), W.dtau.as<double>(), W.dzh.as<double>());
    hipLaunchKernelGGL(k_form_u, dim3(nblk(static_cast<int64_t>(kk), 256)), dim3(256), 0, st, W.dd.as<double>(),
                       W.dzh.as<double>(), k, W.dorg.as<int>(), W.dtau.as<double>(), W.dU.as<double>());
    hipLaunchKernelGGL(k_normalise_rows, dim3(k), dim3(256), 0, st, W.dU.as<double>(), k, (int64_t)k, k);
    // old rows of the non-deflated entries (block columns [lo, hi))
    DACP_TRY(to_device(ctx, W.drows.p, rk.data(), k * sizeof(int)));
    hipLaunchKernelGGL(k_gather_block, dim3(nblk(static_cast<int64_t>(k) * n, 256)), dim3(256), 0, st, W.Z,
                       (int64_t)W.n, W.drows.as<int>(), lo, k, n, W.dA.as<double>(), (int64_t)n);
    // new rows = U * old rows
    DACP_HIP(ctx, launch_dgemm(0, 0, k, n, k, 1.0, W.dU.as<double>(), k, W.dA.as<double>(), n, 0.0, W.dB.as<double>(),
                               n, 0, st));
    DACP_HIP(ctx, hipGetLastError());
    std::vector<int> org(k);
    std::vector<double> tau(k);
    DACP_TRY(to_host(ctx, org.data(), W.dorg.p, k * sizeof(int)));
    DACP_TRY(to_host(ctx, tau.data(), W.dtau.p, k * sizeof(double)));
    DACP_HIP(ctx, hipStreamSynchronize(st));
    for (int q = 0; q < k; ++q) {
      const double v = dk[org[q]] + tau[q];
      if (!std::isfinite(v)) return set_err(ctx, DACP_E_NUMERIC, "divide and conquer: non-finite root");
      ents.push_back({v, 1, q});
    }
  }
  // place rows: deflated rows are copied (they may currently sit anywhere in the block), roots
  // come from dB; stage everything through dA (n x n of the block) then copy to rows lo..hi
  const rules::DcPlacement pl = rules::dc_place(std::move(ents), k);
  const std::vector<int> &src_defl = pl.src_defl, &dst_defl = pl.dst_defl;
  for (int t = 0; t < n; ++t) W.w[lo + t] = pl.w[t];
  // deflated: gather Z rows -> dA rows dst
  DevBuf tmp_idx;
  if (!src_defl.empty()) {
    std::vector<int> idx(src_defl);
    idx.insert(idx.end(), dst_defl.begin(), dst_defl.end());
    DACP_HIP(ctx, tmp_idx.alloc(idx.size() * sizeof(int)));
    DACP_TRY(to_device(ctx, tmp_idx.p, idx.data(), idx.size() * sizeof(int)));
    const int nd2 = static_cast<int>(src_defl.size());
    // stage: gather into contiguous rows, then scatter into dA at dst rows
    DevBuf stage;
    DACP_HIP(ctx, stage.alloc(static_cast<size_t>(nd2) * n * sizeof(double)));
    hipLaunchKernelGGL(k_gather_block, dim3(nblk(static_cast<int64_t>(nd2) * n, 256)), dim3(256), 0, st, W.Z,
                       (int64_t)W.n, tmp_idx.as<int>(), lo, nd2, n, stage.as<double>(), (int64_t)n);
    hipLaunchKernelGGL(k_scatter_block, dim3(nblk(static_cast<int64_t>(nd2) * n, 256)), dim3(256), 0, st,
                       stage.as<double>(), (int64_t)n, tmp_idx.as<int>() + nd2, 0, nd2, n, W.dA.as<double>(),
                       (int64_t)n);
    DACP_HIP(ctx, hipGetLastError());
    DACP_HIP(ctx, hipStreamSynchronize(st));
  }
  if (k > 0) {
    // dB row q (root q) -> dA row dst_of_root[q]
    DACP_TRY(to_device(ctx, W.drows.p, pl.dst_of_root.data(), k * sizeof(int)));
    hipLaunchKernelGGL(k_scatter_block, dim3(nblk(static_cast<int64_t>(k) * n, 256)), dim3(256), 0, st,
                       W.dB.as<double>(), (int64_t)n, W.drows.as<int>(), 0, k, n, W.dA.as<double>(), (int64_t)n);
    DACP_HIP(ctx, hipGetLastError());
  }
  // dA (n x n) -> Z rows lo..hi, columns lo..hi
  DACP_HIP(ctx, launch_copy_cols(W.dA.as<double>(), n, W.Z + static_cast<int64_t>(lo) * W.n + lo, W.n, n, n, st));
  DACP_HIP(ctx, hipStreamSynchronize(st));
  return DACP_OK;
}

dacp_status solve(DcWork &W, std::vector<double> &d, std::vector<double> &e, int lo, int hi) {
  const int n = hi - lo;
  if (n <= kLeaf) {
    std::vector<double> w(n), Zh(static_cast<size_t>(n) * n);
    if (!host_tridiag_eig(d.data() + lo, e.data() + lo, n, w.data(), Zh.data()))
      return set_err(W.ctx, DACP_E_CONVERGENCE, "divide and conquer: leaf QR did not converge");
    std::vector<double> rows(static_cast<size_t>(n) * n);
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i) rows[static_cast<size_t>(j) * n + i] = Zh[static_cast<size_t>(i) * n + j];
    for (int j = 0; j < n; ++j) W.w[lo + j] = w[j];
    DACP_TRY(to_device_2d(W.ctx, W.Z + static_cast<int64_t>(lo) * W.n + lo, W.n, rows.data(), n, n));
    DACP_HIP(W.ctx, hipStreamSynchronize(W.ctx->stream));  // `rows` goes out of scope
    return DACP_OK;
  }
  const int m = lo + n / 2;
  const double beta = e[m - 1];
  // tear: T = diag(T1 - |beta| e e^T, T2 - |beta| e e^T) + |beta| v v^T, v = (sign(beta) e_last; e_first)
  d[m - 1] -= std::fabs(beta);
  d[m] -= std::fabs(beta);
  dacp_status st = solve(W, d, e, lo, m);
  if (st) return st;
  st = solve(W, d, e, m, hi);
  if (st) return st;
  if (beta == 0.0) {
    // already split: merge the two sorted halves without a rank-one update
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::vector<double> wv(W.w.begin() + lo, W.w.begin() + hi);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return wv[a] < wv[b]; });
    DevBuf idx, stage;
    std::vector<int> src(n);
    for (int t = 0; t < n; ++t) {
      src[t] = lo + order[t];
      W.w[lo + t] = wv[order[t]];
    }
    DACP_HIP(W.ctx, idx.alloc(n * sizeof(int)));
    DACP_HIP(W.ctx, stage.alloc(static_cast<size_t>(n) * n * sizeof(double)));
    DACP_TRY(to_device(W.ctx, idx.p, src.data(), n * sizeof(int)));
    hipLaunchKernelGGL(k_gather_block, dim3(nblk(static_cast<int64_t>(n) * n, 256)), dim3(256), 0, W.ctx->stream,
                       W.Z, (int64_t)W.n, idx.as<int>(), lo, n, n, stage.as<double>(), (int64_t)n);
    DACP_HIP(W.ctx, launch_copy_cols(stage.as<double>(), n, W.Z + static_cast<int64_t>(lo) * W.n + lo, W.n, n, n,
                                     W.ctx->stream));
    DACP_HIP(W.ctx, hipStreamSynchronize(W.ctx->stream));
    return DACP_OK;
  }
  return merge(W, lo, m, hi, beta);
}

}  // namespace

// Eigen-decomposition of the symmetric tridiagonal (d, e) (e[i] couples i and i+1).
// w (host) ascending; Z (device n x n, ld n): row j = eigenvector j.  Z is zero-filled
// here (off-block entries of the merged halves must read as zero).
dacp_status dc_tridiag(dacp_ctx ctx, int n, const double *d_in, const double *e_in, double *w, double *Z) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(d_in[i]) || (i + 1 < n && !std::isfinite(e_in[i])))
      return set_err(ctx, DACP_E_NUMERIC, "divide and conquer: non-finite tridiagonal entry");
  DACP_HIP(ctx, hipMemsetAsync(Z, 0, static_cast<size_t>(n) * n * sizeof(double), ctx->stream));
  DcWork W;
  W.ctx = ctx;
  W.n = n;
  W.Z = Z;
  W.w.assign(n, 0.0);
  std::vector<double> d(d_in, d_in + n), e(n, 0.0);
  for (int i = 0; i + 1 < n; ++i) e[i] = e_in[i];
  dacp_status st = solve(W, d, e, 0, n);
  if (st) return st;
  DACP_HIP(ctx, hipStreamSynchronize(ctx->stream));
  std::copy(W.w.begin(), W.w.end(), w);
  return DACP_OK;
}

}  // namespace dacp
