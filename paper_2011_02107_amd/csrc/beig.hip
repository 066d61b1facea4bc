// Batched dense symmetric eigensolver for many small subspace problems (App. C, one workgroup per
// matrix).  The per-problem solver of eig.hip issues several kernels per column and is bound by
// launches at n of a few hundred; here one launch covers every problem of a batch:
//   1. Householder tridiagonalisation in place (one column per step, the step's vectors in LDS;
//      each step's rank-2 update is applied in the next step's pass over the trailing block);
//   2. every eigenvalue of the tridiagonal by bisection, one per thread, for the QR shifts;
//   3. implicit symmetric QR on (d, e), shifted by the nearest eigenvalue not yet deflated (else
//      Wilkinson's shift), in batches of up to S sweeps: wave 0 chases the bulges of batch b+1
//      (the chase carries its running values in registers) while waves 1.. apply the Givens
//      rotations of batch b to the rows of Zr (rows = eigenvectors of the tridiagonal, starting
//      from I), one column per thread, all S sweeps in one pass down the column.  On a large
//      unreduced block the S sweeps of a batch take S shifts chosen at its start and run in
//      lockstep, lane s of wave 0 chasing sweep s a fixed number of rotations behind lane s-1;
//      small blocks, and the batch after a pipelined one that deflated nothing, chase one sweep
//      after another on lane 0 with the shift taken after each.
// Two more launches over every matrix then turn the rows of Zr into eigenvectors of A, Zr Q^T with
// Q = H_0 H_1 ... H_(n-3), never forming Q: k_wy_prep writes each block of kWY reflectors in
// compact WY form (the masked rows V and the triangular T), k_wy_apply applies the blocks to Zr
// from the right, last block first, RB rows of Zr per workgroup held in LDS (rows are
// independent).  The host sorts the eigenvalues and gathers the rows in that order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "internal.h"

namespace dacp {

namespace {

constexpr int kBT = 1024;       // threads per problem
constexpr int kBWaves = kBT / 64;
constexpr int kApplyThreads = kBT - 64;  // waves 1.. apply rotations while wave 0 chases
constexpr int kPrefetch = 8;             // rows of a column loaded ahead of their rotations
constexpr int kRowBatch = 16;            // rows of a column in flight in the BLAS-2 passes
constexpr int kFuseBatch = 8;            // the same in the fused update-and-product pass
constexpr size_t kLdsMax = 160 * 1024;
constexpr int kPipeLag = 5;     // rotations between consecutive sweeps of a pipelined batch
constexpr int kPipeMin = 48;    // smallest unreduced block chased as a pipelined batch
constexpr int kShiftSlots = 8;  // LDS slots for a pipelined batch's shifts (S <= 8)
constexpr int kWY = 64;         // reflectors per compact-WY block of the back-transformation
constexpr int kRB = 8;          // rows of Zr per workgroup of the back-transformation

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

// The same pair (up to a common sign) through one reciprocal square root when x^2 + z^2 can
// neither overflow nor underflow: r = sqrt(x^2 + z^2), c = x / r, s = -z / r.  The fast form is
// computed first and the range test only picks the stable one, off the chase's dependent chain.
__device__ void givens_fast(double x, double z, double &c, double &s) {
  const double r2 = fma(x, x, z * z);
  const double ir = rsqrt(r2);
  c = x * ir;
  s = -z * ir;
  if (!(r2 > 1e-290 && r2 < 1e290)) givens_pair(x, z, c, s);
}

// One implicit QR sweep with shift mu on the unreduced block p..q of (d, e) (Golub and Van Loan's
// symmetric QR step).  The chase keeps d[k], e[k] and its bulge in registers and reads
// d, e two rotations ahead (those reads may run up to two entries past e's end, into the
// reduction slots: in the workgroup's LDS and unused); the pairs (c, s) of rotations p..q-1 go
// to cs.
__device__ void qr_sweep(double *d, double *e, int p, int q, double mu, double *cs) {
  double dk = d[p], ek = e[p], dn = d[p + 1], en = e[p + 1], dn2 = d[p + 2], en2 = e[p + 2];
  double x = dk - mu, z = ek;
  double c, sn;
  for (int k = p; k < q - 1; ++k) {
    const double dn3 = d[k + 3], en3 = e[k + 3];
    givens_fast(x, z, c, sn);
    if (k > p) e[k - 1] = c * x - sn * z;
    const double c2 = c * c, s2 = sn * sn, csn = c * sn;
    d[k] = c2 * dk - 2.0 * csn * ek + s2 * dn;
    const double ndk1 = s2 * dk + 2.0 * csn * ek + c2 * dn;
    x = csn * (dk - dn) + (c2 - s2) * ek;
    z = -sn * en;
    cs[2 * (k - p)] = c;
    cs[2 * (k - p) + 1] = sn;
    dk = ndk1;
    ek = c * en;
    dn = dn2;
    en = en2;
    dn2 = dn3;
    en2 = en3;
  }
  givens_fast(x, z, c, sn);
  if (q - 1 > p) e[q - 2] = c * x - sn * z;
  const double c2 = c * c, s2 = sn * sn, csn = c * sn;
  d[q - 1] = c2 * dk - 2.0 * csn * ek + s2 * dn;
  d[q] = s2 * dk + 2.0 * csn * ek + c2 * dn;
  e[q - 1] = csn * (dk - dn) + (c2 - s2) * ek;
  cs[2 * (q - 1 - p)] = c;
  cs[2 * (q - 1 - p) + 1] = sn;
}

// Eigenvalue j (ascending, 0-based) of the symmetric tridiagonal (d, e) by bisection inside
// [lo, hi] on the Sturm count: the number of negative pivots of the L D L^T factorisation of
// T - x I is the number of eigenvalues below x.  A pivot smaller in magnitude than pivmin is
// replaced by -pivmin.
__device__ double bisect_eig(const double *d, const double *e, int n, int j, double lo, double hi, double pivmin) {
  for (int it = 0; it < 128; ++it) {
    const double x = 0.5 * (lo + hi);
    if (!(x > lo && x < hi)) break;
    int cnt = 0;
    double piv = d[0] - x;
    if (fabs(piv) < pivmin) piv = -pivmin;
    cnt += piv < 0.0;
    for (int i = 1; i < n; ++i) {
      piv = (d[i] - x) - e[i - 1] * e[i - 1] / piv;
      if (fabs(piv) < pivmin) piv = -pivmin;
      cnt += piv < 0.0;
    }
    if (cnt > j) hi = x;
    else lo = x;
  }
  return 0.5 * (lo + hi);
}

// Index of the eigenvalue not yet deflated (used[i] == 0) nearest to x in the ascending list lam,
// or -1 when every one is used.
__device__ int nearest_unused(const double *lam, const double *used, int n, double x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) / 2;
    if (lam[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  int l = lo - 1, r = lo;
  while (l >= 0 && used[l] != 0.0) --l;
  while (r < n && used[r] != 0.0) ++r;
  if (l < 0) return r < n ? r : -1;
  if (r >= n) return l;
  return (x - lam[l] <= lam[r] - x) ? l : r;
}

// Per-matrix state of the QR phase, held by lane 0 of wave 0.
struct QrState {
  int q;
  long iters, max_iters;
  bool failed;
  double small;     // off-diagonals at most this (eps times a bound on the norm) count as zero
  bool pipe_prev;   // the previous batch was pipelined
};

// Thread 0: up to S sweeps (deflating from the bottom between them) into batch buffer `cs`
// (S blocks of n pairs) and its header mt = {count, p_0.., q_0..}.  lam holds all eigenvalues
// of the tridiagonal from bisection, ascending; used marks those already deflated.  A sweep
// shifts by the Wilkinson shift of its block's trailing 2 x 2, or by the nearest eigenvalue not
// yet deflated when that lies within twice the trailing off-diagonal of it: an exact shift
// deflates the bottom in about one sweep instead of two.
template <int S>
__device__ void chase_batch(QrState &st, double *d, double *e, int n, const double *lam, double *used, double *cs,
                            int *mt) {
  const double eps = 2.220446049250313e-16;
  int cnt = 0;
  while (cnt < S && st.q > 0 && !st.failed) {
    const int q = st.q;
    if (fabs(e[q - 1]) <= fmax(st.small, eps * (fabs(d[q - 1]) + fabs(d[q])))) {
      e[q - 1] = 0.0;
      const int j = nearest_unused(lam, used, n, d[q]);
      if (j >= 0) used[j] = 1.0;
      --st.q;
      continue;
    }
    int p = q - 1;
    while (p > 0 && !(fabs(e[p - 1]) <= fmax(st.small, eps * (fabs(d[p - 1]) + fabs(d[p]))))) --p;
    if (p > 0) e[p - 1] = 0.0;
    if (++st.iters > st.max_iters) {
      st.failed = true;
      break;
    }
    const double a = d[q - 1], bb = e[q - 1], cq = d[q];
    const double delta = 0.5 * (a - cq);
    const double den = delta + (delta >= 0.0 ? 1.0 : -1.0) * hypot(delta, bb);
    double mu = (den != 0.0) ? cq - bb * bb / den : cq;
    const int j = nearest_unused(lam, used, n, mu);
    if (j >= 0 && fabs(lam[j] - mu) <= 2.0 * fabs(bb)) mu = lam[j];
    qr_sweep(d, e, p, q, mu, cs + static_cast<size_t>(cnt) * 2 * n);
    mt[1 + cnt] = p;
    mt[1 + S + cnt] = q;
    ++cnt;
  }
  mt[0] = cnt;
}

// Lane 0: the decisions of one batch.  Batch header mt = {count, p_0.., q_0.., pipelined}.
// Without pipelining, on a block of fewer than kPipeMin rows, or when the previous pipelined batch
// left nothing to deflate, this is chase_batch (the sweeps run here, one after another).
// Otherwise it deflates at the bottom, finds the unreduced block [p, q] and picks S shifts: the
// first as in chase_batch, the others the eigenvalues not yet deflated nearest to it (exact shifts
// of the block when they belong to it, ordinary shifts otherwise); the sweeps run in
// chase_pipelined.
template <int S>
__device__ void plan_batch(QrState &st, double *d, double *e, int n, const double *lam, double *used, double *cs,
                           int *mt, double *shifts, bool pipe) {
  const double eps = 2.220446049250313e-16;
  mt[1 + 2 * S] = 0;
  if (!pipe) {
    chase_batch<S>(st, d, e, n, lam, used, cs, mt);
    return;
  }
  int deflated = 0;
  while (st.q > 0 && fabs(e[st.q - 1]) <= fmax(st.small, eps * (fabs(d[st.q - 1]) + fabs(d[st.q])))) {
    e[st.q - 1] = 0.0;
    const int j = nearest_unused(lam, used, n, d[st.q]);
    if (j >= 0) used[j] = 1.0;
    --st.q;
    ++deflated;
  }
  if (st.q == 0 || st.failed) {
    mt[0] = 0;
    return;
  }
  const int q = st.q;
  int p = q - 1;
  while (p > 0 && !(fabs(e[p - 1]) <= fmax(st.small, eps * (fabs(d[p - 1]) + fabs(d[p]))))) --p;
  if (q - p + 1 < kPipeMin || (st.pipe_prev && deflated == 0)) {
    st.pipe_prev = false;
    chase_batch<S>(st, d, e, n, lam, used, cs, mt);
    return;
  }
  if (p > 0) e[p - 1] = 0.0;
  if (st.iters + S > st.max_iters) {
    st.failed = true;
    mt[0] = 0;
    return;
  }
  st.iters += S;
  const double a = d[q - 1], bb = e[q - 1], cq = d[q];
  const double delta = 0.5 * (a - cq);
  const double den = delta + (delta >= 0.0 ? 1.0 : -1.0) * hypot(delta, bb);
  double mu = (den != 0.0) ? cq - bb * bb / den : cq;
  int taken[S];
  int cnt = 0;
  const int j0 = nearest_unused(lam, used, n, mu);
  if (j0 >= 0 && fabs(lam[j0] - mu) <= 2.0 * fabs(bb)) {
    mu = lam[j0];
    taken[cnt] = j0;
  } else {
    taken[cnt] = -1;
  }
  shifts[cnt++] = mu;
  // the unused eigenvalues nearest mu, outward from its position in the ascending list
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) / 2;
    if (lam[mid] < mu) lo = mid + 1;
    else hi = mid;
  }
  int l = lo - 1, r = lo;
  auto skip = [&](int i) {
    if (used[i] != 0.0) return true;
    for (int t = 0; t < cnt; ++t)
      if (taken[t] == i) return true;
    return false;
  };
  while (cnt < S) {
    while (l >= 0 && skip(l)) --l;
    while (r < n && skip(r)) ++r;
    int pick;
    if (l < 0 && r >= n) break;
    if (l < 0) pick = r;
    else if (r >= n) pick = l;
    else pick = (mu - lam[l] <= lam[r] - mu) ? l : r;
    taken[cnt] = pick;
    shifts[cnt++] = lam[pick];
  }
  mt[0] = cnt;
  for (int s = 0; s < S; ++s) {
    mt[1 + s] = p;
    mt[1 + S + s] = q;
  }
  mt[1 + 2 * S] = 1;
  st.pipe_prev = true;
}

// All lanes of wave 0: the sweeps of a pipelined batch (header mt, shifts from plan_batch).  Lane
// s chases sweep s with shift s, kPipeLag rotations behind lane s-1, through the same rotations
// as qr_sweep.  Lane s reads d[k+3] and e[k+3] at its rotation k; lane s-1 wrote them at its
// rotations k+3 and k+4, in earlier steps of the loop (kPipeLag >= 5), and lane s+1 reads what
// lane s writes at rotation k (e[k-1], d[k]) two or more steps later.  The LDS operations of one
// wave are carried out in order; the empty asm keeps the compiler from moving loads or stores
// across a step.  The result is that of the S sweeps applied one after another.
template <int S>
__device__ void chase_pipelined(double *d, double *e, int n, double *cs, const int *mt, const double *shifts,
                                int lane) {
  const int cnt = mt[0], p = mt[1], q = mt[1 + S];
  const bool mine = lane < cnt;
  const double mu = mine ? shifts[lane] : 0.0;
  double *myc = cs + static_cast<size_t>(mine ? lane : 0) * 2 * n;
  const int T = (q - p) + kPipeLag * (cnt - 1);
  double dk = 0.0, ek = 0.0, dn = 0.0, en = 0.0, dn2 = 0.0, en2 = 0.0, x = 0.0, z = 0.0;
  for (int t = 0; t < T; ++t) {
    const int k = p + t - kPipeLag * lane;
    if (mine && k >= p && k < q) {
      if (k == p) {
        dk = d[p];
        ek = e[p];
        dn = d[p + 1];
        en = e[p + 1];
        dn2 = d[p + 2];
        en2 = e[p + 2];
        x = dk - mu;
        z = ek;
      }
      const double dn3 = d[k + 3], en3 = e[k + 3];
      double c, sn;
      givens_fast(x, z, c, sn);
      if (k > p) e[k - 1] = c * x - sn * z;
      const double c2 = c * c, s2 = sn * sn, csn = c * sn;
      d[k] = c2 * dk - 2.0 * csn * ek + s2 * dn;
      const double ndk1 = s2 * dk + 2.0 * csn * ek + c2 * dn;
      const double xn = csn * (dk - dn) + (c2 - s2) * ek;
      if (k == q - 1) {
        d[q] = ndk1;
        e[q - 1] = xn;
      }
      myc[2 * (k - p)] = c;
      myc[2 * (k - p) + 1] = sn;
      x = xn;
      z = -sn * en;
      dk = ndk1;
      ek = c * en;
      dn = dn2;
      en = en2;
      dn2 = dn3;
      en2 = en3;
    }
    asm volatile("" ::: "memory");
  }
}

// Wave 0: one batch (lane 0 decides; a pipelined batch is then chased by the whole wave).
template <int S>
__device__ void chase_wave(QrState &st, double *d, double *e, int n, const double *lam, double *used, double *cs,
                           int *mt, double *shifts, int lane, bool pipe) {
  if (lane == 0) plan_batch<S>(st, d, e, n, lam, used, cs, mt, shifts, pipe);
  asm volatile("" ::: "memory");
  if (mt[1 + 2 * S]) chase_pipelined<S>(d, e, n, cs, mt, shifts, lane);
}

// One column of Zr through the batch's sweeps in one pass.  Rotation k of sweep s acts on rows
// k, k+1 and runs at time t = k + 2s: every rotation that shares a row with it and belongs to an
// earlier sweep runs at an earlier time, rotations of one time touch disjoint rows, so the result
// equals applying the sweeps one after another.  At time t the window holds rows t-2(S-1) .. t+1;
// row t+1 enters (loaded kPrefetch rows ahead) and row t-2(S-1) leaves, finished.
template <int S>
__device__ void apply_batch(double *Zr, int n, int col, const double *cs, const int *mt) {
  const int cnt = mt[0];
  int ps[S], qs[S];
  int pmin = n, qmax = -1;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    ps[s] = (s < cnt) ? mt[1 + s] : 0;
    qs[s] = (s < cnt) ? mt[1 + S + s] : 0;  // empty range for absent sweeps
    if (s < cnt) {
      pmin = min(pmin, ps[s]);
      qmax = max(qmax, qs[s]);
    }
  }
  const int t0 = pmin - 1;
  const int T = qmax - pmin + 2 * S;  // times t0 .. qmax + 2(S-1)
  double *zc = Zr + col;
  double win[2 * S];
#pragma unroll
  for (int j = 0; j < 2 * S; ++j) win[j] = 0.0;
  double pf[kPrefetch];
#pragma unroll
  for (int j = 0; j < kPrefetch; ++j) {
    const int r = pmin + j;
    pf[j] = (r <= qmax) ? zc[static_cast<int64_t>(r) * n] : 0.0;
  }
  for (int base = 0; base < T; base += kPrefetch) {
    double nx[kPrefetch];
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j) {
      const int r = pmin + base + kPrefetch + j;
      nx[j] = (r <= qmax) ? zc[static_cast<int64_t>(r) * n] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j) {
      if (base + j < T) {
        const int t = t0 + base + j;
        win[2 * S - 1] = pf[j];
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int k = t - 2 * s;
          if (k >= ps[s] && k < qs[s]) {
            const double c = cs[(static_cast<size_t>(s) * n + (k - ps[s])) * 2];
            const double sn = cs[(static_cast<size_t>(s) * n + (k - ps[s])) * 2 + 1];
            const double x = win[2 * (S - 1 - s)], y = win[2 * (S - 1 - s) + 1];
            win[2 * (S - 1 - s)] = c * x - sn * y;
            win[2 * (S - 1 - s) + 1] = sn * x + c * y;
          }
        }
        const int out = t - 2 * (S - 1);
        if (out >= pmin && out <= qmax) zc[static_cast<int64_t>(out) * n] = win[0];
#pragma unroll
        for (int w = 0; w + 1 < 2 * S; ++w) win[w] = win[w + 1];
      }
    }
#pragma unroll
    for (int j = 0; j < kPrefetch; ++j) pf[j] = nx[j];
  }
}

// LDS: v, w, d, e (n each), the reduction slots, the shift slots, two batch buffers of S x n
// Givens pairs, two batch headers of 2 + 2S ints and the count of finished chases.  pipe = 1
// enables the pipelined batches.
template <int S>
__global__ __launch_bounds__(kBT) void k_batch_syev(const BatchEigProblem *probs, int pipe) {
  extern __shared__ double sm[];
  const BatchEigProblem pb = probs[blockIdx.x];
  const int n = pb.n;
  double *vsh = sm, *wsh = sm + n, *d = sm + 2 * n, *e = sm + 3 * n, *red = sm + 4 * n;
  double *shifts = red + kBWaves;
  double *csb = shifts + kShiftSlots;
  int *meta = reinterpret_cast<int *>(csb + 4 * static_cast<size_t>(S) * n);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double *A = pb.A;
  if (n == 1) {
    if (tid == 0) {
      pb.w[0] = A[0];
      pb.Zr[0] = 1.0;
      *pb.status = 0;
    }
    return;
  }
  // ---- 1. tridiagonalise.  Step k applies step k-1's rank-2 update in the same pass over the
  // trailing block as its own product A22 v (one read and one write of the block per step);
  // row k gets that update first, since it holds the next Householder vector.
  double *vp = csb, *wp = csb + n;  // step k-1's v and w (index i = row k + i), in the Givens buffers
  double *vc = vsh, *wc = wsh;      // step k's (index i = row k + 1 + i)
  bool have_prev = false;
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;
    double *rowk = A + static_cast<int64_t>(k) * n;
    if (have_prev) {
      const double v0p = vp[0], w0p = wp[0];
      for (int j = k + tid; j < n; j += kBT) rowk[j] -= v0p * wp[j - k] + w0p * vp[j - k];
      __syncthreads();
    }
    const double *x = rowk + k + 1;
    const double x0 = x[0];  // read before the reduction's barriers: thread 0 overwrites it below
    double s = 0.0;
    for (int i = 1 + tid; i < m; i += kBT) s += x[i] * x[i];
    const double sigma = block_sum(s, red);
    double alpha = x0, v0 = 0.0, beta = 0.0;
    if (sigma > 0.0) {
      const double mu = sqrt(x0 * x0 + sigma);
      alpha = (x0 >= 0.0) ? -mu : mu;
      v0 = x0 - alpha;
      beta = 2.0 / (v0 * v0 + sigma);
    }
    for (int i = tid; i < m; i += kBT) vc[i] = (i == 0) ? v0 : x[i];
    __syncthreads();
    if (tid == 0) {
      d[k] = rowk[k];
      e[k] = alpha;
      rowk[k] = beta;    // row k keeps beta and v for the back-transformation
      rowk[k + 1] = v0;
    }
    // step k-1's update of A22 and p = beta A22 v as column sums (A22 is symmetric): one thread
    // per column, kRowBatch rows loaded before any is stored
    double *a22 = A + static_cast<int64_t>(k + 1) * n + k + 1;
    for (int j = tid; j < m; j += kBT) {
      double *cj = a22 + j;
      double t = 0.0;
      if (have_prev) {
        const double vj = vp[j + 1], wj = wp[j + 1];
        int i = 0;
        for (; i + kFuseBatch <= m; i += kFuseBatch) {
          double a[kFuseBatch];
#pragma unroll
          for (int u = 0; u < kFuseBatch; ++u) a[u] = cj[static_cast<int64_t>(i + u) * n];
#pragma unroll
          for (int u = 0; u < kFuseBatch; ++u) {
            a[u] -= vp[i + u + 1] * wj + wp[i + u + 1] * vj;
            cj[static_cast<int64_t>(i + u) * n] = a[u];
            t += a[u] * vc[i + u];
          }
        }
        for (; i < m; ++i) {
          const double a = cj[static_cast<int64_t>(i) * n] - (vp[i + 1] * wj + wp[i + 1] * vj);
          cj[static_cast<int64_t>(i) * n] = a;
          t += a * vc[i];
        }
      } else {
        int i = 0;
        for (; i + kRowBatch <= m; i += kRowBatch) {
          double a[kRowBatch];
#pragma unroll
          for (int u = 0; u < kRowBatch; ++u) a[u] = cj[static_cast<int64_t>(i + u) * n];
#pragma unroll
          for (int u = 0; u < kRowBatch; ++u) t += a[u] * vc[i + u];
        }
        for (; i < m; ++i) t += cj[static_cast<int64_t>(i) * n] * vc[i];
      }
      wc[j] = beta * t;
    }
    __syncthreads();
    // w = p - (beta p^T v / 2) v
    double pv = 0.0;
    for (int i = tid; i < m; i += kBT) pv += wc[i] * vc[i];
    const double half = 0.5 * beta * block_sum(pv, red);
    for (int i = tid; i < m; i += kBT) wc[i] -= half * vc[i];
    __syncthreads();
    double *t1 = vp, *t2 = wp;
    vp = vc;
    wp = wc;
    vc = t1;
    wc = t2;
    have_prev = true;
  }
  if (tid == 0) {
    double *a2 = A + static_cast<int64_t>(n - 2) * n + n - 2;  // the trailing 2 x 2
    if (have_prev) {  // the last step's update (its index 0 is row n - 2)
      a2[0] -= vp[0] * wp[0] + wp[0] * vp[0];
      a2[1] -= vp[0] * wp[1] + wp[0] * vp[1];
      a2[n + 1] -= vp[1] * wp[1] + wp[1] * vp[1];
    }
    d[n - 2] = a2[0];
    e[n - 2] = a2[1];
    d[n - 1] = a2[n + 1];
    e[n - 1] = 0.0;
  }
  // Zr = I
  for (int64_t idx = tid; idx < static_cast<int64_t>(n) * n; idx += kBT)
    pb.Zr[idx] = (idx / n == idx % n) ? 1.0 : 0.0;
  __syncthreads();
  // ---- 2. eigenvalues of the tridiagonal by bisection, one per thread (the QR shifts): lam in v,
  // deflation marks in w
  double tnorm = 0.0;  // Gershgorin bound on the norm of the tridiagonal
  {
    double glo = d[0], ghi = d[0], emax = 0.0;
    for (int i = 0; i < n; ++i) {
      const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i + 1 < n ? fabs(e[i]) : 0.0);
      glo = fmin(glo, d[i] - r);
      ghi = fmax(ghi, d[i] + r);
      if (i + 1 < n) emax = fmax(emax, e[i] * e[i]);
    }
    const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax);
    const double pad = 2.220446049250313e-16 * fmax(fabs(glo), fabs(ghi)) + pivmin;
    for (int j = tid; j < n; j += kBT) {
      vsh[j] = bisect_eig(d, e, n, j, glo - pad, ghi + pad, pivmin);
      wsh[j] = 0.0;
    }
    tnorm = fmax(fabs(glo), fabs(ghi));
  }
  __syncthreads();
  // ---- 3. implicit symmetric QR, batch b+1 chased while batch b is applied
  const int hdr = 2 + 2 * S;
  const int a = tid - 64;  // applying thread index (waves 1..)
  // deflation: an off-diagonal below eps (|d_k| + |d_k+1|) or below eps times the norm bound (a
  // backward error of that size; eigenvalues near zero then need no relative accuracy)
  QrState qs{n - 1, 0, 40L * n + 100, false, 2.220446049250313e-16 * tnorm, false};  // lane 0's
  if (wave == 0) {
    chase_wave<S>(qs, d, e, n, vsh, wsh, csb, meta, shifts, lane, pipe != 0);
  }
  __syncthreads();
  for (int it = 0;; ++it) {
    const int cur = it & 1;
    if (meta[cur * hdr] == 0) break;
    if (wave == 0) {
      // the chase is one dependent chain: let its wave issue ahead of the applying waves
      __builtin_amdgcn_s_setprio(3);
      chase_wave<S>(qs, d, e, n, vsh, wsh, csb + static_cast<size_t>(cur ^ 1) * 2 * S * n, meta + (cur ^ 1) * hdr,
                    shifts, lane, pipe != 0);
      __builtin_amdgcn_s_setprio(0);
    } else {
      for (int col = a; col < n; col += kApplyThreads)
        apply_batch<S>(pb.Zr, n, col, csb + static_cast<size_t>(cur) * 2 * S * n, meta + cur * hdr);
    }
    __syncthreads();
  }
  if (tid == 0) *pb.status = qs.failed ? 1 : 0;
  for (int i = tid; i < n; i += kBT) pb.w[i] = d[i];
}

// Work item of the back-transformation launches: matrix `prob`, reflector block or first row `at`.
struct WyItem {
  int prob, at;
};

// Compact-WY factors of the reflectors H_k = I - beta_k v_k v_k^T that k_batch_syev left in the rows
// of A (row k: beta_k at column k, v_k at columns k+1..), one workgroup per block of kWY reflectors
// k0 = item.at ..: writes the block's rows of V (row k = v_k, zero at columns <= k; V = the
// matrix's work, n x n) and T (kb x kb, row-major, ld kb, at work + n^2 + (k0 / kWY) kWY^2) with
// H_k0 ... H_(k0+kb-1) = I - V^T T V in this row layout: T_jj = beta_j and
// T[0:j, j] = -beta_j T[0:j, 0:j] G[0:j, j], G = the Gram matrix of the v's.
__global__ __launch_bounds__(256) void k_wy_prep(const BatchEigProblem *probs, const WyItem *items) {
  __shared__ double G[kWY][kWY + 1];
  __shared__ double Ts[kWY][kWY + 1];
  __shared__ double bet[kWY];
  const WyItem it = items[blockIdx.x];
  const BatchEigProblem pb = probs[it.prob];
  const double *A = pb.A;
  const int n = pb.n;
  double *V = pb.work, *T = pb.work + static_cast<int64_t>(n) * n;
  const int tid = threadIdx.x;
  const int k0 = it.at, nref = n - 2;
  const int kb = min(kWY, nref - k0);
  for (int64_t e = tid; e < static_cast<int64_t>(kb) * n; e += blockDim.x) {
    const int r = static_cast<int>(e / n), c = static_cast<int>(e - static_cast<int64_t>(r) * n);
    const int k = k0 + r;
    V[static_cast<int64_t>(k) * n + c] = (c > k) ? A[static_cast<int64_t>(k) * n + c] : 0.0;
  }
  if (tid < kb) bet[tid] = A[static_cast<int64_t>(k0 + tid) * n + k0 + tid];
  for (int e = tid; e < kb * kb; e += blockDim.x) {
    const int q = e / kb, j = e - q * kb;
    if (q > j) continue;
    const double *vq = A + static_cast<int64_t>(k0 + q) * n, *vj = A + static_cast<int64_t>(k0 + j) * n;
    double acc = 0.0;
    for (int c = k0 + j + 1; c < n; ++c) acc += vq[c] * vj[c];
    G[q][j] = acc;
    G[j][q] = acc;
  }
  __syncthreads();
  for (int j = 0; j < kb; ++j) {
    if (tid < j) {
      double acc = 0.0;
      for (int q = tid; q < j; ++q) acc += Ts[tid][q] * G[q][j];
      Ts[tid][j] = -bet[j] * acc;
    } else if (tid == j) {
      Ts[j][j] = bet[j];
    } else if (tid < kb) {
      Ts[tid][j] = 0.0;
    }
    __syncthreads();
  }
  double *Tb = T + static_cast<int64_t>(k0 / kWY) * kWY * kWY;
  for (int e = tid; e < kb * kb; e += blockDim.x) Tb[e] = Ts[e / kb][e % kb];
}

// Rows item.at .. item.at + kRB - 1 of Zr <- Zr Q^T = Zr P_B^T ... P_0^T, P_j = I - V_j^T T_j V_j
// (k_wy_prep): the last block first, Z <- Z - ((Z V_j^T) T_j^T) V_j on the columns after k0 (V_j is
// zero on the others).  The rows stay in LDS (dynamic: kRB x n doubles) through every block.
__global__ __launch_bounds__(256) void k_wy_apply(const BatchEigProblem *probs, const WyItem *items) {
  extern __shared__ double zs[];
  __shared__ double w1[kRB][kWY], w2[kRB][kWY];
  const WyItem it = items[blockIdx.x];
  const BatchEigProblem pb = probs[it.prob];
  const int n = pb.n, nref = n - 2;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int rows = min(kRB, n - it.at);
  double *Z = pb.Zr + static_cast<int64_t>(it.at) * n;
  const double *V = pb.work, *T = pb.work + static_cast<int64_t>(n) * n;
  for (int e = tid; e < rows * n; e += blockDim.x) zs[e] = Z[e];
  __syncthreads();
  const int nblk = (nref + kWY - 1) / kWY;
  for (int j = nblk - 1; j >= 0; --j) {
    const int k0 = j * kWY, kb = min(kWY, nref - k0), c0 = k0 + 1;
    const double *Vj = V + static_cast<int64_t>(k0) * n;
    const double *Tj = T + static_cast<int64_t>(j) * kWY * kWY;
    // w1 = Z V_j^T: one (row, reflector) pair per wave at a time, lanes along the columns
    for (int pq = wave; pq < rows * kb; pq += 4) {
      const int r = pq / kb, q = pq - r * kb;
      const double *vq = Vj + static_cast<int64_t>(q) * n;
      const double *zr = zs + r * n;
      double acc = 0.0;
      for (int c = c0 + lane; c < n; c += 64) acc += zr[c] * vq[c];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
      if (lane == 0) w1[r][q] = acc;
    }
    __syncthreads();
    // w2 = w1 T_j^T
    for (int e = tid; e < rows * kb; e += blockDim.x) {
      const int r = e / kb, i = e - r * kb;
      double acc = 0.0;
      for (int q = 0; q < kb; ++q) acc += w1[r][q] * Tj[i * kb + q];
      w2[r][i] = acc;
    }
    __syncthreads();
    // Z -= w2 V_j on the columns after k0: one column per thread, every row of the item
    for (int c = c0 + tid; c < n; c += blockDim.x) {
      double acc[kRB];
#pragma unroll
      for (int r = 0; r < kRB; ++r) acc[r] = 0.0;
      for (int i = 0; i < kb; ++i) {
        const double v = Vj[static_cast<int64_t>(i) * n + c];
#pragma unroll
        for (int r = 0; r < kRB; ++r) acc[r] += w2[r][i] * v;
      }
      for (int r = 0; r < rows; ++r) zs[r * n + c] -= acc[r];
    }
    __syncthreads();
  }
  for (int e = tid; e < rows * n; e += blockDim.x) Z[e] = zs[e];
}

}  // namespace

size_t batch_syev_lds_for(int max_n, int S) {
  return (4 * static_cast<size_t>(max_n) + kBWaves + kShiftSlots + 4 * static_cast<size_t>(S) * max_n) *
             sizeof(double) +
         (2 * (2 + 2 * static_cast<size_t>(S)) + 1) * sizeof(int);
}

// Sweeps per batch: the most of 8, 6, 4, 2, 1, at most max_sweeps, whose two Givens buffers fit
// the LDS beside the rest.
int batch_syev_sweeps(int max_n, int max_sweeps) {
  for (int S : {8, 6, 4, 2})
    if (S <= max_sweeps && batch_syev_lds_for(max_n, S) <= kLdsMax) return S;
  return 1;
}

template <int S>
static hipError_t launch_batch_syev_s(const BatchEigProblem *probs, int count, int max_n, int pipe, hipStream_t s) {
  const size_t lds = batch_syev_lds_for(max_n, S);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_batch_syev<S>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_syev<S>, dim3(count), dim3(kBT), lds, s, probs, pipe);
  return hipGetLastError();
}

hipError_t launch_batch_syev(const BatchEigProblem *probs, int count, int max_n, hipStream_t s, int pipe,
                             int max_sweeps) {
  if (count <= 0) return hipSuccess;
  if (max_n < 1 || max_n > kBatchEigMaxN || pipe < 0 || pipe > 1 || max_sweeps < 1) return hipErrorInvalidValue;
  switch (batch_syev_sweeps(max_n, max_sweeps)) {
    case 8: return launch_batch_syev_s<8>(probs, count, max_n, pipe, s);
    case 6: return launch_batch_syev_s<6>(probs, count, max_n, pipe, s);
    case 4: return launch_batch_syev_s<4>(probs, count, max_n, pipe, s);
    case 2: return launch_batch_syev_s<2>(probs, count, max_n, pipe, s);
    default: return launch_batch_syev_s<1>(probs, count, max_n, pipe, s);
  }
}

namespace {

__global__ void k_fill_int(int *p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Device buffers of one batched solve besides A and Zr: per-matrix w (n doubles each),
// convergence flags and the problem table.
struct BatchEigWork {
  WyItem *items = nullptr;         // batch_syev_items(count, n) entries
  double *wb = nullptr;            // sum n[i] doubles
  int *stat = nullptr;             // count ints
  BatchEigProblem *probs = nullptr;  // count entries
};

// First half on given buffers (no allocation): one launch over the matrices; w[i] (host) gets the
// eigenvalues in the unsorted order of the rows of Zr[i].
dacp_status batch_syev_raw_on(dacp_ctx ctx, int count, const int *n, double *const *A, double *const *Zr,
                              double *const *work, double *const *w, const BatchEigWork &wk) {
  hipStream_t st = ctx->stream;
  int max_n = 0;
  size_t total = 0;
  std::vector<size_t> off(count);
  for (int i = 0; i < count; ++i) {
    max_n = std::max(max_n, n[i]);
    off[i] = total;
    total += static_cast<size_t>(n[i]);
  }
  // flags cleared by a kernel (a memset node would misbehave inside a caller's captured graph)
  hipLaunchKernelGGL(k_fill_int, dim3((count + 255) / 256), dim3(256), 0, st, wk.stat, count, 0);
  DACP_HIP(ctx, hipGetLastError());
  std::vector<BatchEigProblem> probs(count);
  for (int i = 0; i < count; ++i) {
    double *base = wk.wb + off[i];
    probs[i].A = A[i];
    probs[i].Zr = Zr[i];
    probs[i].work = work ? work[i] : nullptr;
    probs[i].w = base;
    probs[i].status = wk.stat + i;
    probs[i].n = n[i];
  }
  DACP_TRY(to_device(ctx, wk.probs, probs.data(), sizeof(BatchEigProblem) * count));
  DACP_HIP(ctx, launch_batch_syev(wk.probs, count, max_n, st, ctx->beig_pipe, ctx->beig_sweeps));
  if (work) {
    // eigenvectors of A: Zr <- Zr Q^T for every matrix, two launches
    std::vector<WyItem> prep, apply;
    for (int i = 0; i < count; ++i) {
      for (int k0 = 0; k0 < n[i] - 2; k0 += kWY) prep.push_back({i, k0});
      if (n[i] > 2)
        for (int r0 = 0; r0 < n[i]; r0 += kRB) apply.push_back({i, r0});
    }
    if (!prep.empty()) {
      std::vector<WyItem> all(prep);
      all.insert(all.end(), apply.begin(), apply.end());
      DACP_TRY(to_device(ctx, wk.items, all.data(), sizeof(WyItem) * all.size()));
      hipLaunchKernelGGL(k_wy_prep, dim3(static_cast<unsigned>(prep.size())), dim3(256), 0, st, wk.probs, wk.items);
      DACP_HIP(ctx, hipGetLastError());
      const size_t lds = static_cast<size_t>(kRB) * max_n * sizeof(double);
      DACP_HIP(ctx, hipFuncSetAttribute(reinterpret_cast<const void *>(k_wy_apply),
                                        hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
      hipLaunchKernelGGL(k_wy_apply, dim3(static_cast<unsigned>(apply.size())), dim3(256), lds, st, wk.probs,
                         wk.items + prep.size());
      DACP_HIP(ctx, hipGetLastError());
    }
  }
  std::vector<int> status(count);
  DACP_TRY(to_host(ctx, status.data(), wk.stat, sizeof(int) * count));
  for (int i = 0; i < count; ++i)
    if (status[i] != 0) return set_err(ctx, DACP_E_CONVERGENCE, "batch_syev: QR iteration did not converge");
  std::vector<double> all(total);
  DACP_TRY(to_host(ctx, all.data(), wk.wb, total * sizeof(double)));
  for (int i = 0; i < count; ++i) std::copy(all.begin() + off[i], all.begin() + off[i] + n[i], w[i]);
  return DACP_OK;
}

// Second half for one matrix on a given permutation buffer dperm (n ints, no allocation): the
// eigenvalues in ascending order, and the rows of Zr (already Zr Q^T) in that order.
dacp_status batch_syev_finish_on(dacp_ctx ctx, int n, const double *w_raw, const double *Zr, double *w_out,
                                 double *Zrows, int *dperm) {
  hipStream_t st = ctx->stream;
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return w_raw[a] < w_raw[b]; });
  for (int j = 0; j < n; ++j) w_out[j] = w_raw[perm[j]];
  if (!Zrows) return DACP_OK;
  DACP_TRY(to_device(ctx, dperm, perm.data(), sizeof(int) * n));
  DACP_HIP(ctx, launch_gather_rows(Zr, n, Zrows, n, dperm, nullptr, n, n, st));
  DACP_HIP(ctx, hipStreamSynchronize(st));  // dperm may be reused on return
  return DACP_OK;
}

}  // namespace

size_t batch_syev_work_doubles(int n) {
  const size_t nblk = n > 2 ? (static_cast<size_t>(n) - 2 + kWY - 1) / kWY : 0;
  return static_cast<size_t>(n) * n + nblk * kWY * kWY;
}

size_t batch_syev_items(int count, const int *n) {
  size_t k = 0;
  for (int i = 0; i < count; ++i)
    if (n[i] > 2) k += (static_cast<size_t>(n[i]) - 2 + kWY - 1) / kWY + (static_cast<size_t>(n[i]) + kRB - 1) / kRB;
  return std::max<size_t>(k, 1);
}

// Host side, first half: launches over `count` matrices A[i] (device, n[i] x n[i], ld n[i],
// destroyed); w[i] (host) receives the eigenvalues, unsorted; Zr[i] (device, n x n) the eigenvectors
// of A[i] as rows in the same order when work[i] (device, batch_syev_work_doubles(n[i]) doubles) is
// given (work null: Zr holds the tridiagonal's eigenvectors only).
dacp_status batch_syev_raw(dacp_ctx ctx, int count, const int *n, double *const *A, double *const *Zr,
                           double *const *work, double *const *w) {
  if (count <= 0) return DACP_OK;
  size_t total = 0;
  for (int i = 0; i < count; ++i) {
    if (n[i] < 1 || n[i] > kBatchEigMaxN) return set_err(ctx, DACP_E_INVALID, "batch_syev: 1 <= n <= 2048");
    total += static_cast<size_t>(n[i]);
  }
  DevBuf wbuf, dprobs, dstat, ditems;
  DACP_HIP(ctx, wbuf.alloc(total * sizeof(double)));
  DACP_HIP(ctx, dstat.alloc(sizeof(int) * count));
  DACP_HIP(ctx, dprobs.alloc(sizeof(BatchEigProblem) * count));
  DACP_HIP(ctx, ditems.alloc(sizeof(WyItem) * batch_syev_items(count, n)));
  BatchEigWork wk;
  wk.wb = wbuf.as<double>();
  wk.stat = dstat.as<int>();
  wk.probs = dprobs.as<BatchEigProblem>();
  wk.items = ditems.as<WyItem>();
  return batch_syev_raw_on(ctx, count, n, A, Zr, work, w, wk);
}

// Second half, for one matrix on the caller's stream: eigenvalues ascending into w_out and, if
// Zrows is set, the rows of Zr (eigenvectors of A from batch_syev_raw with work) in that order.
dacp_status batch_syev_finish(dacp_ctx ctx, int n, const double *w_raw, const double *Zr, double *w_out,
                              double *Zrows) {
  DevBuf dperm;
  if (Zrows) DACP_HIP(ctx, dperm.alloc(sizeof(int) * n));
  return batch_syev_finish_on(ctx, n, w_raw, Zr, w_out, Zrows, dperm.as<int>());
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
    total += static_cast<size_t>(n[i]) * n[i];
  }
  bool vectors = false;
  size_t wtotal = 0;
  std::vector<size_t> woff(count);
  for (int i = 0; i < count; ++i) {
    vectors = vectors || Zrows[i] != nullptr;
    woff[i] = wtotal;
    wtotal += batch_syev_work_doubles(n[i]);
  }
  DevBuf scratch_z, scratch_w;
  DACP_HIP(ctx, scratch_z.alloc(total * sizeof(double)));
  if (vectors) DACP_HIP(ctx, scratch_w.alloc(wtotal * sizeof(double)));
  std::vector<double *> zr(count), wk(count), wr(count);
  std::vector<std::vector<double>> wraw(count);
  for (int i = 0; i < count; ++i) {
    zr[i] = scratch_z.as<double>() + off[i];
    wk[i] = vectors ? scratch_w.as<double>() + woff[i] : nullptr;
    wraw[i].resize(n[i]);
    wr[i] = wraw[i].data();
  }
  DACP_TRY(batch_syev_raw(ctx, count, n, A, zr.data(), vectors ? wk.data() : nullptr, wr.data()));
  for (int i = 0; i < count; ++i) DACP_TRY(batch_syev_finish(ctx, n[i], wr[i], zr[i], w[i], Zrows[i]));
  return DACP_OK;
}

// ------------------------------------------------------------------ allocation-free form
//
// The workspace of dacp_syev_batched_noalloc: one array per device, of a fixed size, held from the
// module's load until the process ends.  In host code `scratch` names a host-side stand-in, not the
// device array: host code uses only the address that hipGetSymbolAddress returns for the device
// that is current (kept per device below).  Every call on one device shares the array.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};
bool g_scratch_done[64] = {};
hipError_t g_scratch_err[64] = {};

size_t round256(size_t x) { return (x + 255) / 256 * 256; }
}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_done[device]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));  // the current device's copy
    g_scratch_err[device] = e;
    g_scratch_ptr[device] = (e == hipSuccess) ? ptr : nullptr;
    g_scratch_done[device] = true;
  }
  return g_scratch_err[device];
}

size_t batch_syev_noalloc_bytes(int count, const int *n) {
  size_t wb = 0, z = 0;
  int max_n = 0;
  for (int i = 0; i < count; ++i) {
    wb += static_cast<size_t>(n[i]);
    z += static_cast<size_t>(n[i]) * n[i];
    max_n = std::max(max_n, n[i]);
  }
  size_t wk = 0;
  for (int i = 0; i < count; ++i) wk += batch_syev_work_doubles(n[i]);
  return round256(sizeof(int) * count) + round256(sizeof(BatchEigProblem) * count) + round256(wb * sizeof(double)) +
         round256(z * sizeof(double)) + round256(wk * sizeof(double)) +
         round256(sizeof(WyItem) * batch_syev_items(count, n)) + round256(sizeof(int) * max_n);
}

dacp_status batch_syev_noalloc(dacp_ctx ctx, int count, const int *n, double *const *A, double *const *w,
                               double *const *Zrows) {
  if (count <= 0) return DACP_OK;
  for (int i = 0; i < count; ++i)
    if (n[i] < 1 || n[i] > kBatchEigMaxN) return set_err(ctx, DACP_E_INVALID, "batch_syev: 1 <= n <= 2048");
  const size_t need = batch_syev_noalloc_bytes(count, n);
  if (need > kNoAllocScratchBytes)
    return set_err(ctx, DACP_E_INVALID,
                   "syev_batched_noalloc: the matrices need " + std::to_string(need) +
                       " bytes of workspace; the fixed workspace holds " + std::to_string(kNoAllocScratchBytes));
  const hipError_t e = noalloc_scratch_init(ctx->device);
  if (e != hipSuccess) return hip_err(ctx, e, "syev_batched_noalloc: hipGetSymbolAddress(scratch)");
  unsigned char *base = static_cast<unsigned char *>(g_scratch_ptr[ctx->device]);
  size_t wb = 0, z = 0;
  int max_n = 0;
  for (int i = 0; i < count; ++i) {
    wb += static_cast<size_t>(n[i]);
    z += static_cast<size_t>(n[i]) * n[i];
    max_n = std::max(max_n, n[i]);
  }
  BatchEigWork wk;
  size_t at = 0;
  wk.stat = reinterpret_cast<int *>(base + at);
  at += round256(sizeof(int) * count);
  wk.probs = reinterpret_cast<BatchEigProblem *>(base + at);
  at += round256(sizeof(BatchEigProblem) * count);
  wk.wb = reinterpret_cast<double *>(base + at);
  at += round256(wb * sizeof(double));
  double *zb = reinterpret_cast<double *>(base + at);
  at += round256(z * sizeof(double));
  double *workb = reinterpret_cast<double *>(base + at);
  size_t wk_total = 0;
  for (int i = 0; i < count; ++i) wk_total += batch_syev_work_doubles(n[i]);
  at += round256(wk_total * sizeof(double));
  wk.items = reinterpret_cast<WyItem *>(base + at);
  at += round256(sizeof(WyItem) * batch_syev_items(count, n));
  int *dperm = reinterpret_cast<int *>(base + at);
  std::vector<double *> zr(count), work(count), wr(count);
  std::vector<std::vector<double>> wraw(count);
  size_t off = 0, woff = 0;
  for (int i = 0; i < count; ++i) {
    zr[i] = zb + off;
    off += static_cast<size_t>(n[i]) * n[i];
    work[i] = workb + woff;
    woff += batch_syev_work_doubles(n[i]);
    wraw[i].resize(n[i]);
    wr[i] = wraw[i].data();
  }
  DACP_TRY(batch_syev_raw_on(ctx, count, n, A, zr.data(), work.data(), wr.data(), wk));
  for (int i = 0; i < count; ++i) DACP_TRY(batch_syev_finish_on(ctx, n[i], wr[i], zr[i], w[i], Zrows[i], dperm));
  return DACP_OK;
}

}  // namespace dacp
