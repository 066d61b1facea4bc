// FP64 GEMM on the gfx950 matrix cores (v_mfma_f64_16x16x4_f64).
//
// C = alpha * op(A) * op(B) + beta * C, row-major.  A 256-thread workgroup
// computes a 128 x 128 tile of C; each of its four 64-lane waves owns a
// 64 x 64 quadrant held as 4 x 4 MFMA accumulators of 16 x 16.  K advances in
// slabs of 16 staged through double-buffered LDS.
// Used for the Gram S = V^T V and P = V^T (H V) (upper triangle only), the
// subspace transforms of the generalised eigenproblem and the Ritz vectors.
//
// LDS layout.  The 16 x 16 x 4 MFMA takes from lane l the A element (row l % 16, k = l / 16) and
// the B element (k = l / 16, column l % 16), so over the four k-steps of a slab lane l needs
// k = l / 16 + 4 s, s = 0..3, of one row.  Each operand tile is stored row-major by m (or n) with
// the slab's k permuted as kp(k) = 4 (k % 4) + k / 4: those four values are contiguous, and a
// lane fetches them with two 16-byte LDS reads.  Rows are 18 doubles (144 bytes) apart, so the 16
// lanes of a read group hit distinct 16-byte bank groups.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace dacp {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

constexpr int BM = 128, BN = 128, BK = 16, KS = 18;

// Global -> registers -> LDS staging of one 128 x 16 operand slab.  KMAJOR: element (k, x) at
// src[k * ld + x] (x = m or n contiguous); each thread takes one x and 8 consecutive k and stores
// pairs (k, k + 4), which are adjacent after the permutation, as 16-byte LDS writes.  Otherwise
// element (k, x) at src[x * ld + k]; each thread takes one k and 8 rows x.
template <bool KMAJOR>
struct Slab {
  double v[8];
  // Row q of the thread's 8 starts at a wave-uniform pointer (KMAJOR: k is uniform per wave) or at
  // a uniform pointer plus one per-lane offset computed once, so the loads need no per-element
  // 64-bit address registers.
  __device__ __forceinline__ void load(const double *src, int64_t ld, int64_t x0, int64_t X, int64_t kb, int64_t kend,
                                       int tid) {
    if (KMAJOR) {
      const int x = tid & 127, kk = (tid >> 7) * 8;
      const bool xin = x0 + x < X;
      const double *base = src + (kb + kk) * ld + x0;
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = (kb + kk + q < kend && xin) ? base[q * ld + x] : 0.0;
    } else {
      const int k = tid & 15, xr = tid >> 4;
      const bool kin = kb + k < kend;
      const int64_t off = static_cast<int64_t>(xr) * ld + k;
      const double *base = src + x0 * ld + kb;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        v[q] = (kin && x0 + xr + 16 * q < X) ? base[static_cast<int64_t>(16 * q) * ld + off] : 0.0;
    }
  }
  __device__ __forceinline__ void store(double (*S)[KS], int tid) const {
    if (KMAJOR) {
      const int x = tid & 127, h = tid >> 7;
#pragma unroll
      for (int c = 0; c < 4; ++c) *reinterpret_cast<v2d *>(&S[x][4 * c + 2 * h]) = v2d{v[c], v[c + 4]};
    } else {
      const int k = tid & 15, kp = 4 * (k & 3) + (k >> 2);
#pragma unroll
      for (int q = 0; q < 8; ++q) S[(tid >> 4) + 16 * q][kp] = v[q];
    }
  }
};

// Split K: workgroup z of the grid's third dimension sums k in [z kchunk, (z + 1) kchunk) and,
// when `work` is set, stores alpha * (its partial tile) to work[z][M][N] for k_splitk_reduce.
template <int TA, int TB>
__global__ __launch_bounds__(256, 2) void k_dgemm(int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                                                  int64_t lda, const double *B, int64_t ldb, double beta, double *C,
                                                  int64_t ldc, int upper, int ntn, int64_t kchunk, double *work) {
  __shared__ __attribute__((aligned(16))) double As[2][BM][KS];
  __shared__ __attribute__((aligned(16))) double Bs[2][BN][KS];
  // XCD-aware tile order: workgroups are dealt to the 8 XCDs round-robin, so workgroup
  // b = 8 q + x runs on XCD x.  Each XCD takes rounds of 64 output tiles (round
  // s = 8 (q / 64) + x, tile q % 64 inside it), one round resident at a time: mostly whole 8 x 8
  // blocks of tiles, which share 8 row panels of op(A) and 8 column panels of op(B) in its L2.
  // Upper mode takes the blocks strictly above the diagonal first, then the upper triangles of the
  // diagonal blocks (36 tiles each) packed 64 tiles to a round, so no round idles 28 of its
  // workgroups on the tiles below the diagonal.
  const int tmc = static_cast<int>((M + BM - 1) / BM);
  const int sbm = (tmc + 7) / 8, sbn = (ntn + 7) / 8;
  const int bid = blockIdx.x;
  const int slot = bid >> 3, x = bid & 7;
  int sb = (slot >> 6) * 8 + x;
  const int t64 = slot & 63;
  int tm, tn;
  if (upper) {
    const int nfull = sbn * (sbn - 1) / 2;
    if (sb < nfull) {
      int si = 0;
      while (sb >= sbn - 1 - si) {
        sb -= sbn - 1 - si;
        ++si;
      }
      const int sj = si + 1 + sb;
      tm = si * 8 + (t64 >> 3);
      tn = sj * 8 + (t64 & 7);
    } else {
      const int d = (sb - nfull) * 64 + t64;  // tile d of the diagonal blocks' upper triangles
      if (d >= 36 * sbn) return;
      const int blk = d / 36;
      int w = d - blk * 36, r = 0;
      while (w >= 8 - r) {
        w -= 8 - r;
        ++r;
      }
      tm = blk * 8 + r;
      tn = blk * 8 + r + w;
    }
  } else {
    if (sb >= sbm * sbn) return;
    const int si = sb / sbn, sj = sb - si * sbn;
    tm = si * 8 + (t64 >> 3);
    tn = sj * 8 + (t64 & 7);
  }
  if (tm >= tmc || tn >= ntn || (upper && tm > tn)) return;
  const int64_t m0 = static_cast<int64_t>(tm) * BM;
  const int64_t n0 = static_cast<int64_t>(tn) * BN;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64;
  const int wn = (wave & 1) * 64;

  const int64_t kbeg = static_cast<int64_t>(blockIdx.z) * kchunk;
  const int64_t kend = (kbeg + kchunk < K) ? kbeg + kchunk : K;
  Slab<TA == 1> sa;  // A stored K x M when transposed
  Slab<TB == 0> sbt;  // B stored K x N when not transposed

  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  const int64_t nk = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;
  sa.load(A, lda, m0, M, kbeg, kend, tid);
  sbt.load(B, ldb, n0, N, kbeg, kend, tid);
  sa.store(As[0], tid);
  sbt.store(Bs[0], tid);
  __syncthreads();
  const int r = lane & 15, q4 = (lane >> 4) * 4;
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = static_cast<int>(kt & 1);
    if (kt + 1 < nk) {
      sa.load(A, lda, m0, M, kbeg + (kt + 1) * BK, kend, tid);
      sbt.load(B, ldb, n0, N, kbeg + (kt + 1) * BK, kend, tid);
    }
    // two k-steps per 16-byte read: halves 0 (k-steps 0, 1) and 1 (k-steps 2, 3) of the slab
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
      v2d av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        av[i] = *reinterpret_cast<const v2d *>(&As[buf][wm + i * 16 + r][q4 + 2 * hf]);
        bv[i] = *reinterpret_cast<const v2d *>(&Bs[buf][wn + i * 16 + r][q4 + 2 * hf]);
      }
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][s2], bv[j][s2], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) {
      sa.store(As[buf ^ 1], tid);
      sbt.store(Bs[buf ^ 1], tid);
    }
    __syncthreads();
  }
  // Output layout of the f64 16x16 accumulator (measured on gfx950): lane l,
  // item r -> row (l / 16) + 4 r, column l % 16.
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t row = m0 + wm + i * 16 + (lane >> 4) + 4 * e;
        const int64_t col = n0 + wn + j * 16 + (lane & 15);
        if (row < M && col < N) {
          double v = alpha * acc[i][j][e];
          if (work) {
            work[static_cast<int64_t>(blockIdx.z) * M * N + row * N + col] = v;
          } else {
            if (beta != 0.0) v += beta * C[row * ldc + col];
            C[row * ldc + col] = v;
          }
        }
      }
}

// C = sum_z work[z] + beta C (fixed order over z)
__global__ void k_splitk_reduce(const double *work, int splits, int64_t M, int64_t N, double beta, double *C,
                                int64_t ldc) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= M * N) return;
  const int64_t row = e / N, col = e - row * N;
  double v = 0.0;
  for (int z = 0; z < splits; ++z) v += work[static_cast<int64_t>(z) * M * N + e];
  if (beta != 0.0) v += beta * C[row * ldc + col];
  C[row * ldc + col] = v;
}

hipError_t launch_dgemm_impl(int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                             int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                             int upper, int splits, double *work, hipStream_t s) {
  if (M <= 0 || N <= 0) return hipSuccess;
  const int64_t tmc = (M + BM - 1) / BM, tnc = (N + BN - 1) / BN;
  if (splits < 1 || (splits > 1 && !work)) return hipErrorInvalidValue;
  if (upper && M != N) return hipErrorInvalidValue;
  const int64_t kchunk = splits == 1 ? K : ((K + splits - 1) / splits + BK - 1) / BK * BK;
  // rounds of 64 tiles (8 x 8 blocks, or packed diagonal-block triangles in upper mode), dealt 8 at
  // a time (one per XCD), 64 workgroups each
  const int64_t sbm = (tmc + 7) / 8, sbn = (tnc + 7) / 8;
  const int64_t nsb = upper ? sbn * (sbn - 1) / 2 + (36 * sbn + 63) / 64 : sbm * sbn;
  const int64_t nblocks = 8 * 64 * ((nsb + 7) / 8);
  if (nblocks > 0x7fffffff) return hipErrorInvalidValue;
  dim3 grid(static_cast<unsigned>(nblocks), 1, static_cast<unsigned>(splits)), block(256);
  const int ntn = static_cast<int>(tnc);
  double *wk = splits > 1 ? work : nullptr;
#define DACP_GEMM_LAUNCH(a_, b_)                                                                                    \
  hipLaunchKernelGGL((k_dgemm<a_, b_>), grid, block, 0, s, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, upper, ntn, \
                     kchunk, wk)
  if (!transA && !transB) DACP_GEMM_LAUNCH(0, 0);
  else if (!transA && transB) DACP_GEMM_LAUNCH(0, 1);
  else if (transA && !transB) DACP_GEMM_LAUNCH(1, 0);
  else DACP_GEMM_LAUNCH(1, 1);
#undef DACP_GEMM_LAUNCH
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || splits == 1) return e;
  hipLaunchKernelGGL(k_splitk_reduce, dim3(static_cast<unsigned>((M * N + 255) / 256)), dim3(256), 0, s, work, splits,
                     M, N, beta, C, ldc);
  return hipGetLastError();
}

hipError_t launch_dgemm(int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                        int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc, int upper,
                        hipStream_t s) {
  return launch_dgemm_impl(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, upper, 1, nullptr, s);
}

// With upper set (M == N), only tiles on or above the diagonal are computed and the reduction
// leaves the tiles below it undefined: the caller mirrors the upper triangle afterwards.
hipError_t launch_dgemm_splitk(int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                               int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                               int upper, int splits, double *work, hipStream_t s) {
  return launch_dgemm_impl(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, upper, splits, work, s);
}

// Copy the upper triangle onto the lower one (tiled through LDS).
__global__ void k_mirror_upper(double *C, int64_t n, int64_t ldc) {
  __shared__ double t[32][33];
  const int64_t bi = blockIdx.y, bj = blockIdx.x;
  if (bi > bj) return;  // source tile (bi, bj) in the upper part
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bi * 32 + r, j = bj * 32 + tx;
    t[r][tx] = (i < n && j < n) ? C[i * ldc + j] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bj * 32 + r, j = bi * 32 + tx;  // destination (row i, col j) = source (j, i)
    if (i < n && j < n && i > j) C[i * ldc + j] = t[tx][r];
  }
}

hipError_t launch_mirror_upper(double *C, int64_t n, int64_t ldc, hipStream_t s) {
  const unsigned nt = static_cast<unsigned>((n + 31) / 32);
  hipLaunchKernelGGL(k_mirror_upper, dim3(nt, nt), dim3(32, 8), 0, s, C, n, ldc);
  return hipGetLastError();
}

// C <- (C + C^T) / 2, tile pairs handled by the upper tile's workgroup.
__global__ void k_symmetrize(double *C, int64_t n, int64_t ldc) {
  __shared__ double tu[32][33], tl[32][33];
  const int64_t bi = blockIdx.y, bj = blockIdx.x;
  if (bi > bj) return;
  const int tx = threadIdx.x, ty = threadIdx.y;
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bi * 32 + r, j = bj * 32 + tx;
    tu[r][tx] = (i < n && j < n) ? C[i * ldc + j] : 0.0;
    const int64_t i2 = bj * 32 + r, j2 = bi * 32 + tx;
    tl[r][tx] = (i2 < n && j2 < n) ? C[i2 * ldc + j2] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int64_t i = bi * 32 + r, j = bj * 32 + tx;
    const double v = 0.5 * (tu[r][tx] + tl[tx][r]);
    if (i < n && j < n) C[i * ldc + j] = v;
    const int64_t i2 = bj * 32 + r, j2 = bi * 32 + tx;
    const double v2 = 0.5 * (tl[r][tx] + tu[tx][r]);
    if (i2 < n && j2 < n && bi != bj) C[i2 * ldc + j2] = v2;
  }
}

hipError_t launch_symmetrize(double *C, int64_t n, int64_t ldc, hipStream_t s) {
  const unsigned nt = static_cast<unsigned>((n + 31) / 32);
  hipLaunchKernelGGL(k_symmetrize, dim3(nt, nt), dim3(32, 8), 0, s, C, n, ldc);
  return hipGetLastError();
}

}  // namespace dacp
