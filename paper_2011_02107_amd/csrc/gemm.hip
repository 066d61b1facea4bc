// FP64 GEMM on the gfx950 matrix cores (v_mfma_f64_16x16x4_f64).
//
// C = alpha * op(A) * op(B) + beta * C, row-major.  A 256-thread workgroup
// computes a 128 x 128 tile of C; each of its four 64-lane waves owns a
// 64 x 64 quadrant held as 4 x 4 MFMA accumulators of 16 x 16.  K advances in
// slabs of 16 staged through double-buffered LDS (k-major, padded rows).
// Used for the Gram S = V^T V and P = V^T (H V) (upper triangle only), the
// subspace transforms of the generalised eigenproblem and the Ritz vectors.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace dacp {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int BM = 128, BN = 128, BK = 16, PADD = 4;

// Split K: workgroup z of the grid's third dimension sums k in [z kchunk, (z + 1) kchunk) and,
// when `work` is set, stores alpha * (its partial tile) to work[z][M][N] for k_splitk_reduce.
template <int TA, int TB>
__global__ __launch_bounds__(256, 2) void k_dgemm(int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                                                  int64_t lda, const double *B, int64_t ldb, double beta, double *C,
                                                  int64_t ldc, int upper, int ntn, int64_t kchunk, double *work) {
  __shared__ double As[2][BK][BM + PADD];
  __shared__ double Bs[2][BK][BN + PADD];
  // XCD-aware tile order: workgroups are dealt to the 8 XCDs round-robin, so workgroup
  // b = 8 q + x runs on XCD x.  Each XCD takes whole 8 x 8 blocks of output tiles (super-block
  // s = 8 (q / 64) + x, tile q % 64 inside it): the tiles resident on one XCD at a time share 8 row
  // panels of op(A) and 8 column panels of op(B) in its L2.  Upper mode enumerates the super-blocks
  // with block row <= block column and idles the tiles below the diagonal.
  const int tmc = static_cast<int>((M + BM - 1) / BM);
  const int sbm = (tmc + 7) / 8, sbn = (ntn + 7) / 8;
  const int bid = blockIdx.x;
  const int slot = bid >> 3, x = bid & 7;
  int sb = (slot >> 6) * 8 + x;
  const int t64 = slot & 63;
  int si, sj;
  if (upper) {
    si = 0;
    while (si < sbm && sb >= sbn - si) {
      sb -= sbn - si;
      ++si;
    }
    if (si >= sbm) return;
    sj = si + sb;
  } else {
    if (sb >= sbm * sbn) return;
    si = sb / sbn;
    sj = sb - si * sbn;
  }
  const int tm = si * 8 + (t64 >> 3), tn = sj * 8 + (t64 & 7);
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
  double ra[8], rb[8];
  auto load_a = [&](int64_t k0) {
    if (TA) {  // A stored K x M
      const int kk = tid >> 4, mm = (tid & 15) * 8;
      const int64_t k = kbeg + k0 + kk;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t m = m0 + mm + q;
        ra[q] = (k < kend && m < M) ? A[k * lda + m] : 0.0;
      }
    } else {  // A stored M x K
      const int mm = tid >> 1, kk = (tid & 1) * 8;
      const int64_t m = m0 + mm;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t k = kbeg + k0 + kk + q;
        ra[q] = (k < kend && m < M) ? A[m * lda + k] : 0.0;
      }
    }
  };
  auto load_b = [&](int64_t k0) {
    if (!TB) {  // B stored K x N
      const int kk = tid >> 4, nn = (tid & 15) * 8;
      const int64_t k = kbeg + k0 + kk;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t n = n0 + nn + q;
        rb[q] = (k < kend && n < N) ? B[k * ldb + n] : 0.0;
      }
    } else {  // B stored N x K
      const int nn = tid >> 1, kk = (tid & 1) * 8;
      const int64_t n = n0 + nn;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int64_t k = kbeg + k0 + kk + q;
        rb[q] = (k < kend && n < N) ? B[n * ldb + k] : 0.0;
      }
    }
  };
  auto store_ab = [&](int buf) {
    if (TA) {
      const int kk = tid >> 4, mm = (tid & 15) * 8;
#pragma unroll
      for (int q = 0; q < 8; ++q) As[buf][kk][mm + q] = ra[q];
    } else {
      const int mm = tid >> 1, kk = (tid & 1) * 8;
#pragma unroll
      for (int q = 0; q < 8; ++q) As[buf][kk + q][mm] = ra[q];
    }
    if (!TB) {
      const int kk = tid >> 4, nn = (tid & 15) * 8;
#pragma unroll
      for (int q = 0; q < 8; ++q) Bs[buf][kk][nn + q] = rb[q];
    } else {
      const int nn = tid >> 1, kk = (tid & 1) * 8;
#pragma unroll
      for (int q = 0; q < 8; ++q) Bs[buf][kk + q][nn] = rb[q];
    }
  };

  v4d acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  const int64_t nk = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;
  load_a(0);
  load_b(0);
  store_ab(0);
  __syncthreads();
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = static_cast<int>(kt & 1);
    if (kt + 1 < nk) {
      load_a((kt + 1) * BK);
      load_b((kt + 1) * BK);
    }
#pragma unroll
    for (int k4 = 0; k4 < BK / 4; ++k4) {
      const int kr = k4 * 4 + (lane >> 4);
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = As[buf][kr][wm + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = Bs[buf][kr][wn + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) store_ab(buf ^ 1);
    __syncthreads();
  }
  // Output layout of the f64 16x16 accumulator (measured on gfx950): lane l,
  // item r -> row (l / 16) + 4 r, column l % 16.
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t row = m0 + wm + i * 16 + (lane >> 4) + 4 * r;
        const int64_t col = n0 + wn + j * 16 + (lane & 15);
        if (row < M && col < N) {
          double v = alpha * acc[i][j][r];
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
  if (splits < 1 || (splits > 1 && (!work || upper))) return hipErrorInvalidValue;
  if (upper && M != N) return hipErrorInvalidValue;
  const int64_t kchunk = splits == 1 ? K : ((K + splits - 1) / splits + BK - 1) / BK * BK;
  // super-blocks of 8 x 8 tiles, dealt 8 at a time (one per XCD), 64 workgroups each
  const int64_t sbm = (tmc + 7) / 8, sbn = (tnc + 7) / 8;
  const int64_t nsb = upper ? sbn * (sbn + 1) / 2 : sbm * sbn;
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

hipError_t launch_dgemm_splitk(int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                               int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                               int splits, double *work, hipStream_t s) {
  return launch_dgemm_impl(transA, transB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, 0, splits, work, s);
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
