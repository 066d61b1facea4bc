// Internal declarations of the DACP HIP library (gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/dacp.h"

namespace dacp {

// One off-diagonal group of the Hamiltonian: y[s] += coef * (-1)^popcount((s ^ x) & z) * x[s ^ x].
struct FlipEntry {
  uint32_t xmask;
  uint32_t zmask;
  double coef;
};

constexpr int kMaxFlips = 1024;
constexpr int kApplyThreads = 256;
constexpr int kTileElemsDefault = 1024;  // default elements of one LDS tile of the apply kernel

// Arguments of the fused "apply + three-term combine" kernel:
//   y = alpha * H x + beta * u + gamma * z      (u, z optional; z may alias y)
//   if st != nullptr: st[s * ldst + j] = y  (FP64 copy, the basis sample store)
template <typename T>
struct StepArgs {
  const T *x;
  int64_t ldx;
  T *y;
  int64_t ldy;
  const T *u;
  int64_t ldu;
  const T *z;
  int64_t ldz;
  double *st;
  int64_t ldst;
  T alpha, beta, gamma;
  const T *diag;
  const FlipEntry *flips;  // ordered: in-tile masks, masks above the tile, mixed masks
  int nflip;
  int nlow;     // flips whose x-mask stays inside one tile (LDS)
  int nhigh;    // end of the flips whose x-mask lies entirely above the tile
  int b;        // columns
  int log2R;    // rows per tile = 2^log2R
  int ntiles;
  int xcd_remap;
};

// Arguments of the high-bit pass of the two-pass apply: the tile is the coset
// {l0 + w + (j << lo_bits) : w < W, j < 2^(L - lo_bits)}, l0 = tile * W, and
//   y += alpha * sum over flips with every mask bit >= lo_bits (from LDS)
//      + alpha * sum over mixed-mask flips (partner rows gathered from global)
// followed by the optional FP64 sample store.
template <typename T>
struct HiArgs {
  const T *x;
  int64_t ldx;
  T *y;
  int64_t ldy;
  double *st;
  int64_t ldst;
  T alpha;
  const FlipEntry *flips;  // high-range flips, then mixed flips
  int nhi;
  int nflip;
  int b;
  int lo_bits;
  int hi_bits;
  int W;
  int ntiles;
};

// Fused alternating-split kernels for a chain z_{j+1} = c_j H z_j + r_j, with
// H = (D + Lo) + Hi (diagonal and flips below bit lo_bits | flips at or above it) and r_j a
// combination of earlier terms.  With the partial P = c_j (other half) z_j + r_j, one kernel
// completes z_{j+1} with its half X of H and starts the next partial with the same half:
//   T_new = P + a_fin X T_cur ;  P <- a_start X T_new + b_cur T_cur (+ c_old Old)
// X = D + Lo for the lo tile kernel and Hi for the hi coset kernel.  The evolution
// T_{j+1} = 2G T_j - T_{j-1} takes a_fin = a_start = 2/E_b, b_cur = -1 and no Old term; the
// filter's two applies per order take the coefficients of its recurrence (filter_steps_fused).
// T_new may be written over the buffer of an earlier term; P is updated in place.
// The blocks are contiguous [D][b] with b * sizeof(T) a multiple of 16 bytes and
// D * b * sizeof(T) < 2^32 (32-bit byte offsets from the block's base).
template <typename T>
struct RecArgs {
  const T *tcur;
  T *tnew;
  T *p;
  const T *old;  // optional third block of the new partial (same layout)
  double *st;   // optional FP64 copy of T_new (basis sample), row stride ldst
  int64_t ldst;
  int64_t ld;   // row stride of tcur, tnew, p (= b)
  T a_fin, a_start, b_cur, c_old;
  const T *diag;
  const FlipEntry *flips;  // read-only while a kernel runs (loaded through the scalar cache)
  int nflip;
  int nplain;   // flips[0, nplain) have z-mask 0
  int b;
  int lo_bits;
  int hi_bits;
  int W;        // hi kernel: adjacent rows per coset tile (power of two)
  int threads;  // 512 or 1024
  int ntiles;
  int grid;     // > 0 and < ntiles: persistent launch of `grid` workgroups (tiles prefetched)
  int xcd_remap;
};

// One column of one realisation for the batched persistent kernel (batch.hip).  Read by the
// kernel through the scalar cache: the table is not written while the kernel runs.
struct BatchCol {
  const FlipEntry *flips;  // the realisation's flip table, sign-free flips first (all applied from LDS)
  const double *d64;       // diagonal tables
  const float *d32;
  const double *psi0;      // start column: psi0[s * ld_psi]
  double *V;               // the realisation's basis shifted to this column: panel p at V[s * ldv + p * b]
  const int *ks;           // sample orders k_1 < ... < k_n (device)
  int *bound_flag;         // set to 1 when |T_k(G) psi_E| > 1 is seen (bound below ||H||)
  double *scratch;         // 2 x 2^L doubles owned by this column (older recurrence terms at L = 14)
  double *A;               // anchors (moment projection) shifted to this column: anchor i at A[s * lda + i * b]
  const int *ka;           // anchor orders, ascending (device; n_anchor of them, 0 = none)
  int64_t ld_psi, ldv, lda;
  double f_alpha, f_beta, f_gamma;  // damped filter step coefficients
  double f_first_a, f_first_b;      // first order: T^_1 = a H (H psi) + b psi
  double inv_e;                     // 1 / E_b
  int L, nflip, nplain, K, n32, n_samples, b, n_anchor;  // flips[0, nplain) have z-mask 0
};
hipError_t launch_batch_chebyshev(const BatchCol *cols, int ncols, int max_L, hipStream_t s);

// One Lanczos run (kind 0) or one Chebyshev-moment vector (kind 1) of one realisation for the
// batched spectral kernel (batch.hip); output layout documented there.
struct BatchSpec {
  const FlipEntry *flips;  // sign-free flips first
  const double *d64;
  const double *start;     // start vector: start[s * ld]
  double *scratch;         // 2^L doubles at L = 14, else unused
  double *out;             // kind 0: 2 steps + 1 doubles; kind 1: steps doubles
  int64_t ld;
  double inv_e;            // kind 1: 1 / E_b
  int L, nflip, nplain, kind, steps;
};
hipError_t launch_batch_spectral(const BatchSpec *specs, int n, int max_L, hipStream_t s);

// One problem of the batched dense eigensolver (beig.hip): A (n x n, ld n) is destroyed and keeps
// the Householder reflectors (row k: beta_k at column k, v_k at columns k+1..); Zr gets the
// tridiagonal's eigenvectors as rows (unsorted), w the eigenvalues (unsorted, w[j] pairs with row j
// of Zr); status 0 = converged.
struct BatchEigProblem {
  double *A;
  double *Zr;
  double *work;  // batch_syev_work_doubles(n) doubles for the back-transformation, or null
  double *w;
  int *status;
  int n;
};
constexpr int kBatchEigMaxN = 2048;
// dacp_central_eigs_batched calls with at most this many realisations use the per-problem
// eigensolver on the finishing threads' streams instead of the batched launch.
constexpr int kBatchEigMinCount = 8;
// pipe = 1: pipelined multishift batches on large blocks; max_sweeps caps the sweeps per batch.
hipError_t launch_batch_syev(const BatchEigProblem *probs, int count, int max_n, hipStream_t s, int pipe,
                             int max_sweeps);

// Launch helpers (kernels.hip).
template <typename T>
hipError_t launch_rec_lo(const RecArgs<T> &a, hipStream_t s);
template <typename T>
hipError_t launch_rec_hi(const RecArgs<T> &a, hipStream_t s);
template <typename T>
hipError_t launch_step(const StepArgs<T> &a, hipStream_t s, int role);
template <typename T>
hipError_t launch_step_hi(const HiArgs<T> &a, hipStream_t s, int role);
template <typename T>
hipError_t launch_step_lo(const StepArgs<T> &a, hipStream_t s, int role);

hipError_t launch_diag(const uint32_t *zm, const double *c, int nterm, int64_t D, double *d64, float *d32,
                       hipStream_t s);
// partial[blk][j] = sum over a row range of x[s][j] * y[s][j]; out[j] = fixed-order sum of partials.
hipError_t launch_coldots(const void *x, int64_t ldx, const void *y, int64_t ldy, int dtype, int64_t D, int b,
                          double *partial, int nblk, double *out, hipStream_t s);
int coldots_blocks(int64_t D, int b);
hipError_t launch_colscale(double *x, int64_t ldx, int64_t D, int b, const double *sq_norms, hipStream_t s);
hipError_t launch_copy_cols(const double *x, int64_t ldx, double *y, int64_t ldy, int64_t D, int b, hipStream_t s);
hipError_t launch_convert_f64_to_f32(const double *x, int64_t ldx, float *y, int64_t ldy, int64_t D, int b,
                                     hipStream_t s);
hipError_t launch_convert_f32_to_f64(const float *x, int64_t ldx, double *y, int64_t ldy, int64_t D, int b,
                                     hipStream_t s);
hipError_t launch_philox_gauss(double *out, int64_t D, int b, uint64_t seed, hipStream_t s);
// Columns j < b_even of the [D][b] block <- psi + P psi, the others psi - P psi, P the global spin
// flip (s -> s ^ (D - 1)).
hipError_t launch_parity_split(double *psi, int64_t D, int b, int b_even, hipStream_t s);
hipError_t launch_axpby(double *y, const double *x, double a, double bcoef, int64_t n, hipStream_t s);
// residual: with r_j = hx_j - theta_j x_j, out[3j] = ||r_j||^2, out[3j+1] = ||x_j||^2,
// out[3j+2] = x_j . r_j (two stages; partial holds nblk * 3 b doubles).
hipError_t launch_resid(const double *x, const double *hx, int64_t ld, const double *theta, int64_t D, int b,
                        double *partial, int nblk, double *out, hipStream_t s);

// Moment mode (App. C, Eq. shift; kernels.hip).  out (bx x gy, contiguous) = X^T Y for X (D x bx)
// and Y (D x gy), bx gy <= 1024; partial holds nblk bx gy doubles, nblk = tall_gram_blocks(D).
int tall_gram_blocks(int64_t D);
hipError_t launch_tall_gram(const double *X, int64_t ldx, int bx, const double *Y, int64_t ldy, int gy, int64_t D,
                            double *partial, int nblk, double *out, hipStream_t s);
// The anchors' moments on the device (kernels.hip): M (2 x nrules b x b blocks, mu then nu) from the
// Gram product G ((2 na b) x m) by the derivation rules (ai, q, other; other = -1 or an earlier rule).
hipError_t launch_moment_chain(const double *G, int64_t m, int b, int na, const int *rules, int nrules, double scale0,
                               double scale1, double *M, int *bad, hipStream_t s);
// out (m x m, m = npan b) block (p, q) = scale (M_{x+y} + M_{|x-y|}) / 2 from the moment slots.
hipError_t launch_gram_assemble(const double *mu, const int *idx_of, const int64_t *orders, int b, int npan,
                                double scale, double *out, int64_t ld, hipStream_t s);
// dst[r][c] = src[r][cols[c]] * scale[c] for r < D, c < w (scale may be null).
hipError_t launch_gather_cols(const double *src, int64_t lds, const int *cols, const double *scale, int64_t D, int w,
                              double *dst, int64_t ldd, hipStream_t s);

// FP64 MFMA GEMM (gemm.hip).  C = alpha op(A) op(B) + beta C, row-major.
// upper: only output tiles with tile_row <= tile_col (symmetric results).
hipError_t launch_dgemm(int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                        int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc, int upper,
                        hipStream_t s);
// Same with K split over `splits` workgroup layers; work holds splits * M * N doubles (not upper).
hipError_t launch_dgemm_splitk(int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha, const double *A,
                               int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc,
                               int upper, int splits, double *work, hipStream_t s);
hipError_t launch_mirror_upper(double *C, int64_t n, int64_t ldc, hipStream_t s);
hipError_t launch_symmetrize(double *C, int64_t n, int64_t ldc, hipStream_t s);

hipError_t launch_gather_rows(const double *src, int64_t lds, double *dst, int64_t ldd, const int *perm,
                              const double *scale, int rows, int cols, hipStream_t s);

// Cached, stream-ordered allocation for the calling thread.  While an AllocStream is alive on a
// thread, the DevBufs that thread allocates come from a per-device block cache and the DevBufs it
// frees go back to it: a freed block carries an event recorded on the freeing thread's stream,
// and the next user's stream waits on that event before the block is handed out, so reuse is
// ordered behind every use on the freeing stream.  hipFree synchronises the whole device and
// hipMalloc maps fresh memory; threads that each drive their own stream would otherwise serialise
// on them.  The cache keeps freed blocks (rounded up to a size class, at most 1/4 larger) until
// the process ends, up to kBlockCacheBytes per device; beyond that a freed block is released.
// A pooled buffer must be used only on its scope's stream, or on other streams whose work the
// host has waited for before the buffer is freed.
constexpr size_t kBlockCacheBytes = size_t(32) << 30;
// The calling thread's allocation scope (on = an AllocStream is alive; s may be the null stream).
struct AllocState {
  bool on = false;
  hipStream_t s = nullptr;
  int device = 0;
};
AllocState &alloc_state_tl();
struct AllocStream {
  AllocState prev;
  AllocStream(hipStream_t s, int device);
  ~AllocStream();
  AllocStream(const AllocStream &) = delete;
  AllocStream &operator=(const AllocStream &) = delete;
};
hipError_t pool_alloc(size_t nbytes, hipStream_t s, int device, void **p, size_t *cls);
void pool_free(void *p, size_t cls, int device, hipStream_t s);

// Device allocation owned by a scope.
struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
  size_t pool_cls = 0;                // size class of a cached block, 0 = plain hipMalloc
  hipStream_t pool_stream = nullptr;  // stream it was handed out on
  int pool_device = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  hipError_t alloc(size_t nbytes) {
    release();
    bytes = nbytes;
    if (!nbytes) return hipSuccess;
    const AllocState &as = alloc_state_tl();
    hipError_t e;
    if (as.on) {
      e = pool_alloc(nbytes, as.s, as.device, &p, &pool_cls);
      if (e == hipSuccess) {
        pool_stream = as.s;
        pool_device = as.device;
      }
    } else {
      e = hipMalloc(&p, nbytes);
    }
    if (e != hipSuccess) {
      p = nullptr;
      pool_cls = 0;
    }
    return e;
  }
  void release() {
    if (p) {
      if (pool_cls) {
        const AllocState &as = alloc_state_tl();
        pool_free(p, pool_cls, pool_device, as.on ? as.s : pool_stream);
      } else {
        (void)hipFree(p);
      }
    }
    p = nullptr;
    bytes = 0;
    pool_cls = 0;
    pool_stream = nullptr;
  }
  template <typename T>
  T *as() const {
    return static_cast<T *>(p);
  }
};

}  // namespace dacp

struct dacp_ctx_s {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  double *red = nullptr;  // reduction partials
  size_t red_elems = 0;
  double *red_out = nullptr;
  size_t red_out_elems = 0;
  int tile_elems = dacp::kTileElemsDefault;  // apply-kernel tile size (elements), power of two in [256, 8192]
  int two_pass_min_L = 15;    // use the two-pass apply from this L on (0 disables it)
  int fused_rec = 1;          // alternating-split fused recurrence in the evolution (0 disables it)
  int pass_tile_elems = 4096;  // elements per LDS tile of the two-pass / fused kernels
  int group_default = 8;       // evolution column-group width for L >= 15
  int rec_hi_w = 0;            // fused recurrence: adjacent rows per high-bit tile (0 = automatic)
  int rec_threads = 1024;      // fused recurrence: threads per workgroup (512 or 1024)
  int rec_tile_elems = 8192;   // fused recurrence: largest tile, elements
  int rec_persist = 0;         // fused recurrence: persistent workgroups per CU (0 = one per tile)
  int rec_graph = 0;           // evolution: steps per captured graph below 2^19 rows (0 = no graphs)
  int batch_eig = 1;           // batched realisations' eigensolver: 1 = batched launches when the call has more
                               // than kBatchEigMinCount realisations, 2 = always, 0 = never
  int moment_explicit = 1;     // moment projection (moment_mode 2): explicit S, P of the same basis when the core
                               // falls short of N (1), always (2), never (0)
  int beig_pipe = 1;           // batched eigensolver: pipelined multishift QR batches on large blocks
  int beig_sweeps = 6;         // batched eigensolver: at most this many QR sweeps per batch (1..8)
  int project_whole = 1;       // projection: P in one GEMM when H V fits beside V (0 = column chunks)
  int project_splitk = 1;      // projection: upper-triangle split-K products when the output has few tiles
  int rec_xcd = 2;             // fused recurrence: XCD-contiguous tile order, bit 0 low pass, bit 1 high pass
  int num_cus = 256;           // compute units of the device
  int batch_workers = 16;      // host threads (each with its own stream) finishing batched realisations
  int filter_group_f64 = 8;    // filter column-group width for L >= 15, FP64 recurrence
  int filter_group_f32 = 8;    // filter column-group width for L >= 15, FP32 recurrence (its FP64 tail
                               // runs on the same groups, and the fused chain needs 8 FP64 columns)
  int dc_min_n = 96;           // eigenvectors by divide and conquer from this size on (0 = never)
  int blocked_min_n = 3500;    // blocked tridiagonalisation and compact-WY Q from this size on (0 = never);
                               // below it the unblocked form issues fewer launches and is faster
};

struct dacp_ham_s {
  dacp_ctx ctx = nullptr;
  int L = 0;
  int64_t D = 0;
  double sum_abs = 0.0, sum_sq = 0.0;
  // coupling statistics of the merged Pauli strings (features of the learned window)
  double w_diag = 0.0, w_zz = 0.0, w_flip1 = 0.0, max_abs = 0.0;
  int n_strings = 0;
  bool flip_sym = false;  // H commutes with the global spin flip prod_i sigma^x_i
  double *d64 = nullptr;  // diagonal of H, FP64
  float *d32 = nullptr;   // same in FP32
  dacp::FlipEntry *flips = nullptr;
  std::vector<dacp::FlipEntry> flips_host;  // sorted by x-mask
  std::mutex tables_mu;                      // guards the lazily built flip orders below
  struct TileOrder {
    dacp::FlipEntry *dev = nullptr;
    int nlow = 0, nhigh = 0;
  };
  TileOrder by_log2r[31];  // flip table ordered for a tile of 2^log2R rows (built on first use)
  struct SplitOrder {
    dacp::FlipEntry *lo = nullptr;  // flips with every mask bit < lo_bits
    dacp::FlipEntry *hi = nullptr;  // flips with every mask bit >= lo_bits, then mixed ones
    int nlo = 0, nhi = 0, nmix = 0;
    int nlo_plain = 0, nhi_plain = 0;  // leading z-mask-free entries of lo / of the pure part of hi
  };
  SplitOrder split[31];  // flip tables for the two-pass apply with lo_bits = index
};
namespace dacp {
typedef dacp_ham_s::SplitOrder SplitOrder_t;
}  // namespace dacp

namespace dacp {
// Error helpers used by the API layer.
dacp_status set_err(dacp_ctx ctx, dacp_status st, const std::string &msg);
dacp_status hip_err(dacp_ctx ctx, hipError_t e, const char *what);
// Progress lines on stderr when the environment variable DACP_VERBOSE is set.
bool verbose();
void vlog(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
// Dense symmetric eigensolver (eig.hip).
dacp_status gpu_syev(dacp_ctx ctx, int n, double *A, int64_t ld, double *w, double *Zrows);
// Batched form (beig.hip): count matrices A[i] (device, n[i] x n[i], ld n[i], destroyed, n <= 2048)
// in one launch; w[i] (host) ascending; Zrows[i] (device, n x n, may be null) row j = eigenvector j.
dacp_status batch_syev(dacp_ctx ctx, int count, const int *n, double *const *A, double *const *w,
                       double *const *Zrows);
// Its two halves: the launches (Zr device n x n scratch per matrix, which receives the eigenvectors
// of A as unsorted rows when work[i] gives batch_syev_work_doubles(n) device doubles; w host,
// unsorted) and, per matrix on the caller's stream, the sort and the gather of Zr's rows into Zrows
// in ascending order.
dacp_status batch_syev_raw(dacp_ctx ctx, int count, const int *n, double *const *A, double *const *Zr,
                           double *const *work, double *const *w);
dacp_status batch_syev_finish(dacp_ctx ctx, int n, const double *w_raw, const double *Zr, double *w_out,
                              double *Zrows);
size_t batch_syev_work_doubles(int n);
// The allocation-free form (dacp_syev_batched_noalloc): every device buffer besides A and Zrows comes
// from one fixed device array of kNoAllocScratchBytes per device (beig.hip).  noalloc_scratch_init
// resolves that device's address once (call it with the device current); batch_syev_noalloc_bytes
// is the workspace a request needs.
constexpr size_t kNoAllocScratchBytes = size_t(128) << 20;
hipError_t noalloc_scratch_init(int device);
size_t batch_syev_noalloc_bytes(int count, const int *n);
dacp_status batch_syev_noalloc(dacp_ctx ctx, int count, const int *n, double *const *A, double *const *w,
                               double *const *Zrows);
bool host_tridiag_eig(const double *diag, const double *off, int n, double *w, double *Z);
dacp_status dc_tridiag(dacp_ctx ctx, int n, const double *d, const double *e, double *w, double *Z);
}  // namespace dacp

#define DACP_HIP(ctx, call)                                  \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return dacp::hip_err(ctx, e_, #call); \
  } while (0)

#define DACP_TRY(call)                \
  do {                                \
    const dacp_status s_ = (call);    \
    if (s_ != DACP_OK) return s_;     \
  } while (0)

namespace dacp {
// Host <-> device copies of host-side bookkeeping (pageable host memory).  Each one waits for
// the context stream, then copies with a blocking call: the host buffer is complete (to_host)
// or no longer needed (to_device) on return, and later work on the stream sees the data.
dacp_status to_host(dacp_ctx ctx, void *host, const void *dev, size_t bytes);
dacp_status to_device(dacp_ctx ctx, void *dev, const void *host, size_t bytes);
// rows x cols doubles between a contiguous host array and a device array with row stride lddev
// (staged through a contiguous device buffer: no pitched runtime copies)
dacp_status to_host_2d(dacp_ctx ctx, double *host, const double *dev, int64_t lddev, int64_t rows, int64_t cols);
dacp_status to_device_2d(dacp_ctx ctx, double *dev, int64_t lddev, const double *host, int64_t rows, int64_t cols);
}  // namespace dacp
