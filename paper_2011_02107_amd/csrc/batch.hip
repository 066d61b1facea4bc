// Batched Chebyshev path for many small realisations (L <= 14) in one persistent launch.
//
// Workgroup g owns column j of realisation r (descriptor cols[g]) and runs that column's
// whole recurrence on-chip: the vector being applied sits in LDS (one 2^L-long column,
// <= 128 KB in FP64), the other recurrence terms in registers (2^L / 1024 elements per
// thread).  In order it runs
//   1. the exp-semicircle filter T_K(F) psi (Sec. II.A, Eqs. F, filter) with the damped
//      recurrence T^_{k+1} = alpha H(H T^_k) + beta T^_k + gamma T^_{k-1}: the first K - tail
//      orders in FP32 (FP32 storage and accumulation), the last `tail` orders in FP64;
//   2. column normalisation (a fixed-order workgroup reduction);
//   3. the Chebyshev evolution T_{k+1} = 2 G T_k - T_{k-1}, G = H / E_b (Sec. II.B), storing
//      the panels T_{k_m - 1}, T_{k_m} into the realisation's basis V (App. C, Eq. set2) and
//      checking |T_{k_m}| <= |psi_E| at every sample.
// Global memory is touched only for the start column, the diagonal table (cached) and the
// samples.  Every element's flip sum runs in the flip-table order, as in the other kernels.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace dacp {

namespace {

constexpr int kBT = 1024;  // threads per workgroup

typedef const __attribute__((address_space(4))) BatchCol *ConstBatchCols;
typedef const __attribute__((address_space(4))) FlipEntry *ConstFlipTable;
typedef const __attribute__((address_space(4))) int *ConstInts;

// Global accesses as a uniform base plus a 32-bit byte offset (every offset here is < 2^32,
// checked on the host), so the per-element address is one 32-bit register instead of a
// 64-bit pointer per array kept live across the step loops.
// threadIdx.x * scale, opaque to loop-invariant code motion: an empty asm statement (no
// instruction) redefines the value, so the addresses derived from it are formed where they are
// used instead of being hoisted out of the step loops and held in registers for the whole kernel.
__device__ __forceinline__ uint32_t tid_off(uint32_t scale) {
  uint32_t o = threadIdx.x * scale;
  asm volatile("" : "+v"(o));
  return o;
}

template <typename T>
__device__ __forceinline__ T ld_at(const T *base, uint32_t byte_off) {
  return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(base) + byte_off);
}
template <typename T>
__device__ __forceinline__ void st_at(T *base, uint32_t byte_off, T x) {
  *reinterpret_cast<T *>(reinterpret_cast<char *>(base) + byte_off) = x;
}

// The flip terms of H for the elements ib .. ib + C - 1 of this thread, added to v from lds (which
// holds the vector being applied): the sign-free flips first, then the others.
template <typename T, int E, int C>
__device__ __forceinline__ void chunk_flips(T (&v)[E], const T *lds, ConstFlipTable flips, int nplain, int nflip,
                                            int ib) {
#pragma nounroll
  for (int t = 0; t < nplain; ++t) {
    const uint32_t xm = flips[t].xmask;
    const T c = static_cast<T>(flips[t].coef);
#pragma unroll
    for (int i = ib; i < ib + C; ++i) v[i] += c * lds[(threadIdx.x + i * kBT) ^ xm];
  }
#pragma nounroll
  for (int t = nplain; t < nflip; ++t) {
    const uint32_t xm = flips[t].xmask;
    const uint32_t zm = flips[t].zmask;
    const T c = static_cast<T>(flips[t].coef);
#pragma unroll
    for (int i = ib; i < ib + C; ++i) {
      const uint32_t src = (threadIdx.x + i * kBT) ^ xm;
      v[i] += ((__popc(src & zm) & 1) ? -c : c) * lds[src];
    }
  }
}

// Stores this thread's elements s = tid + i * kBT (i < E) of v into lds between barriers.
template <typename T, int E>
__device__ __forceinline__ void stage_column(const T (&v)[E], T *lds, uint32_t D) {
  __syncthreads();  // the previous apply's readers are done with lds
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const uint32_t s = threadIdx.x + i * kBT;
    if (E > 1 || s < D) lds[s] = v[i];
  }
  __syncthreads();
}

// v <- H v for this thread's elements s = tid + i * kBT (i < E); lds holds the whole column
// while the flips are summed.  E = 1 also covers D < kBT (threads with s >= D idle).  Elements go
// in chunks of at most 4, each chunk running the whole flip list: bounds the loads in flight, and
// the registers holding them, independently of E.  A chunk's diagonal entries are loaded first and
// applied last (to the element's own value, read back from lds), so their global-load latency runs
// under the chunk's flips.
template <typename T, int E>
__device__ __forceinline__ void apply_inplace(T (&v)[E], T *lds, const T *diag, ConstFlipTable flips, int nplain,
                                              int nflip, uint32_t D) {
  stage_column<T, E>(v, lds, D);
  if (E == 1 && threadIdx.x >= D) return;
  constexpr int C = E < 4 ? E : 4;
#pragma unroll
  for (int ib = 0; ib < E; ib += C) {
    T dg[C];
#pragma unroll
    for (int i = ib; i < ib + C; ++i) {
      dg[i - ib] = ld_at(diag, tid_off(sizeof(T)) + static_cast<uint32_t>(i * kBT * sizeof(T)));
      v[i] = static_cast<T>(0);
    }
    chunk_flips<T, E, C>(v, lds, flips, nplain, nflip, ib);
#pragma unroll
    for (int i = ib; i < ib + C; ++i) v[i] += dg[i - ib] * lds[threadIdx.x + i * kBT];
  }
}

// Sum over the workgroup in a fixed order (wave shuffles, then the waves in index order).
__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < kBT / 64; ++w) t += red[w];
  return t;
}

template <int E>
__device__ __forceinline__ double sum_sq(const double (&v)[E], uint32_t D, double *red) {
  double p = 0.0;
#pragma unroll
  for (int i = 0; i < E; ++i)
    if (E > 1 || threadIdx.x < D) p += v[i] * v[i];
  return block_sum(p, red);
}

template <int E>
__device__ __forceinline__ void store_panel(double *V, int64_t ldv, int64_t col, const double (&v)[E], uint32_t D) {
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const uint32_t s = tid_off(1u) + static_cast<uint32_t>(i * kBT);
    if (E > 1 || s < D) st_at(V, (s * static_cast<uint32_t>(ldv) + static_cast<uint32_t>(col)) * 8u, v[i]);
  }
}

// Store T_kk when kk is a sample order; at k_m also check |T_{k_m}|^2 <= 1 (unit start column).
template <int E>
__device__ __forceinline__ void sample_at(const BatchCol &c, ConstInts ks, int &next, int64_t kk, const double (&T)[E],
                                          uint32_t D, double *red) {
  if (next >= c.n_samples) return;
  const int64_t km = ks[next];
  if (kk == km - 1) store_panel<E>(c.V, c.ldv, static_cast<int64_t>(2 * next + 1) * c.b, T, D);
  if (kk == km) {
    store_panel<E>(c.V, c.ldv, static_cast<int64_t>(2 * next + 2) * c.b, T, D);
    const double n2 = sum_sq<E>(T, D, red);
    if (!(n2 <= 1.0 + 2e-6) && threadIdx.x == 0) *c.bound_flag = 1;
    ++next;
  }
}

// Store T_kk into the anchor slot when kk is the next anchor order (the moment projection).
template <int E>
__device__ __forceinline__ void anchor_at(const BatchCol &c, ConstInts ka, int &next, int64_t kk, const double (&T)[E],
                                          uint32_t D) {
  if (next >= c.n_anchor || ka[next] != kk) return;
  store_panel<E>(c.A, c.lda, static_cast<int64_t>(next) * c.b, T, D);
  ++next;
}

// A recurrence term held per thread: in registers when a thread holds <= 8 elements (g is then
// never used and may be null), otherwise in a 2^L-double slice of the column's global scratch,
// read back only by the thread that wrote it (L2 resident).
template <int E>
struct Held {
  static constexpr bool kRegs = E <= 8;
  double r[kRegs ? E : 1];
  double *g;
  // i: element slot; boff: its byte offset (element index * 8)
  __device__ __forceinline__ double get(int i, uint32_t boff) const { return kRegs ? r[kRegs ? i : 0] : ld_at(g, boff); }
  __device__ __forceinline__ void set(int i, uint32_t boff, double x) {
    if (kRegs) r[kRegs ? i : 0] = x;
    else st_at(g, boff, x);
  }
};

// One evolution step T_(k+1) = (2 / e) H T_k - T_(k-1) (Sec. II.B): v holds T_k on entry and
// T_(k+1) on exit, A holds T_(k-1) on entry and T_k on exit.  The apply of apply_inplace with the
// combination done per chunk, so that the chunk's T_(k-1) loads (global when A lives in the column
// scratch) run under its flips together with the diagonal loads.
template <int E>
__device__ __forceinline__ void evolve_step(double (&v)[E], double *lds, const double *diag, ConstFlipTable flips,
                                            int nplain, int nflip, uint32_t D, Held<E> &A, double two_inv_e) {
  stage_column<double, E>(v, lds, D);
  if (E == 1 && threadIdx.x >= D) return;
  constexpr int C = E < 4 ? E : 4;
#pragma unroll
  for (int ib = 0; ib < E; ib += C) {
    double dg[C], pa[C];
#pragma unroll
    for (int i = ib; i < ib + C; ++i) {
      const uint32_t bo = tid_off(8u) + static_cast<uint32_t>(i * kBT * 8);
      dg[i - ib] = ld_at(diag, bo);
      pa[i - ib] = A.get(i, bo);
      v[i] = 0.0;
    }
    chunk_flips<double, E, C>(v, lds, flips, nplain, nflip, ib);
#pragma unroll
    for (int i = ib; i < ib + C; ++i) {
      const uint32_t bo = tid_off(8u) + static_cast<uint32_t>(i * kBT * 8);
      const double x = lds[threadIdx.x + i * kBT];
      const double hv = v[i] + dg[i - ib] * x;
      A.set(i, bo, x);
      v[i] = two_inv_e * hv - pa[i - ib];
    }
  }
}

template <int E>
__device__ __forceinline__ void run_column(const BatchCol &c, ConstFlipTable flips, ConstInts ks, ConstInts ka,
                                           unsigned char *smem, double *red) {
  const uint32_t D = 1u << c.L;
  double *lds64 = reinterpret_cast<double *>(smem);
  float *lds32 = reinterpret_cast<float *>(smem);
  const bool active = E > 1 || threadIdx.x < D;
  Held<E> A, Bk;  // T_(k-1); T^_k during an FP64 filter order
  A.g = c.scratch;
  Bk.g = c.scratch ? c.scratch + D : nullptr;
  double v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const uint32_t s = threadIdx.x + i * kBT;
    v[i] = active ? ld_at(c.psi0, s * static_cast<uint32_t>(c.ld_psi) * 8u) : 0.0;  // start column
  }

  // ---- filter: on exit v = T^_K, A = T^_(K-1)
  int tail = 0;
  if (c.K == 0) {
    // psi_E = psi
  } else if (c.n32 >= 1) {
    float Af[E], Bf[E], Tf[E];
    const float fa = static_cast<float>(c.f_alpha), fb = static_cast<float>(c.f_beta);
    const float fg = static_cast<float>(c.f_gamma);
#pragma unroll
    for (int i = 0; i < E; ++i) {
      Af[i] = static_cast<float>(v[i]);
      Tf[i] = Af[i];
    }
    apply_inplace<float, E>(Tf, lds32, c.d32, flips, c.nplain, c.nflip, D);
    apply_inplace<float, E>(Tf, lds32, c.d32, flips, c.nplain, c.nflip, D);
    const float f1a = static_cast<float>(c.f_first_a), f1b = static_cast<float>(c.f_first_b);
#pragma unroll
    for (int i = 0; i < E; ++i) Bf[i] = f1a * Tf[i] + f1b * Af[i];
    for (int k = 1; k < c.n32; ++k) {
#pragma unroll
      for (int i = 0; i < E; ++i) Tf[i] = Bf[i];
      apply_inplace<float, E>(Tf, lds32, c.d32, flips, c.nplain, c.nflip, D);
      apply_inplace<float, E>(Tf, lds32, c.d32, flips, c.nplain, c.nflip, D);
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const float nb = fa * Tf[i] + fb * Bf[i] + fg * Af[i];
        Af[i] = Bf[i];
        Bf[i] = nb;
      }
    }
    if (active) {
#pragma unroll
      for (int i = 0; i < E; ++i) {
        A.set(i, tid_off(8u) + static_cast<uint32_t>(i * kBT * 8), static_cast<double>(Af[i]));
        v[i] = static_cast<double>(Bf[i]);
      }
    }
    tail = c.K - c.n32;
  } else {
    if (active) {
#pragma unroll
      for (int i = 0; i < E; ++i) A.set(i, tid_off(8u) + static_cast<uint32_t>(i * kBT * 8), v[i]);
    }
    apply_inplace<double, E>(v, lds64, c.d64, flips, c.nplain, c.nflip, D);
    apply_inplace<double, E>(v, lds64, c.d64, flips, c.nplain, c.nflip, D);
    if (active) {
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const uint32_t bo = tid_off(8u) + static_cast<uint32_t>(i * kBT * 8);
        v[i] = c.f_first_a * v[i] + c.f_first_b * A.get(i, bo);
      }
    }
    tail = c.K - 1;
  }
  for (int k = 0; k < tail; ++k) {
    if (active) {
#pragma unroll
      for (int i = 0; i < E; ++i) Bk.set(i, tid_off(8u) + static_cast<uint32_t>(i * kBT * 8), v[i]);
    }
    apply_inplace<double, E>(v, lds64, c.d64, flips, c.nplain, c.nflip, D);
    apply_inplace<double, E>(v, lds64, c.d64, flips, c.nplain, c.nflip, D);
    if (active) {
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const uint32_t bo = tid_off(8u) + static_cast<uint32_t>(i * kBT * 8);
        const double b = Bk.get(i, bo);
        const double nb = c.f_alpha * v[i] + c.f_beta * b + c.f_gamma * A.get(i, bo);
        A.set(i, bo, b);
        v[i] = nb;
      }
    }
  }

  // ---- normalise: psi_E = v / |v|
  {
    const double inv = 1.0 / sqrt(sum_sq<E>(v, D, red));
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] *= inv;
  }

  // ---- evolution: A = T_(k-1), v = T_k
  store_panel<E>(c.V, c.ldv, 0, v, D);
  int next = 0, next_a = 0;
  anchor_at<E>(c, ka, next_a, 0, v, D);
  if (active) {
#pragma unroll
    for (int i = 0; i < E; ++i) A.set(i, tid_off(8u) + static_cast<uint32_t>(i * kBT * 8), v[i]);
  }
  apply_inplace<double, E>(v, lds64, c.d64, flips, c.nplain, c.nflip, D);
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] *= c.inv_e;
  sample_at<E>(c, ks, next, 1, v, D, red);
  anchor_at<E>(c, ka, next_a, 1, v, D);
  int64_t kmax = c.n_samples > 0 ? ks[c.n_samples - 1] : 1;
  if (c.n_anchor > 0 && ka[c.n_anchor - 1] > kmax) kmax = ka[c.n_anchor - 1];
  const double two_inv_e = 2.0 * c.inv_e;
  for (int64_t k = 1; k < kmax; ++k) {
    evolve_step<E>(v, lds64, c.d64, flips, c.nplain, c.nflip, D, A, two_inv_e);
    sample_at<E>(c, ks, next, k + 1, v, D, red);
    anchor_at<E>(c, ka, next_a, k + 1, v, D);
  }
}

__global__ __launch_bounds__(kBT) void k_batch_chebyshev(const BatchCol *cols_g) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[kBT / 64];
  // field by field through the constant address space (uniform scalar loads)
  const ConstBatchCols cc = (ConstBatchCols)cols_g + blockIdx.x;
  BatchCol c;
  c.flips = cc->flips;
  c.d64 = cc->d64;
  c.d32 = cc->d32;
  c.psi0 = cc->psi0;
  c.V = cc->V;
  c.ks = cc->ks;
  c.bound_flag = cc->bound_flag;
  c.scratch = cc->scratch;
  c.A = cc->A;
  c.ka = cc->ka;
  c.ld_psi = cc->ld_psi;
  c.ldv = cc->ldv;
  c.lda = cc->lda;
  c.f_alpha = cc->f_alpha;
  c.f_beta = cc->f_beta;
  c.f_gamma = cc->f_gamma;
  c.f_first_a = cc->f_first_a;
  c.f_first_b = cc->f_first_b;
  c.inv_e = cc->inv_e;
  c.L = cc->L;
  c.nflip = cc->nflip;
  c.nplain = cc->nplain;
  c.K = cc->K;
  c.n32 = cc->n32;
  c.n_samples = cc->n_samples;
  c.b = cc->b;
  c.n_anchor = cc->n_anchor;
  const ConstFlipTable flips = (ConstFlipTable)c.flips;
  const ConstInts ks = (ConstInts)c.ks;
  const ConstInts ka = (ConstInts)c.ka;
  switch (c.L) {  // elements per thread: 2^L / 1024, at least 1
    case 14: run_column<16>(c, flips, ks, ka, smem_raw, red); break;
    case 13: run_column<8>(c, flips, ks, ka, smem_raw, red); break;
    case 12: run_column<4>(c, flips, ks, ka, smem_raw, red); break;
    case 11: run_column<2>(c, flips, ks, ka, smem_raw, red); break;
    default: run_column<1>(c, flips, ks, ka, smem_raw, red); break;
  }
}

// ---------------------------------------------------------------------------
// Batched spectral estimates (the bound and density step of Sec. III for many realisations):
// workgroup g runs either the Lanczos recurrence of one realisation (kind 0) or the Chebyshev
// moment recurrence of one random vector of one realisation (kind 1) with the whole column on
// chip, and writes the scalars the host needs:
//   kind 0: out[j] = alpha_j, out[steps + j] = beta_j, out[2 steps] = number of steps taken;
//   kind 1: out[0] = <r, r>, out[1] = <r, T_1 r>, out[2k] = <T_k r, T_k r>,
//           out[2k + 1] = <T_(k+1) r, T_k r>  (k >= 1, indices below `steps` = M).
// ---------------------------------------------------------------------------
template <int E>
__device__ __forceinline__ double dot_held(const double (&v)[E], const Held<E> &A, uint32_t D, double *red) {
  double p = 0.0;
  if (E > 1 || threadIdx.x < D) {
#pragma unroll
    for (int i = 0; i < E; ++i) p += v[i] * A.get(i, tid_off(8u) + static_cast<uint32_t>(i * kBT * 8));
  }
  return block_sum(p, red);
}

template <int E>
__device__ __forceinline__ void run_spectral(const BatchSpec &c, ConstFlipTable flips, unsigned char *smem,
                                             double *red) {
  const uint32_t D = 1u << c.L;
  double *lds = reinterpret_cast<double *>(smem);
  const bool active = E > 1 || threadIdx.x < D;
  Held<E> A;
  A.g = c.scratch;
  double v[E];
#pragma unroll
  for (int i = 0; i < E; ++i) {
    const uint32_t s = threadIdx.x + i * kBT;
    v[i] = active ? ld_at(c.start, s * static_cast<uint32_t>(c.ld) * 8u) : 0.0;
  }
  if (c.kind == 0) {
    // Lanczos: A = v_(j-1), v = v_j, w (in v after the apply) = H v_j - beta_(j-1) v_(j-1)
    {
      const double inv = 1.0 / sqrt(sum_sq<E>(v, D, red));
#pragma unroll
      for (int i = 0; i < E; ++i) v[i] *= inv;
    }
    double bprev = 0.0;
    int taken = 0;
    for (int j = 0; j < c.steps; ++j) {
      double w[E];
#pragma unroll
      for (int i = 0; i < E; ++i) w[i] = v[i];
      apply_inplace<double, E>(w, lds, c.d64, flips, c.nplain, c.nflip, D);  // lds keeps v_j
      if (j > 0 && active) {
#pragma unroll
        for (int i = 0; i < E; ++i) w[i] -= bprev * A.get(i, tid_off(8u) + static_cast<uint32_t>(i * kBT * 8));
      }
      double pa = 0.0;
      if (active) {
#pragma unroll
        for (int i = 0; i < E; ++i) pa += w[i] * v[i];
      }
      const double alpha = block_sum(pa, red);
#pragma unroll
      for (int i = 0; i < E; ++i) w[i] -= alpha * v[i];
      const double beta = sqrt(fmax(sum_sq<E>(w, D, red), 0.0));
      if (threadIdx.x == 0) {
        c.out[j] = alpha;
        c.out[c.steps + j] = beta;
      }
      taken = j + 1;
      if (!(beta > 1e-300) || j + 1 == c.steps) break;
      if (active) {
#pragma unroll
        for (int i = 0; i < E; ++i) {
          A.set(i, tid_off(8u) + static_cast<uint32_t>(i * kBT * 8), v[i]);
          v[i] = w[i] / beta;
        }
      }
      bprev = beta;
    }
    if (threadIdx.x == 0) c.out[2 * c.steps] = static_cast<double>(taken);
    return;
  }
  // Chebyshev moments of one random vector: A = T_(k-1) r, v = T_k r
  {
    const double n0 = sum_sq<E>(v, D, red);
    if (threadIdx.x == 0) c.out[0] = n0;
  }
  if (c.steps <= 1) return;
  if (active) {
#pragma unroll
    for (int i = 0; i < E; ++i) A.set(i, tid_off(8u) + static_cast<uint32_t>(i * kBT * 8), v[i]);
  }
  apply_inplace<double, E>(v, lds, c.d64, flips, c.nplain, c.nflip, D);
#pragma unroll
  for (int i = 0; i < E; ++i) v[i] *= c.inv_e;
  {
    const double m1 = dot_held<E>(v, A, D, red);
    if (threadIdx.x == 0) c.out[1] = m1;
  }
  const double two_inv_e = 2.0 * c.inv_e;
  for (int k = 1; 2 * k < c.steps; ++k) {
    const double tkk = sum_sq<E>(v, D, red);
    if (threadIdx.x == 0) c.out[2 * k] = tkk;
    if (2 * k + 1 >= c.steps) break;
    apply_inplace<double, E>(v, lds, c.d64, flips, c.nplain, c.nflip, D);  // lds keeps T_k r
    if (active) {
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const uint32_t bo = tid_off(8u) + static_cast<uint32_t>(i * kBT * 8);
        const double nb = two_inv_e * v[i] - A.get(i, bo);
        A.set(i, bo, ld_at(lds, bo));
        v[i] = nb;
      }
    }
    const double tk1k = dot_held<E>(v, A, D, red);
    if (threadIdx.x == 0) c.out[2 * k + 1] = tk1k;
  }
}

typedef const __attribute__((address_space(4))) BatchSpec *ConstBatchSpecs;

__global__ __launch_bounds__(kBT) void k_batch_spectral(const BatchSpec *specs_g) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ double red[kBT / 64];
  const ConstBatchSpecs cs = (ConstBatchSpecs)specs_g + blockIdx.x;
  BatchSpec c;
  c.flips = cs->flips;
  c.d64 = cs->d64;
  c.start = cs->start;
  c.scratch = cs->scratch;
  c.out = cs->out;
  c.ld = cs->ld;
  c.inv_e = cs->inv_e;
  c.L = cs->L;
  c.nflip = cs->nflip;
  c.nplain = cs->nplain;
  c.kind = cs->kind;
  c.steps = cs->steps;
  const ConstFlipTable flips = (ConstFlipTable)c.flips;
  switch (c.L) {
    case 14: run_spectral<16>(c, flips, smem_raw, red); break;
    case 13: run_spectral<8>(c, flips, smem_raw, red); break;
    case 12: run_spectral<4>(c, flips, smem_raw, red); break;
    case 11: run_spectral<2>(c, flips, smem_raw, red); break;
    default: run_spectral<1>(c, flips, smem_raw, red); break;
  }
}

}  // namespace

hipError_t launch_batch_chebyshev(const BatchCol *cols, int ncols, int max_L, hipStream_t s) {
  if (ncols <= 0) return hipSuccess;
  if (max_L < 1 || max_L > 14) return hipErrorInvalidValue;
  const size_t lds = (size_t(1) << max_L) * sizeof(double);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_batch_chebyshev),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_chebyshev, dim3(ncols), dim3(kBT), lds, s, cols);
  return hipGetLastError();
}

hipError_t launch_batch_spectral(const BatchSpec *specs, int n, int max_L, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (max_L < 1 || max_L > 14) return hipErrorInvalidValue;
  const size_t lds = (size_t(1) << max_L) * sizeof(double);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_batch_spectral),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_batch_spectral, dim3(n), dim3(kBT), lds, s, specs);
  return hipGetLastError();
}

}  // namespace dacp
