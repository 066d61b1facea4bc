// Streaming kernels of the DACP path on gfx950: the matrix-free Hamiltonian
// apply fused with the Chebyshev three-term combine, column reductions,
// start-state generation and small element-wise helpers.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace dacp {

// ---------------------------------------------------------------------------
// Fused apply + combine.
//
// A workgroup owns a tile of R = 2^log2R consecutive rows of the [D][b] block
// (R * b <= tile elements, 1024 by default).  The tile of x is staged in LDS; flips whose
// x-mask lies below bit log2R stay inside the tile and read LDS, the others
// read the partner rows s ^ x from global memory (L2 / MALL / HBM).  The
// diagonal d(s) comes from the precomputed table.  Work-groups are dealt to
// the 8 XCDs round-robin, so tile ids are remapped to give each XCD one
// contiguous eighth of the state space: partner rows of all but the top
// three bits then live in the same XCD's L2 region.
// ---------------------------------------------------------------------------
// ROLE only separates kernel symbols for profiling: 0 = plain apply / other,
// 1 = filter recurrence, 2 = evolution recurrence.
//
// Every thread owns EPT elements e = tid + i * 256 of the tile.  Elements past
// the tile end (only when R * b is not a multiple of 256) are clamped to the
// last element for loading and skipped when storing, so every load below is
// unconditional: the compiler then issues each term's EPT loads back to back
// and waits once, instead of serialising them behind per-element branches.
// For a flip whose mask lies above the tile, s ^ x = (row0 ^ x) + r, so the
// partner address is a wave-uniform base plus the element's own offset.
template <typename T, int EPT, int ROLE>
__global__ __launch_bounds__(kApplyThreads) void k_step(StepArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  T *tile = reinterpret_cast<T *>(smem_raw);
  const int bid = blockIdx.x;
  int t_id = bid;
  if (a.xcd_remap) {
    const int per = a.ntiles >> 3;
    t_id = (bid & 7) * per + (bid >> 3);
  }
  const int b = a.b;
  const int nel = (1 << a.log2R) * b;
  const uint32_t row0 = static_cast<uint32_t>(t_id) << a.log2R;
  const int64_t ldx = a.ldx;

  int rr[EPT], jj[EPT];
  uint32_t off[EPT];  // byte offset of the element inside any tile-shaped slab (fits 32 bits, checked on the host)
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    int e = threadIdx.x + i * kApplyThreads;
    e = e < nel ? e : nel - 1;
    rr[i] = e / b;
    jj[i] = e - rr[i] * b;
    off[i] = static_cast<uint32_t>((static_cast<int64_t>(rr[i]) * ldx + jj[i]) * static_cast<int64_t>(sizeof(T)));
  }
  T own[EPT], dg[EPT];
  {
    const char *xb = reinterpret_cast<const char *>(a.x + static_cast<int64_t>(row0) * ldx);
#pragma unroll
    for (int i = 0; i < EPT; ++i) own[i] = *reinterpret_cast<const T *>(xb + off[i]);
#pragma unroll
    for (int i = 0; i < EPT; ++i) dg[i] = a.diag[row0 + rr[i]];
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kApplyThreads;
    if (e < nel) tile[e] = own[i];
  }
  T acc[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) acc[i] = dg[i] * own[i];
  __syncthreads();

  for (int t = 0; t < a.nlow; ++t) {
    const uint32_t xm = a.flips[t].xmask;
    const uint32_t zm = a.flips[t].zmask;
    const T c = static_cast<T>(a.flips[t].coef);
    if (zm == 0) {  // X-type term: no sign (wave-uniform branch)
#pragma unroll
      for (int i = 0; i < EPT; ++i) acc[i] += c * tile[(rr[i] ^ static_cast<int>(xm)) * b + jj[i]];
    } else {
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const uint32_t src = (row0 + static_cast<uint32_t>(rr[i])) ^ xm;
        const T sg = (__popc(src & zm) & 1) ? -c : c;
        acc[i] += sg * tile[(rr[i] ^ static_cast<int>(xm)) * b + jj[i]];
      }
    }
  }
  // High flips, UNR terms at a time so that UNR * EPT loads are in flight per wave.
  constexpr int UNR = 4;
  int t = a.nlow;
  for (; t + UNR <= a.nhigh; t += UNR) {
    T g[UNR][EPT];
#pragma unroll
    for (int q = 0; q < UNR; ++q) {
      const char *xp = reinterpret_cast<const char *>(a.x + static_cast<int64_t>(row0 ^ a.flips[t + q].xmask) * ldx);
#pragma unroll
      for (int i = 0; i < EPT; ++i) g[q][i] = *reinterpret_cast<const T *>(xp + off[i]);
    }
#pragma unroll
    for (int q = 0; q < UNR; ++q) {
      const uint32_t pbase = row0 ^ a.flips[t + q].xmask;
      const uint32_t zm = a.flips[t + q].zmask;
      const T c = static_cast<T>(a.flips[t + q].coef);
      if (zm == 0) {
#pragma unroll
        for (int i = 0; i < EPT; ++i) acc[i] += c * g[q][i];
      } else {
#pragma unroll
        for (int i = 0; i < EPT; ++i) {
          const T sg = (__popc((pbase + static_cast<uint32_t>(rr[i])) & zm) & 1) ? -c : c;
          acc[i] += sg * g[q][i];
        }
      }
    }
  }
  for (; t < a.nhigh; ++t) {
    const uint32_t xm = a.flips[t].xmask;
    const uint32_t zm = a.flips[t].zmask;
    const T c = static_cast<T>(a.flips[t].coef);
    const uint32_t pbase = row0 ^ xm;
    const char *xp = reinterpret_cast<const char *>(a.x + static_cast<int64_t>(pbase) * ldx);
    T g[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) g[i] = *reinterpret_cast<const T *>(xp + off[i]);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const T sg = (__popc((pbase + static_cast<uint32_t>(rr[i])) & zm) & 1) ? -c : c;
      acc[i] += sg * g[i];
    }
  }
  // Masks with bits both inside and above the tile: partner row (row0 ^ x_hi) + (r ^ x_lo).
  const uint32_t lowmask = (1u << a.log2R) - 1u;
  for (; t < a.nflip; ++t) {
    const uint32_t xm = a.flips[t].xmask;
    const uint32_t zm = a.flips[t].zmask;
    const T c = static_cast<T>(a.flips[t].coef);
    const uint32_t xlo = xm & lowmask;
    const uint32_t pbase = row0 ^ (xm & ~lowmask);
    const T *xp = a.x + static_cast<int64_t>(pbase) * ldx;
    T g[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) g[i] = xp[static_cast<int64_t>(rr[i] ^ static_cast<int>(xlo)) * ldx + jj[i]];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const uint32_t src = pbase + (static_cast<uint32_t>(rr[i]) ^ xlo);
      const T sg = (__popc(src & zm) & 1) ? -c : c;
      acc[i] += sg * g[i];
    }
  }

  T uv[EPT], zv[EPT];
  if (a.u) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) uv[i] = a.u[static_cast<int64_t>(row0 + rr[i]) * a.ldu + jj[i]];
  }
  if (a.z) {
#pragma unroll
    for (int i = 0; i < EPT; ++i) zv[i] = a.z[static_cast<int64_t>(row0 + rr[i]) * a.ldz + jj[i]];
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * kApplyThreads;
    if (e < nel) {
      const int64_t s = row0 + rr[i];
      const int j = jj[i];
      T v = a.alpha * acc[i];
      if (a.u) v += a.beta * uv[i];
      if (a.z) v += a.gamma * zv[i];
      a.y[s * a.ldy + j] = v;
      if (a.st) a.st[s * a.ldst + j] = static_cast<double>(v);
    }
  }
}

template <typename T, int ROLE>
hipError_t launch_step_role(const StepArgs<T> &a, hipStream_t s) {
  const int nel = (1 << a.log2R) * a.b;
  const int ept = (nel + kApplyThreads - 1) / kApplyThreads;
  const size_t lds = static_cast<size_t>(nel) * sizeof(T);
  dim3 grid(a.ntiles), block(kApplyThreads);
  if (ept <= 1) hipLaunchKernelGGL((k_step<T, 1, ROLE>), grid, block, lds, s, a);
  else if (ept <= 2) hipLaunchKernelGGL((k_step<T, 2, ROLE>), grid, block, lds, s, a);
  else if (ept <= 4) hipLaunchKernelGGL((k_step<T, 4, ROLE>), grid, block, lds, s, a);
  else if (ept <= 8) hipLaunchKernelGGL((k_step<T, 8, ROLE>), grid, block, lds, s, a);
  else if (ept <= 16) hipLaunchKernelGGL((k_step<T, 16, ROLE>), grid, block, lds, s, a);
  else if (ept <= 32) hipLaunchKernelGGL((k_step<T, 32, ROLE>), grid, block, lds, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step(const StepArgs<T> &a, hipStream_t s, int role) {
  if (role == 1) return launch_step_role<T, 1>(a, s);
  if (role == 2) return launch_step_role<T, 2>(a, s);
  return launch_step_role<T, 0>(a, s);
}
template hipError_t launch_step<double>(const StepArgs<double> &, hipStream_t, int);
template hipError_t launch_step<float>(const StepArgs<float> &, hipStream_t, int);

// ---------------------------------------------------------------------------
// Low-bit pass of the two-pass apply: a tile of 2^log2R consecutive rows in
// LDS, every flip of the list has its mask below bit log2R, no global gathers:
//   y = alpha (d x + sum_t c_t sign_t x[s ^ m_t]) + beta u + gamma z.
// 1024 threads, EPT elements each; b is a power of two (b = 2^lb), so the
// element -> (row, column) split is a shift and a mask.
// ---------------------------------------------------------------------------
template <typename T, int EPT, int ROLE>
__global__ __launch_bounds__(1024) void k_step_lo(StepArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  T *tile = reinterpret_cast<T *>(smem_raw);
  const int lb = __ffs(a.b) - 1;
  const int nel = (1 << a.log2R) << lb;
  const uint32_t row0 = static_cast<uint32_t>(blockIdx.x) << a.log2R;
  const T *xb = a.x + static_cast<int64_t>(row0) * a.ldx;
  T acc[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * 1024;
    const int r = e >> lb, j = e & (a.b - 1);
    const T v = xb[static_cast<int64_t>(r) * a.ldx + j];
    tile[e] = v;
    acc[i] = a.diag[row0 + r] * v;
  }
  __syncthreads();
  for (int t = 0; t < a.nflip; ++t) {
    const uint32_t xm = a.flips[t].xmask;
    const uint32_t zm = a.flips[t].zmask;
    const T c = static_cast<T>(a.flips[t].coef);
    const int sh = static_cast<int>(xm) << lb;
    if (zm == 0) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) acc[i] += c * tile[(threadIdx.x + i * 1024) ^ sh];
    } else {
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = threadIdx.x + i * 1024;
        const T sg = (__popc(((row0 + static_cast<uint32_t>(e >> lb)) ^ xm) & zm) & 1) ? -c : c;
        acc[i] += sg * tile[e ^ sh];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * 1024;
    const int64_t r = row0 + (e >> lb);
    const int j = e & (a.b - 1);
    T v = a.alpha * acc[i];
    if (a.u) v += a.beta * a.u[r * a.ldu + j];
    if (a.z) v += a.gamma * a.z[r * a.ldz + j];
    a.y[r * a.ldy + j] = v;
  }
  (void)nel;
}

template <typename T, int ROLE>
hipError_t launch_step_lo_role(const StepArgs<T> &a, hipStream_t s) {
  const int nel = (1 << a.log2R) * a.b;
  const int ept = (nel + 1023) / 1024;
  const size_t lds = static_cast<size_t>(nel) * sizeof(T);
  dim3 grid(a.ntiles), block(1024);
  if (ept <= 1) hipLaunchKernelGGL((k_step_lo<T, 1, ROLE>), grid, block, lds, s, a);
  else if (ept <= 2) hipLaunchKernelGGL((k_step_lo<T, 2, ROLE>), grid, block, lds, s, a);
  else if (ept <= 4) hipLaunchKernelGGL((k_step_lo<T, 4, ROLE>), grid, block, lds, s, a);
  else if (ept <= 8) hipLaunchKernelGGL((k_step_lo<T, 8, ROLE>), grid, block, lds, s, a);
  else if (ept <= 16) hipLaunchKernelGGL((k_step_lo<T, 16, ROLE>), grid, block, lds, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step_lo(const StepArgs<T> &a, hipStream_t s, int role) {
  if (role == 1) return launch_step_lo_role<T, 1>(a, s);
  if (role == 2) return launch_step_lo_role<T, 2>(a, s);
  return launch_step_lo_role<T, 0>(a, s);
}
template hipError_t launch_step_lo<double>(const StepArgs<double> &, hipStream_t, int);
template hipError_t launch_step_lo<float>(const StepArgs<float> &, hipStream_t, int);

// ---------------------------------------------------------------------------
// High-bit pass of the two-pass apply.  1024 threads; element e of the tile is
// (j, w, col) with col fastest, then w, then j (b = 2^lb, W = 2^lw), so the W
// adjacent rows of one j form a contiguous W * b run in memory and in LDS.
// Every flip whose mask lies in the high bits maps j to j ^ (mask >> lo_bits)
// inside the tile, i.e. e to e ^ ((mask >> lo_bits) << (lw + lb)).
// ---------------------------------------------------------------------------
template <typename T, int EPT, int ROLE>
__global__ __launch_bounds__(1024) void k_step_hi(HiArgs<T> a) {
  extern __shared__ unsigned char smem_raw[];
  T *tile = reinterpret_cast<T *>(smem_raw);
  const int lb = __ffs(a.b) - 1;
  const int lw = __ffs(a.W) - 1;
  const uint32_t l0 = static_cast<uint32_t>(blockIdx.x) << lw;
  const uint32_t lomask_w = (1u << lw) - 1u;
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * 1024;
    const uint32_t t = static_cast<uint32_t>(e) >> lb;
    const uint32_t row = l0 + (t & lomask_w) + ((t >> lw) << a.lo_bits);
    tile[e] = a.x[static_cast<int64_t>(row) * a.ldx + (e & (a.b - 1))];
  }
  T acc[EPT];
#pragma unroll
  for (int i = 0; i < EPT; ++i) acc[i] = T(0);
  __syncthreads();
  for (int t = 0; t < a.nhi; ++t) {
    const uint32_t xm = a.flips[t].xmask;
    const uint32_t zm = a.flips[t].zmask;
    const T c = static_cast<T>(a.flips[t].coef);
    const int sh = static_cast<int>(xm >> a.lo_bits) << (lw + lb);
    if (zm == 0) {
#pragma unroll
      for (int i = 0; i < EPT; ++i) acc[i] += c * tile[(threadIdx.x + i * 1024) ^ sh];
    } else {
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int e = threadIdx.x + i * 1024;
        const uint32_t tt = static_cast<uint32_t>(e) >> lb;
        const uint32_t row = l0 + (tt & lomask_w) + ((tt >> lw) << a.lo_bits);
        const T sg = (__popc((row ^ xm) & zm) & 1) ? -c : c;
        acc[i] += sg * tile[e ^ sh];
      }
    }
  }
  for (int t = a.nhi; t < a.nflip; ++t) {  // masks with bits in both halves: gather from global
    const uint32_t xm = a.flips[t].xmask;
    const uint32_t zm = a.flips[t].zmask;
    const T c = static_cast<T>(a.flips[t].coef);
#pragma unroll 4
    for (int i = 0; i < EPT; ++i) {
      const int e = threadIdx.x + i * 1024;
      const uint32_t tt = static_cast<uint32_t>(e) >> lb;
      const uint32_t row = l0 + (tt & lomask_w) + ((tt >> lw) << a.lo_bits);
      const T sg = (__popc((row ^ xm) & zm) & 1) ? -c : c;
      acc[i] += sg * a.x[static_cast<int64_t>(row ^ xm) * a.ldx + (e & (a.b - 1))];
    }
  }
#pragma unroll 8
  for (int i = 0; i < EPT; ++i) {
    const int e = threadIdx.x + i * 1024;
    const uint32_t tt = static_cast<uint32_t>(e) >> lb;
    const int64_t row = l0 + (tt & lomask_w) + ((tt >> lw) << a.lo_bits);
    const int j = e & (a.b - 1);
    const T v = a.y[row * a.ldy + j] + a.alpha * acc[i];
    a.y[row * a.ldy + j] = v;
    if (a.st) a.st[row * a.ldst + j] = static_cast<double>(v);
  }
}

template <typename T, int ROLE>
hipError_t launch_step_hi_role(const HiArgs<T> &a, hipStream_t s) {
  const int nel = (a.W << a.hi_bits) * a.b;
  const int ept = (nel + 1023) / 1024;
  const size_t lds = static_cast<size_t>(nel) * sizeof(T);
  dim3 grid(a.ntiles), block(1024);
  if (ept <= 1) hipLaunchKernelGGL((k_step_hi<T, 1, ROLE>), grid, block, lds, s, a);
  else if (ept <= 2) hipLaunchKernelGGL((k_step_hi<T, 2, ROLE>), grid, block, lds, s, a);
  else if (ept <= 4) hipLaunchKernelGGL((k_step_hi<T, 4, ROLE>), grid, block, lds, s, a);
  else if (ept <= 8) hipLaunchKernelGGL((k_step_hi<T, 8, ROLE>), grid, block, lds, s, a);
  else if (ept <= 16) hipLaunchKernelGGL((k_step_hi<T, 16, ROLE>), grid, block, lds, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step_hi(const HiArgs<T> &a, hipStream_t s, int role) {
  if (role == 1) return launch_step_hi_role<T, 1>(a, s);
  if (role == 2) return launch_step_hi_role<T, 2>(a, s);
  return launch_step_hi_role<T, 0>(a, s);
}
template hipError_t launch_step_hi<double>(const HiArgs<double> &, hipStream_t, int);
template hipError_t launch_step_hi<float>(const HiArgs<float> &, hipStream_t, int);

// ---------------------------------------------------------------------------
// Fused alternating-split recurrence (see RecArgs).  The blocks are moved as
// 16-byte vectors (2 doubles / 4 floats of one row; b * sizeof(T) >= 16), so
// every global access and every LDS read is 16 bytes per lane.  Both kernels
// keep their vectors of T_cur and P in registers, complete T_new from the LDS
// copy of T_cur, then stage T_new in LDS to start the next step.
//   lo kernel: tile = 2^lo_bits consecutive rows (contiguous in memory);
//   hi kernel: tile = rows l0 + w + (j << lo_bits), w < W, j < 2^hi_bits, so each
//              j contributes one contiguous run of W * b elements (W chosen on
//              the host so that a run fills whole 128-byte lines).
// Vector index v inside a tile: v = ((j << lw) | w) << lbv | cv with 2^lbv
// vectors per row; a high flip maps j to j ^ (mask >> lo_bits), i.e. v to
// v ^ ((mask >> lo_bits) << (lw + lbv)); a low flip maps v to v ^ (mask << lbv).
// ---------------------------------------------------------------------------
template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
  typedef double type __attribute__((ext_vector_type(2)));
  static constexpr int n = 2, log2n = 1;
};
template <>
struct Vec16<float> {
  typedef float type __attribute__((ext_vector_type(4)));
  static constexpr int n = 4, log2n = 2;
};

// The flip table is not written while a kernel runs, so it is read through the constant
// address space: uniform scalar loads that do not wait for the kernel's own global stores.
typedef const __attribute__((address_space(4))) FlipEntry *ConstFlips;

// Lane index threadIdx.x as an opaque value: expressions built from it are recomputed where they
// are used instead of being hoisted and kept live across the kernel's phases.
__device__ __forceinline__ uint32_t lane_tid() {
  uint32_t t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// acc += sum_t c_t sign_t tile[v ^ vs_t] for the flips of one split; vs_t is the mask moved to
// the vector index (left shift by `shift`, or right shift by -shift for high masks, whose low
// bits are zero).  Vector i of the thread is v = tid + i NT, so v ^ vs = (tid ^ (vs mod NT)) +
// ((i NT) ^ (vs - vs mod NT)): one per-lane index per flip plus a uniform part per i.
// Sign-free flips come first and run U at a time, so U * NV LDS reads are in flight per wait; the
// accumulation order per element is the table order.  rowf(i) gives the row of vector i (for
// the signs of flips with a z-mask).
template <typename T, int NT, int NV, typename RowF>
__device__ __forceinline__ void rec_flips(typename Vec16<T>::type (&acc)[NV], const typename Vec16<T>::type *tile,
                                          const FlipEntry *flips_g, int nplain, int nflip, int shift, RowF rowf) {
  using V = typename Vec16<T>::type;
  constexpr int U = (NT == 1024 && NV == 4) ? 1 : NV >= 2 ? 2 : 4;
  const ConstFlips flips = (ConstFlips)flips_g;
  auto vshift = [shift](uint32_t xm) { return shift >= 0 ? (xm << shift) : (xm >> -shift); };
  auto at = [&](uint32_t lo, uint32_t hi, int i) -> const V & {
    return tile[lo + ((static_cast<uint32_t>(i) * NT) ^ hi)];
  };
  int t = 0;
  if constexpr (U == 1) {
    // one flip's NV reads per wait; no unrolling, so no second set of loads is kept live
#pragma unroll 1
    for (; t < nplain; ++t) {
      const uint32_t vs = vshift(flips[t].xmask);
      const T c = static_cast<T>(flips[t].coef);
      const uint32_t lo = lane_tid() ^ (vs & (NT - 1)), hi = vs & ~uint32_t(NT - 1);
      V g[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) g[i] = at(lo, hi, i);
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] += c * g[i];
    }
  }
  for (; t + U <= nplain; t += U) {
    uint32_t lo[U], hi[U];
    T c[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const uint32_t vs = vshift(flips[t + q].xmask);
      lo[q] = threadIdx.x ^ (vs & (NT - 1));
      hi[q] = vs & ~uint32_t(NT - 1);
      c[q] = static_cast<T>(flips[t + q].coef);
    }
    V g[U][NV];
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int i = 0; i < NV; ++i) g[q][i] = at(lo[q], hi[q], i);
#pragma unroll
    for (int q = 0; q < U; ++q)
#pragma unroll
      for (int i = 0; i < NV; ++i) acc[i] += c[q] * g[q][i];
  }
  for (; t < nplain; ++t) {
    const uint32_t vs = vshift(flips[t].xmask);
    const T c = static_cast<T>(flips[t].coef);
    const uint32_t lo = threadIdx.x ^ (vs & (NT - 1)), hi = vs & ~uint32_t(NT - 1);
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] += c * at(lo, hi, i);
  }
#pragma unroll 1
  for (; t < nflip; ++t) {
    const uint32_t xm = flips[t].xmask;
    const uint32_t zm = flips[t].zmask;
    const T c = static_cast<T>(flips[t].coef);
    const uint32_t vs = vshift(xm);
    const uint32_t lo = lane_tid() ^ (vs & (NT - 1)), hi = vs & ~uint32_t(NT - 1);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const T sg = (__popc((rowf(i) ^ xm) & zm) & 1) ? -c : c;
      acc[i] += sg * at(lo, hi, i);
    }
  }
}

// Waves per SIMD that let two one-tile workgroups share a CU (1024 threads with up to 4 vectors
// each, or 512 threads with up to 4); other shapes run one workgroup per CU.
constexpr int rec_min_waves(int nt, int nv) { return (nt == 1024 && nv <= 4) ? 8 : (nt == 512 && nv <= 4) ? 4 : 1; }

template <typename T>
__device__ __forceinline__ void store_sample(double *st, int64_t ldst, uint32_t row, uint32_t cv,
                                             const typename Vec16<T>::type &x) {
  double *d = st + static_cast<int64_t>(row) * ldst + (static_cast<int64_t>(cv) << Vec16<T>::log2n);
#pragma unroll
  for (int q = 0; q < Vec16<T>::n; ++q) d[q] = static_cast<double>(x[q]);
}

// Both kernels keep three vector sets per thread (T_cur, the accumulator and one flip's loads in
// flight) and recompute every index from the lane id, so the 1024-thread shape with 4 vectors
// fits 64 VGPRs and two tiles share a CU: one tile's LDS phase then overlaps the other's loads
// and stores.  The partial P is loaded only when the first flip sweep is done, and the low pass
// keeps the tile's diagonal entries in LDS after the vectors (2^lo_bits of them).  Global
// vector i of a thread sits at a uniform base (one per i) plus the lane's 32-bit byte offset.
template <typename V>
__device__ __forceinline__ V *vec_at(V *base, uint32_t vi) {
  return reinterpret_cast<V *>(reinterpret_cast<char *>(base) + (vi << 4));
}
template <typename V>
__device__ __forceinline__ const V *vec_at(const V *base, uint32_t vi) {
  return reinterpret_cast<const V *>(reinterpret_cast<const char *>(base) + (vi << 4));
}

template <typename T, int NT, int NV>
__global__ __launch_bounds__(NT, rec_min_waves(NT, NV)) void k_rec_lo(RecArgs<T> a) {
  using V = typename Vec16<T>::type;
  extern __shared__ unsigned char smem_raw[];
  V *tile = reinterpret_cast<V *>(smem_raw);
  T *dtile = reinterpret_cast<T *>(smem_raw + sizeof(V) * NT * NV);
  const int lbv = (__ffs(a.b) - 1) - Vec16<T>::log2n;  // log2(vectors per row)
  const uint32_t cvmask = (1u << lbv) - 1u;
  int bid = blockIdx.x;
  if (a.xcd_remap) bid = (bid & 7) * (a.ntiles >> 3) + (bid >> 3);
  const uint32_t row0 = static_cast<uint32_t>(bid) << a.lo_bits;
  const uint32_t vbase = row0 << lbv;
  const V *tc = reinterpret_cast<const V *>(a.tcur) + vbase;
  V *tn = reinterpret_cast<V *>(a.tnew) + vbase;
  V *pp = reinterpret_cast<V *>(a.p) + vbase;
  auto rowf = [&](int i) { return row0 + ((lane_tid() + static_cast<uint32_t>(i) * NT) >> lbv); };
  auto dg = [&](int i) { return dtile[(lane_tid() + static_cast<uint32_t>(i) * NT) >> lbv]; };
  V cur[NV], acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) cur[i] = *vec_at(tc + i * NT, lane_tid());
  const uint32_t nrows = 1u << a.lo_bits;
  for (uint32_t r = threadIdx.x; r < nrows; r += NT) dtile[r] = a.diag[row0 + r];
#pragma unroll
  for (int i = 0; i < NV; ++i) tile[threadIdx.x + i * NT] = cur[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = dg(i) * cur[i];
  rec_flips<T, NT, NV>(acc, tile, a.flips, a.nplain, a.nflip, lbv, rowf);
  {
    // all NV loads of P in flight before the first use (no branch between them)
    V p[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) p[i] = *vec_at(pp + i * NT, lane_tid());
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      acc[i] = p[i] + a.a_fin * acc[i];  // T_new
      *vec_at(tn + i * NT, lane_tid()) = acc[i];
    }
  }
  if (a.st) {
#pragma unroll
    for (int i = 0; i < NV; ++i) store_sample<T>(a.st, a.ldst, rowf(i), (lane_tid() + i * NT) & cvmask, acc[i]);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    tile[threadIdx.x + i * NT] = acc[i];
    acc[i] = dg(i) * acc[i];
  }
  __syncthreads();
  rec_flips<T, NT, NV>(acc, tile, a.flips, a.nplain, a.nflip, lbv, rowf);
  if (a.old) {
    const V *od = reinterpret_cast<const V *>(a.old) + vbase;
    V o[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) o[i] = *vec_at(od + i * NT, lane_tid());
#pragma unroll
    for (int i = 0; i < NV; ++i)
      *vec_at(pp + i * NT, lane_tid()) = (a.a_start * acc[i] + a.b_cur * cur[i]) + a.c_old * o[i];
  } else {
#pragma unroll
    for (int i = 0; i < NV; ++i) *vec_at(pp + i * NT, lane_tid()) = a.a_start * acc[i] + a.b_cur * cur[i];
  }
}

// High pass: vector v = tid + i NT of the tile is (j, w, c) = (v >> (lw + lbv), (v >> lbv) & (W - 1),
// v & (2^lbv - 1)) and lives at global vector ((l0 + w + (j << lo_bits)) << lbv) | c.  With
// W 2^lbv dividing NT, vector i sits at the offset of vector 0 plus the uniform
// i (NT >> (lw + lbv)) << (lo_bits + lbv).
template <typename T, int NT, int NV>
__global__ __launch_bounds__(NT, rec_min_waves(NT, NV)) void k_rec_hi(RecArgs<T> a) {
  using V = typename Vec16<T>::type;
  extern __shared__ unsigned char smem_raw[];
  V *tile = reinterpret_cast<V *>(smem_raw);
  const int lbv = (__ffs(a.b) - 1) - Vec16<T>::log2n;
  const int lw = __ffs(a.W) - 1;
  const uint32_t cvmask = (1u << lbv) - 1u;
  const uint32_t wmask = static_cast<uint32_t>(a.W) - 1u;
  int bid = blockIdx.x;
  if (a.xcd_remap) bid = (bid & 7) * (a.ntiles >> 3) + (bid >> 3);
  const uint32_t l0 = static_cast<uint32_t>(bid) << lw;
  const uint32_t istep = static_cast<uint32_t>(NT >> (lw + lbv)) << (a.lo_bits + lbv);
  const V *tc = reinterpret_cast<const V *>(a.tcur);
  V *tn = reinterpret_cast<V *>(a.tnew);
  V *pp = reinterpret_cast<V *>(a.p);
  auto rowf = [&](int i) {
    const uint32_t rv = (lane_tid() + static_cast<uint32_t>(i) * NT) >> lbv;
    return l0 + (rv & wmask) + ((rv >> lw) << a.lo_bits);
  };
  // global vector offset of the lane's vector 0
  auto off0 = [&]() {
    const uint32_t t = lane_tid();
    const uint32_t rv = t >> lbv;
    return ((l0 + (rv & wmask) + ((rv >> lw) << a.lo_bits)) << lbv) | (t & cvmask);
  };
  V cur[NV], acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) cur[i] = *vec_at(tc + i * istep, off0());
#pragma unroll
  for (int i = 0; i < NV; ++i) tile[threadIdx.x + i * NT] = cur[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = V(T(0));
  // high masks act on j: shift right by lo_bits, then left by lw + lbv
  const int hs = lw + lbv - a.lo_bits;
  rec_flips<T, NT, NV>(acc, tile, a.flips, a.nplain, a.nflip, hs, rowf);
  {
    V p[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) p[i] = *vec_at(pp + i * istep, off0());
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      acc[i] = p[i] + a.a_fin * acc[i];  // T_new
      *vec_at(tn + i * istep, off0()) = acc[i];
    }
  }
  if (a.st) {
#pragma unroll
    for (int i = 0; i < NV; ++i) store_sample<T>(a.st, a.ldst, rowf(i), lane_tid() & cvmask, acc[i]);
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) tile[threadIdx.x + i * NT] = acc[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = V(T(0));
  rec_flips<T, NT, NV>(acc, tile, a.flips, a.nplain, a.nflip, hs, rowf);
  if (a.old) {
    V o[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) o[i] = *vec_at(reinterpret_cast<const V *>(a.old) + i * istep, off0());
#pragma unroll
    for (int i = 0; i < NV; ++i)
      *vec_at(pp + i * istep, off0()) = (a.a_start * acc[i] + a.b_cur * cur[i]) + a.c_old * o[i];
  } else {
#pragma unroll
    for (int i = 0; i < NV; ++i) *vec_at(pp + i * istep, off0()) = a.a_start * acc[i] + a.b_cur * cur[i];
  }
}

// Persistent variants: gridDim.x workgroups walk the tiles t = blockIdx.x + k gridDim.x and
// load tile t + gridDim.x into registers while tile t is in the LDS phase, so a CU keeps its
// memory pipe busy across the flip loops.
template <typename T, int NT, int NV>
__global__ __launch_bounds__(NT) void k_rec_lo_p(RecArgs<T> a) {
  using V = typename Vec16<T>::type;
  extern __shared__ unsigned char smem_raw[];
  V *tile = reinterpret_cast<V *>(smem_raw);
  const int lbv = (__ffs(a.b) - 1) - Vec16<T>::log2n;
  const uint32_t cvmask = (1u << lbv) - 1u;
  const int G = gridDim.x;
  int t = blockIdx.x;
  V cn[NV], pn[NV];
  T dn[NV];
  auto fetch = [&](int tt) {
    const uint32_t r0 = static_cast<uint32_t>(tt) << a.lo_bits;
    const uint32_t vb = r0 << lbv;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const uint32_t v = threadIdx.x + i * NT;
      cn[i] = reinterpret_cast<const V *>(a.tcur)[vb + v];
      pn[i] = reinterpret_cast<const V *>(a.p)[vb + v];
      dn[i] = a.diag[r0 + (v >> lbv)];
    }
  };
  if (t < a.ntiles) fetch(t);
  for (; t < a.ntiles; t += G) {
    const uint32_t row0 = static_cast<uint32_t>(t) << a.lo_bits;
    const uint32_t vbase = row0 << lbv;
    V cur[NV], nw[NV], acc[NV];
    T dg[NV];
    uint32_t row[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      cur[i] = cn[i];
      nw[i] = pn[i];
      dg[i] = dn[i];
      row[i] = row0 + ((threadIdx.x + i * NT) >> lbv);
    }
    if (t + G < a.ntiles) fetch(t + G);
#pragma unroll
    for (int i = 0; i < NV; ++i) tile[threadIdx.x + i * NT] = cur[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = dg[i] * cur[i];
    rec_flips<T, NT, NV>(acc, tile, a.flips, a.nplain, a.nflip, lbv, [&](int i) { return row[i]; });
    V *tn = reinterpret_cast<V *>(a.tnew) + vbase;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const uint32_t v = threadIdx.x + i * NT;
      nw[i] += a.a_fin * acc[i];
      tn[v] = nw[i];
      if (a.st) store_sample<T>(a.st, a.ldst, row[i], v & cvmask, nw[i]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) tile[threadIdx.x + i * NT] = nw[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = dg[i] * nw[i];
    rec_flips<T, NT, NV>(acc, tile, a.flips, a.nplain, a.nflip, lbv, [&](int i) { return row[i]; });
    V *pp = reinterpret_cast<V *>(a.p) + vbase;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      V o = V(T(0));
      if (a.old) o = reinterpret_cast<const V *>(a.old)[vbase + threadIdx.x + i * NT];
      pp[threadIdx.x + i * NT] =
          a.old ? (a.a_start * acc[i] + a.b_cur * cur[i]) + a.c_old * o : a.a_start * acc[i] + a.b_cur * cur[i];
    }
    __syncthreads();  // the next tile overwrites the LDS copy
  }
}

template <typename T, int NT, int NV>
__global__ __launch_bounds__(NT) void k_rec_hi_p(RecArgs<T> a) {
  using V = typename Vec16<T>::type;
  extern __shared__ unsigned char smem_raw[];
  V *tile = reinterpret_cast<V *>(smem_raw);
  const int lbv = (__ffs(a.b) - 1) - Vec16<T>::log2n;
  const int lw = __ffs(a.W) - 1;
  const uint32_t cvmask = (1u << lbv) - 1u;
  const uint32_t wmask = static_cast<uint32_t>(a.W) - 1u;
  const int hs = lw + lbv - a.lo_bits;
  const int G = gridDim.x;
  int t = blockIdx.x;
  // element offsets relative to the tile's first row l0 = t W (row = l0 + rel)
  uint32_t rel[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const uint32_t v = threadIdx.x + i * NT;
    const uint32_t rv = v >> lbv;
    rel[i] = (rv & wmask) + ((rv >> lw) << a.lo_bits);
  }
  V cn[NV], pn[NV];
  auto fetch = [&](int tt) {
    const uint32_t l0 = static_cast<uint32_t>(tt) << lw;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const uint32_t off = ((l0 + rel[i]) << lbv) | ((threadIdx.x + i * NT) & cvmask);
      cn[i] = reinterpret_cast<const V *>(a.tcur)[off];
      pn[i] = reinterpret_cast<const V *>(a.p)[off];
    }
  };
  if (t < a.ntiles) fetch(t);
  for (; t < a.ntiles; t += G) {
    const uint32_t l0 = static_cast<uint32_t>(t) << lw;
    V cur[NV], nw[NV], acc[NV];
    uint32_t row[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      cur[i] = cn[i];
      nw[i] = pn[i];
      row[i] = l0 + rel[i];
    }
    if (t + G < a.ntiles) fetch(t + G);
#pragma unroll
    for (int i = 0; i < NV; ++i) tile[threadIdx.x + i * NT] = cur[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = V(T(0));
    rec_flips<T, NT, NV>(acc, tile, a.flips, a.nplain, a.nflip, hs, [&](int i) { return row[i]; });
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const uint32_t cv = (threadIdx.x + i * NT) & cvmask;
      nw[i] += a.a_fin * acc[i];
      reinterpret_cast<V *>(a.tnew)[(row[i] << lbv) | cv] = nw[i];
      if (a.st) store_sample<T>(a.st, a.ldst, row[i], cv, nw[i]);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) tile[threadIdx.x + i * NT] = nw[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) acc[i] = V(T(0));
    rec_flips<T, NT, NV>(acc, tile, a.flips, a.nplain, a.nflip, hs, [&](int i) { return row[i]; });
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const uint32_t cv = (threadIdx.x + i * NT) & cvmask;
      const uint32_t gv = (row[i] << lbv) | cv;
      V o = V(T(0));
      if (a.old) o = reinterpret_cast<const V *>(a.old)[gv];
      reinterpret_cast<V *>(a.p)[gv] =
          a.old ? (a.a_start * acc[i] + a.b_cur * cur[i]) + a.c_old * o : a.a_start * acc[i] + a.b_cur * cur[i];
    }
    __syncthreads();
  }
}

// Dynamic LDS above the 64 KiB default must be allowed per kernel; done once per instantiation
// (function-local statics are initialised once, also under concurrent first calls).
template <typename T, int NT, int NV>
hipError_t rec_lo_allow_lds() {
  static const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_rec_lo<T, NT, NV>),
                                                  hipFuncAttributeMaxDynamicSharedMemorySize,
                                                  static_cast<int>(NT * NV * 16 + 8192 * sizeof(T)));
  return e;
}

template <typename T, int NT>
hipError_t launch_rec_nt(const RecArgs<T> &a, int nvec, bool hi, hipStream_t s) {
  // low pass: the vectors, then the tile's 2^lo_bits diagonal entries
  const size_t rows_lo = size_t(1) << a.lo_bits;
  const size_t lds_vec = static_cast<size_t>(nvec) * 16;  // persistent forms: vectors only
  const size_t lds = lds_vec + (hi ? 0 : rows_lo * sizeof(T));
  if (!hi && rows_lo > 8192) return hipErrorInvalidValue;
  // (the 1024-thread persistent form with 4 vectors per thread would spill: launch one tile per workgroup)
  const bool persist = a.grid > 0 && a.grid < a.ntiles && !(NT == 1024 && nvec / NT == 4);
  dim3 grid(persist ? a.grid : a.ntiles), block(NT);
#define DACP_REC(nv_)                                                                  \
  do {                                                                                 \
    if (persist) {                                                                     \
      if (hi) hipLaunchKernelGGL((k_rec_hi_p<T, NT, nv_>), grid, block, lds_vec, s, a); \
      else hipLaunchKernelGGL((k_rec_lo_p<T, NT, nv_>), grid, block, lds_vec, s, a);    \
    } else {                                                                           \
      if (hi) {                                                                        \
        hipLaunchKernelGGL((k_rec_hi<T, NT, nv_>), grid, block, lds, s, a);           \
      } else {                                                                         \
        const hipError_t e = rec_lo_allow_lds<T, NT, nv_>();                           \
        if (e != hipSuccess) return e;                                                 \
        hipLaunchKernelGGL((k_rec_lo<T, NT, nv_>), grid, block, lds, s, a);           \
      }                                                                                \
    }                                                                                  \
  } while (0)
  switch (nvec / NT) {
    case 1: DACP_REC(1); break;
    case 2: DACP_REC(2); break;
    case 4: DACP_REC(4); break;
    default: return hipErrorInvalidValue;
  }
#undef DACP_REC
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rec(const RecArgs<T> &a, bool hi, hipStream_t s) {
  const int64_t rows = hi ? (static_cast<int64_t>(a.W) << a.hi_bits) : (int64_t(1) << a.lo_bits);
  const int64_t nel = rows * a.b;
  if ((a.b * static_cast<int>(sizeof(T))) % 16 != 0 || nel * static_cast<int64_t>(sizeof(T)) > 65536)
    return hipErrorInvalidValue;
  const int nvec = static_cast<int>(nel * sizeof(T) / 16);
  // 32-bit byte offsets over the whole block (high pass), and W rows of vectors dividing the
  // thread count (the high pass steps its vectors by a uniform offset)
  const int64_t D = int64_t(1) << (a.lo_bits + a.hi_bits);
  if (D * a.b * static_cast<int64_t>(sizeof(T)) >= (int64_t(1) << 32)) return hipErrorInvalidValue;
  if (hi && static_cast<int64_t>(a.W) * (a.b * static_cast<int64_t>(sizeof(T)) / 16) > a.threads)
    return hipErrorInvalidValue;
  if (a.threads == 512 && nvec % 512 == 0) return launch_rec_nt<T, 512>(a, nvec, hi, s);
  if (a.threads == 1024 && nvec % 1024 == 0) return launch_rec_nt<T, 1024>(a, nvec, hi, s);
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t launch_rec_lo(const RecArgs<T> &a, hipStream_t s) {
  return launch_rec<T>(a, false, s);
}
template <typename T>
hipError_t launch_rec_hi(const RecArgs<T> &a, hipStream_t s) {
  return launch_rec<T>(a, true, s);
}
template hipError_t launch_rec_lo<double>(const RecArgs<double> &, hipStream_t);
template hipError_t launch_rec_lo<float>(const RecArgs<float> &, hipStream_t);
template hipError_t launch_rec_hi<double>(const RecArgs<double> &, hipStream_t);
template hipError_t launch_rec_hi<float>(const RecArgs<float> &, hipStream_t);

// ---------------------------------------------------------------------------
// Diagonal table d(s) = sum_t c_t (-1)^popcount(s & z_t)  (x-mask-free terms).
// ---------------------------------------------------------------------------
__global__ void k_diag(const uint32_t *zm, const double *c, int nterm, int64_t D, double *d64, float *d32) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= D) return;
  double acc = 0.0;
  for (int t = 0; t < nterm; ++t) {
    const double ct = c[t];
    acc += (__popc(static_cast<uint32_t>(s) & zm[t]) & 1) ? -ct : ct;
  }
  d64[s] = acc;
  d32[s] = static_cast<float>(acc);
}

hipError_t launch_diag(const uint32_t *zm, const double *c, int nterm, int64_t D, double *d64, float *d32,
                       hipStream_t s) {
  const int threads = 256;
  const int64_t blocks = (D + threads - 1) / threads;
  hipLaunchKernelGGL(k_diag, dim3(blocks), dim3(threads), 0, s, zm, c, nterm, D, d64, d32);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Column reductions (fixed order, so results are reproducible run to run).
// ---------------------------------------------------------------------------
int coldots_blocks(int64_t D, int b) {
  int64_t nb = (D * static_cast<int64_t>(b)) / 16384;
  if (nb < 1) nb = 1;
  if (nb > 1024) nb = 1024;
  if (nb > D) nb = D;
  return static_cast<int>(nb);
}

template <typename T>
__global__ __launch_bounds__(256) void k_coldots(const T *x, int64_t ldx, const T *y, int64_t ldy, int64_t D, int b,
                                                 double *partial) {
  __shared__ double sm[256];
  const int cpt = b < 256 ? b : 256;
  const int rstride = 256 / cpt;
  const int tid = threadIdx.x;
  const int j0 = tid % cpt;
  const int r0 = tid / cpt;
  const int64_t rows_per = (D + gridDim.x - 1) / gridDim.x;
  const int64_t rbeg = static_cast<int64_t>(blockIdx.x) * rows_per;
  int64_t rend = rbeg + rows_per;
  if (rend > D) rend = D;
  for (int jc = 0; jc < b; jc += cpt) {
    const int j = jc + j0;
    double acc = 0.0;
    if (r0 < rstride && j < b)
      for (int64_t r = rbeg + r0; r < rend; r += rstride)
        acc += static_cast<double>(x[r * ldx + j]) * static_cast<double>(y[r * ldy + j]);
    sm[tid] = acc;
    __syncthreads();
    if (r0 == 0 && j < b) {
      double s = 0.0;
      for (int q = 0; q < rstride; ++q) s += sm[q * cpt + j0];
      partial[static_cast<int64_t>(blockIdx.x) * b + j] = s;
    }
    __syncthreads();
  }
}

__global__ void k_reduce_partials(const double *partial, int nblk, int w, double *out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= w) return;
  double s = 0.0;
  for (int q = 0; q < nblk; ++q) s += partial[static_cast<int64_t>(q) * w + j];
  out[j] = s;
}

hipError_t launch_coldots(const void *x, int64_t ldx, const void *y, int64_t ldy, int dtype, int64_t D, int b,
                          double *partial, int nblk, double *out, hipStream_t s) {
  if (dtype == DACP_F64)
    hipLaunchKernelGGL((k_coldots<double>), dim3(nblk), dim3(256), 0, s, static_cast<const double *>(x), ldx,
                       static_cast<const double *>(y), ldy, D, b, partial);
  else
    hipLaunchKernelGGL((k_coldots<float>), dim3(nblk), dim3(256), 0, s, static_cast<const float *>(x), ldx,
                       static_cast<const float *>(y), ldy, D, b, partial);
  hipLaunchKernelGGL(k_reduce_partials, dim3((b + 255) / 256), dim3(256), 0, s, partial, nblk, b, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_resid(const double *x, const double *hx, int64_t ld, const double *theta,
                                               int64_t D, int b, double *partial) {
  __shared__ double sm[3][256];
  const int cpt = b < 256 ? b : 256;
  const int rstride = 256 / cpt;
  const int tid = threadIdx.x;
  const int j0 = tid % cpt;
  const int r0 = tid / cpt;
  const int64_t rows_per = (D + gridDim.x - 1) / gridDim.x;
  const int64_t rbeg = static_cast<int64_t>(blockIdx.x) * rows_per;
  int64_t rend = rbeg + rows_per;
  if (rend > D) rend = D;
  for (int jc = 0; jc < b; jc += cpt) {
    const int j = jc + j0;
    double ar = 0.0, ax = 0.0, axr = 0.0;
    if (r0 < rstride && j < b) {
      const double th = theta[j];
      for (int64_t r = rbeg + r0; r < rend; r += rstride) {
        const double xv = x[r * ld + j];
        const double rv = hx[r * ld + j] - th * xv;
        ar += rv * rv;
        ax += xv * xv;
        axr += xv * rv;
      }
    }
    sm[0][tid] = ar;
    sm[1][tid] = ax;
    sm[2][tid] = axr;
    __syncthreads();
    if (r0 == 0 && j < b) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int q = 0; q < rstride; ++q) {
        s0 += sm[0][q * cpt + j0];
        s1 += sm[1][q * cpt + j0];
        s2 += sm[2][q * cpt + j0];
      }
      double *o = partial + static_cast<int64_t>(blockIdx.x) * 3 * b + 3 * j;
      o[0] = s0;
      o[1] = s1;
      o[2] = s2;
    }
    __syncthreads();
  }
}

hipError_t launch_resid(const double *x, const double *hx, int64_t ld, const double *theta, int64_t D, int b,
                        double *partial, int nblk, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_resid, dim3(nblk), dim3(256), 0, s, x, hx, ld, theta, D, b, partial);
  hipLaunchKernelGGL(k_reduce_partials, dim3((3 * b + 255) / 256), dim3(256), 0, s, partial, nblk, 3 * b, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Moment mode (App. C, Eq. shift).
// ---------------------------------------------------------------------------
// Tall Gram block X^T Y of X (D x bx, row stride ldx) and Y (D x gy, stride ldy): each workgroup
// sums a range of rows into partial[blk][i gy + j]; rows are staged 32 at a time through LDS with
// coalesced loads, and each thread accumulates its (i, j) pairs over them in row order.
constexpr int kGramRows = 32;
__global__ __launch_bounds__(256) void k_tall_gram(const double *X, int64_t ldx, int bx, const double *Y, int64_t ldy,
                                                   int gy, int64_t D, double *partial) {
  extern __shared__ double gsm[];
  double *xs = gsm;                    // kGramRows x bx
  double *ys = gsm + kGramRows * bx;   // kGramRows x gy
  const int npair = bx * gy;
  const int64_t rows_per = (D + gridDim.x - 1) / gridDim.x;
  const int64_t rbeg = static_cast<int64_t>(blockIdx.x) * rows_per;
  const int64_t rend = rbeg + rows_per < D ? rbeg + rows_per : D;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // pairs tid, tid + 256, ... (npair <= 1024)
  for (int64_t r0 = rbeg; r0 < rend; r0 += kGramRows) {
    const int nr = static_cast<int>(rend - r0 < kGramRows ? rend - r0 : kGramRows);
    for (int e = threadIdx.x; e < nr * bx; e += 256) {
      const int rr = e / bx, c = e - rr * bx;
      xs[e] = X[(r0 + rr) * ldx + c];
    }
    for (int e = threadIdx.x; e < nr * gy; e += 256) {
      const int rr = e / gy, c = e - rr * gy;
      ys[e] = Y[(r0 + rr) * ldy + c];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int pr = threadIdx.x + q * 256;
      if (pr < npair) {
        const int i = pr / gy, j = pr - (pr / gy) * gy;
        double a = acc[q];
        for (int rr = 0; rr < nr; ++rr) a += xs[rr * bx + i] * ys[rr * gy + j];
        acc[q] = a;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int pr = threadIdx.x + q * 256;
    if (pr < npair) partial[static_cast<int64_t>(blockIdx.x) * npair + pr] = acc[q];
  }
}

int tall_gram_blocks(int64_t D) {
  int64_t nb = D / 1024;
  if (nb < 1) nb = 1;
  if (nb > 1024) nb = 1024;
  return static_cast<int>(nb);
}

hipError_t launch_tall_gram(const double *X, int64_t ldx, int bx, const double *Y, int64_t ldy, int gy, int64_t D,
                            double *partial, int nblk, double *out, hipStream_t s) {
  if (bx < 1 || gy < 1 || bx * gy > 1024) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * kGramRows * (bx + gy);
  hipLaunchKernelGGL(k_tall_gram, dim3(nblk), dim3(256), lds, s, X, ldx, bx, Y, ldy, gy, D, partial);
  hipLaunchKernelGGL(k_reduce_partials, dim3((bx * gy + 255) / 256), dim3(256), 0, s, partial, nblk, bx * gy, out);
  return hipGetLastError();
}

// Moments from the anchors' Gram products (see anchor_projection): thread (part, i, j) walks the
// derivation rules in order; rule c takes block (part na + ai, q) of the Gram product G (row-major,
// row stride m) scaled by scale[part], and gives M_c[i][j] = s G[.][.] (other < 0) or
// 2 s G[.][.] - M_other[i][j].  A thread reads only the entries it wrote itself.  bad is set to 1
// when a moment is not finite.
__global__ void k_moment_chain(const double *G, int64_t m, int b, int na, const int *rules, int nrules, double scale0,
                               double scale1, double *M, int *bad) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int bb = b * b;
  if (t >= 2 * bb) return;
  const int part = t / bb, i = (t - part * bb) / b, j = t - part * bb - i * b;
  const double sc = part == 0 ? scale0 : scale1;
  double *Mp = M + static_cast<int64_t>(part) * nrules * bb;
  bool finite = true;
  for (int c = 0; c < nrules; ++c) {
    const int ai = rules[3 * c], q = rules[3 * c + 1], o = rules[3 * c + 2];
    const double g = sc * G[static_cast<int64_t>((part * na + ai) * b + i) * m + static_cast<int64_t>(q) * b + j];
    const double v = o < 0 ? g : 2.0 * g - Mp[static_cast<int64_t>(o) * bb + i * b + j];
    Mp[static_cast<int64_t>(c) * bb + i * b + j] = v;
    finite = finite && isfinite(v);
  }
  if (!finite) *bad = 1;
}

hipError_t launch_moment_chain(const double *G, int64_t m, int b, int na, const int *rules, int nrules, double scale0,
                               double scale1, double *M, int *bad, hipStream_t s) {
  const int n = 2 * b * b;
  hipLaunchKernelGGL(k_moment_chain, dim3((n + 255) / 256), dim3(256), 0, s, G, m, b, na, rules, nrules, scale0,
                     scale1, M, bad);
  return hipGetLastError();
}

// out block (p, q) = scale (M_{x+y} + M_{|x-y|}) / 2, x, y the orders of panels p, q, M_k the b x b
// moment in slot idx_of[k] of mu (the product identity T_x T_y = (T_{x+y} + T_{|x-y|}) / 2).
__global__ void k_gram_assemble(const double *mu, const int *idx_of, const int64_t *orders, int b, int m, double scale,
                                double *out, int64_t ld) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= static_cast<int64_t>(m) * m) return;
  const int row = static_cast<int>(e / m), col = static_cast<int>(e - static_cast<int64_t>(row) * m);
  const int p = row / b, i = row - p * b, q = col / b, j = col - q * b;
  const int64_t x = orders[p], y = orders[q];
  const int64_t d = x >= y ? x - y : y - x;
  const double ms = mu[static_cast<int64_t>(idx_of[x + y]) * b * b + i * b + j];
  const double md = mu[static_cast<int64_t>(idx_of[d]) * b * b + i * b + j];
  out[row * ld + col] = 0.5 * scale * (ms + md);
}

hipError_t launch_gram_assemble(const double *mu, const int *idx_of, const int64_t *orders, int b, int npan,
                                double scale, double *out, int64_t ld, hipStream_t s) {
  const int m = b * npan;
  const int64_t n = static_cast<int64_t>(m) * m;
  hipLaunchKernelGGL(k_gram_assemble, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, mu, idx_of,
                     orders, b, m, scale, out, ld);
  return hipGetLastError();
}

// dst[r][c] = src[r][cols[c]] * scale[c] (scale may be null).
__global__ void k_gather_cols(const double *src, int64_t lds, const int *cols, const double *scale, int64_t D, int w,
                              double *dst, int64_t ldd) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= D * w) return;
  const int64_t r = e / w;
  const int c = static_cast<int>(e - r * w);
  const double v = src[r * lds + cols[c]];
  dst[r * ldd + c] = scale ? v * scale[c] : v;
}

hipError_t launch_gather_cols(const double *src, int64_t lds, const int *cols, const double *scale, int64_t D, int w,
                              double *dst, int64_t ldd, hipStream_t s) {
  const int64_t n = D * w;
  hipLaunchKernelGGL(k_gather_cols, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, src, lds, cols,
                     scale, D, w, dst, ldd);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Element-wise helpers on [D][b] blocks.
// ---------------------------------------------------------------------------
__global__ void k_colscale(double *x, int64_t ldx, int64_t D, int b, const double *sq) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= D * b) return;
  const int64_t r = e / b;
  const int j = static_cast<int>(e - r * b);
  x[r * ldx + j] *= 1.0 / sqrt(sq[j]);
}

hipError_t launch_colscale(double *x, int64_t ldx, int64_t D, int b, const double *sq_norms, hipStream_t s) {
  const int64_t n = D * b;
  hipLaunchKernelGGL(k_colscale, dim3((n + 255) / 256), dim3(256), 0, s, x, ldx, D, b, sq_norms);
  return hipGetLastError();
}

template <typename S, typename Dt>
__global__ void k_copy_cols(const S *x, int64_t ldx, Dt *y, int64_t ldy, int64_t D, int b) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= D * b) return;
  const int64_t r = e / b;
  const int j = static_cast<int>(e - r * b);
  y[r * ldy + j] = static_cast<Dt>(x[r * ldx + j]);
}

hipError_t launch_copy_cols(const double *x, int64_t ldx, double *y, int64_t ldy, int64_t D, int b, hipStream_t s) {
  const int64_t n = D * b;
  hipLaunchKernelGGL((k_copy_cols<double, double>), dim3((n + 255) / 256), dim3(256), 0, s, x, ldx, y, ldy, D, b);
  return hipGetLastError();
}
hipError_t launch_convert_f64_to_f32(const double *x, int64_t ldx, float *y, int64_t ldy, int64_t D, int b,
                                     hipStream_t s) {
  const int64_t n = D * b;
  hipLaunchKernelGGL((k_copy_cols<double, float>), dim3((n + 255) / 256), dim3(256), 0, s, x, ldx, y, ldy, D, b);
  return hipGetLastError();
}
hipError_t launch_convert_f32_to_f64(const float *x, int64_t ldx, double *y, int64_t ldy, int64_t D, int b,
                                     hipStream_t s) {
  const int64_t n = D * b;
  hipLaunchKernelGGL((k_copy_cols<float, double>), dim3((n + 255) / 256), dim3(256), 0, s, x, ldx, y, ldy, D, b);
  return hipGetLastError();
}

__global__ void k_axpby(double *y, const double *x, double a, double bcoef, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + bcoef * y[i];
}

hipError_t launch_axpby(double *y, const double *x, double a, double bcoef, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3((n + 255) / 256), dim3(256), 0, s, y, x, a, bcoef, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Start states: Philox4x32-10 (Salmon et al., SC'11) + Box-Muller.
// ---------------------------------------------------------------------------
__device__ inline void philox_round(uint32_t &c0, uint32_t &c1, uint32_t &c2, uint32_t &c3, uint32_t k0,
                                    uint32_t k1) {
  const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
  const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
  const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
  const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
  const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
  c0 = n0;
  c1 = lo1;
  c2 = n2;
  c3 = lo0;
}

__global__ void k_philox_gauss(double *out, int64_t D, int b, uint32_t k0, uint32_t k1) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= D * b) return;
  const int64_t s = e / b;
  const int j = static_cast<int>(e - s * b);
  uint32_t c0 = static_cast<uint32_t>(s), c1 = static_cast<uint32_t>(j), c2 = 0, c3 = 0;
  uint32_t kk0 = k0, kk1 = k1;
  for (int r = 0; r < 10; ++r) {
    if (r) {
      kk0 += 0x9E3779B9u;
      kk1 += 0xBB67AE85u;
    }
    philox_round(c0, c1, c2, c3, kk0, kk1);
  }
  const uint64_t a = (static_cast<uint64_t>(c0) << 32) | c1;
  const uint64_t c = (static_cast<uint64_t>(c2) << 32) | c3;
  const double u1 = (static_cast<double>(a >> 11) + 0.5) * 0x1.0p-53;
  const double u2 = (static_cast<double>(c >> 11) + 0.5) * 0x1.0p-53;
  out[e] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925286766559 * u2);
}

// Projects the columns of a [D][b] block onto the eigenspaces of the global spin flip
// P = prod_i sigma^x_i, (P psi)(s) = psi(s ^ (D - 1)): columns j < b_even become psi + P psi, the
// others psi - P psi.  One thread per pair (s, s ^ (D - 1)), s < D / 2, and column.
__global__ void k_parity_split(double *psi, int64_t D, int b, int b_even) {
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (e >= (D / 2) * b) return;
  const int64_t s = e / b;
  const int j = static_cast<int>(e - s * b);
  const int64_t p = s ^ (D - 1);
  const double x = psi[s * b + j], y = psi[p * b + j];
  if (j < b_even) {
    psi[s * b + j] = x + y;
    psi[p * b + j] = x + y;
  } else {
    psi[s * b + j] = x - y;
    psi[p * b + j] = y - x;
  }
}

hipError_t launch_parity_split(double *psi, int64_t D, int b, int b_even, hipStream_t s) {
  if (D < 2 || b < 1 || b_even < 0 || b_even > b) return hipErrorInvalidValue;
  const int64_t n = (D / 2) * b;
  hipLaunchKernelGGL(k_parity_split, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, psi, D, b, b_even);
  return hipGetLastError();
}

hipError_t launch_philox_gauss(double *out, int64_t D, int b, uint64_t seed, hipStream_t s) {
  const int64_t n = D * b;
  hipLaunchKernelGGL(k_philox_gauss, dim3((n + 255) / 256), dim3(256), 0, s, out, D, b,
                     static_cast<uint32_t>(seed & 0xFFFFFFFFu), static_cast<uint32_t>(seed >> 32));
  return hipGetLastError();
}

}  // namespace dacp
