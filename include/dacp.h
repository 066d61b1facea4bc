/*
 * dacp.h -- C ABI of the MI355X (gfx950) DACP central-eigenvalue library.
 *
 * DACP (dual application of Chebyshev polynomial, Guan & Zhang): given the
 * couplings of a spin-1/2 Hamiltonian made of one- and two-body Pauli terms
 * and a count N, return the N eigenvalues nearest the band centre E = 0
 * (problem statement: Sec. II opening and Sec. III).  The path is
 *   bound + window  ->  exp-semicircle filter (Sec. II.A)
 *   ->  Chebyshev evolution basis (Sec. II.B, App. B)
 *   ->  projection S, P (Sec. II.C, Eq. gep)
 *   ->  subspace diagonalisation (App. C)  ->  residual acceptance (Sec. II.C).
 *
 * Conventions for every entry point:
 *   - Every call returns dacp_status (0 = OK, < 0 = error); no exception
 *     crosses the ABI.  dacp_last_error(ctx) gives a message for the last
 *     failure on that context.
 *   - "device" pointers are HIP device memory on the context's device; "host"
 *     pointers are ordinary host memory.  The caller owns every buffer it
 *     passes; handles (dacp_ctx, dacp_ham) are owned by the library and freed
 *     by dacp_destroy / dacp_free_hamiltonian.
 *   - Device work is enqueued on the context's stream.  A call that returns
 *     host data synchronises that stream before returning; a call that only
 *     writes device outputs may return before the work completes.
 *   - On error the outputs are unspecified unless stated otherwise.
 *   - A context is not thread-safe: use one context per host thread.
 *   - Basis convention: bit i of a state index s is spin i,
 *     sigma^z |b> = (1 - 2b) |b>.  D = 2^L.
 *   - Blocks of b states are stored row-major [D][b] with a row stride ld >= b
 *     (element (s, j) at base[s * ld + j]); all matrices are row-major.
 */
#ifndef DACP_H
#define DACP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DACP_OK = 0,
  DACP_E_INVALID = -1,     /* bad argument (message says which)                        */
  DACP_E_NOMEM = -2,       /* device or host allocation failed                         */
  DACP_E_HIP = -3,         /* a HIP runtime call failed                                */
  DACP_E_BOUNDS = -4,      /* spectral bound below ||H|| detected (|T_k(G)| grew > 1)  */
  DACP_E_WINDOW = -5,      /* fewer than N eigenvalues accepted in the window          */
  DACP_E_NUMERIC = -6,     /* NaN/Inf, or the overlap matrix S lost all rank           */
  DACP_E_CONVERGENCE = -7  /* the dense eigensolver did not converge                   */
} dacp_status;

typedef enum { DACP_F64 = 0, DACP_F32 = 1 } dacp_dtype;

/* Pauli operator codes for dacp_term.op_a / op_b. */
enum { DACP_I = 0, DACP_X = 1, DACP_Y = 2, DACP_Z = 3 };

/* One real term c * sigma^{op_a}_{site_a} sigma^{op_b}_{site_b} (Sec. III: each
 * Pauli operator or product of two is one function on states).  op_b = DACP_I
 * for a one-body term (site_b ignored).  A term with an odd number of Y
 * factors is imaginary and rejected.  16 bytes. */
typedef struct {
  uint8_t op_a, op_b;
  uint16_t site_a, site_b;
  uint16_t reserved; /* must be 0 */
  double coeff;
} dacp_term;

typedef struct dacp_ctx_s *dacp_ctx;
typedef struct dacp_ham_s *dacp_ham;

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device`.  `hip_stream` is a hipStream_t
 * (may be NULL for the null stream); it is not owned by the library. */
dacp_status dacp_create(int device, void *hip_stream, dacp_ctx *out);
void dacp_destroy(dacp_ctx ctx);
const char *dacp_last_error(dacp_ctx ctx);
/* Replace the stream used by later calls on `ctx`. */
dacp_status dacp_set_stream(dacp_ctx ctx, void *hip_stream);
/* Tile size (elements of the [rows][b] slab one workgroup stages in LDS) of
 * the apply / recurrence kernel: a power of two in [256, 8192], default 1024.
 * Chosen by the autotuner.  For Hamiltonians whose off-diagonal Pauli strings
 * flip one spin each, results are bit-identical for every tile size; with
 * multi-spin flips the term summation order, hence the rounding, may differ. */
dacp_status dacp_set_tile(dacp_ctx ctx, int tile_elems);
/* Set a tuning knob of the recurrence kernels (the autotuner's interface):
 *   "tile"        single-pass apply tile, elements (same as dacp_set_tile)
 *   "pass_tile"   tile of the two-pass apply kernels, elements,
 *                 power of two in [512, 16384] (default 4096)
 *   "two_pass_L"  smallest L using the two-pass kernels (0 disables; default 15)
 *   "fused"       1 = alternating-split fused recurrence in the evolution (default), 0 = off
 *   "rec_tile"    largest tile of the fused recurrence kernels, elements (power of two in
 *                 [1024, 8192], default 8192)
 *   "rec_hi_w"    fused recurrence: adjacent rows per high-bit tile (0 = automatic: enough
 *                 for 128-byte runs; else 1, 2, 4 or 8)
 *   "rec_threads" fused recurrence: threads per workgroup, 512 or 1024 (default 1024)
 *   "rec_graph"   evolution below 2^19 rows: runs of this many steps without a sample replay one
 *                 captured hipGraph (even, up to 256; default 0 = launch every step)
 *   "rec_persist" fused recurrence: 0 = one workgroup per tile (default); n = 1..8 persistent
 *                 workgroups per compute unit that prefetch their next tile
 *   "project_whole" projection: 1 = P = V^T (H V) as one GEMM when the block H V (D x m FP64)
 *                 fits in free device memory beside V (default), 0 = always in column chunks
 *   "project_splitk" projection: 1 = when the upper triangle of the m x m output has fewer
 *                 128 x 128 tiles than the GPU has compute units, S and P with K = D split over up
 *                 to 64 workgroup layers (each at least 1024 rows), then mirrored (default); 0 = off
 *   "rec_xcd"     fused recurrence tile order, bit 0 for the low pass and bit 1 for the high
 *                 pass: set = each of the 8 XCDs takes a contiguous eighth of the tiles, clear =
 *                 tiles dealt round-robin in launch order (default 2: high pass only)
 *   "batch_workers" host threads finishing the realisations of dacp_central_eigs_batched (1..64, default 16)
 *   "batch_eig"   dacp_central_eigs_batched: 1 = the finishing threads' dense eigen-decompositions are
 *                 collected and solved in batched launches when the call has more than 8
 *                 realisations (default; smaller calls, such as a retry round, solve each problem
 *                 on its thread's stream), 2 = batched launches always, 0 = one solver per
 *                 problem always
 *   "moment_explicit" dacp_central_eigs and the batched calls with moment_mode 2: 1 = when the
 *                 certified core falls short of N, S and P of the same stored basis are formed
 *                 explicitly and solved again (by the per-problem eigensolver in a batched call)
 *                 before the window is widened (default); 2 = always after the moment solve;
 *                 0 = never
 *   "beig_pipe"   batched eigensolver: 1 = on unreduced blocks of 48 rows or more, the QR sweeps
 *                 of a batch take their shifts at its start and are chased in lockstep, one lane
 *                 per sweep (default); 0 = one sweep after another
 *   "beig_sweeps" batched eigensolver: at most this many QR sweeps per batch, 1..8 (default 6;
 *                 fewer where the rotation buffers would not fit the LDS)
 *   "group"       evolution column-group width when L >= 15 (power of two, default 8)
 *   "filter_group_f64", "filter_group_f32"
 *                 filter column-group width when L >= 15 for the FP64 / FP32 recurrence
 *                 (power of two, defaults 8 and 8)
 *   "blocked"     dense eigensolver: panel tridiagonalisation and compact-WY Q formation for
 *                 n >= value (default 3500, at least 256; 0 = never)
 *   "dc"          dense eigensolver: eigenvectors by divide and conquer for n >= value
 *                 (default 96; 0 = always implicit QR with replayed rotations)
 * Results agree for every setting up to the rounding order of each element's sum ("moment_explicit":
 * within the values' certified error estimates, since S and P are formed differently).
 * Returns DACP_E_INVALID for an unknown key or a value out of range. */
dacp_status dacp_tune(dacp_ctx ctx, const char *key, int value);
/* Current value of a tuning knob (same keys as dacp_tune); value: host. */
dacp_status dacp_tune_get(dacp_ctx ctx, const char *key, int *value);
/* Library version string (static storage). */
const char *dacp_version(void);

/* -------------------------------------------------------------- Hamiltonian */

/* Build device tables for H = sum_t coeff_t P_t from host `terms` (Sec. III,
 * model definitions).  One-body and two-body terms of any real Pauli type are
 * accepted.  Equal Pauli strings are merged.  Errors (DACP_E_INVALID):
 * L outside [1, 30], a site >= L, site_a == site_b in a two-body term, an odd
 * number of Y, reserved != 0, a non-finite coefficient. */
dacp_status dacp_build_hamiltonian(dacp_ctx ctx, int L, int n_terms, const dacp_term *terms, dacp_ham *out);
void dacp_free_hamiltonian(dacp_ham h);
/* Host query: number of spins, sum |c| (triangle bound on ||H||), sum c^2
 * (= tr H^2 / D), number of off-diagonal flip groups. */
dacp_status dacp_ham_info(dacp_ham h, int *L, double *sum_abs, double *sum_sq, int *n_flip_groups);
/* Host query: *flip_sym = 1 when H commutes with the global spin flip prod_i sigma^x_i (every
 * merged Pauli string has an even number of Z and Y factors; dacp_opts.sectors then splits the
 * start columns between its two eigenspaces), else 0. */
dacp_status dacp_ham_flip_symmetry(dacp_ham h, int *flip_sym);

/* y = H x on [D][b] blocks (device), dtype DACP_F64 or DACP_F32 for both x and
 * y, row strides ldx, ldy >= b.  x and y must not overlap.  This is the
 * matrix-free basic step of Sec. II (the paper's tau). */
dacp_status dacp_apply(dacp_ctx ctx, dacp_ham h, int dtype, int b, const void *x, int64_t ldx, void *y, int64_t ldy);

/* ------------------------------------------------------ bound and density */

/* Spectral bound E_b >= ||H|| (Sec. III: upper-bound estimator for E_max).
 * `steps`-step Lanczos from device vector v0 (length D, FP64; NULL draws a
 * seeded Gaussian vector), E_b = safety * max(|theta_max| + r_max,
 * |theta_min| + r_min) with r the Ritz residual norms |beta_k y_k|, clamped to
 * sum |c|.  Host outputs: e_bound, theta_min, theta_max (any may be NULL). */
dacp_status dacp_spectral_bound(dacp_ctx ctx, dacp_ham h, int steps, const double *v0, uint64_t seed, double safety,
                                double *e_bound, double *theta_min, double *theta_max);

/* Chebyshev moments mu_k = <R, T_k(H / e_bound) R> / <R, R>, k < n_moments
 * (kernel polynomial estimate of the density of states; Sec. III sets the
 * window from a density estimate).  R: device [D][nvec] FP64 or NULL for a
 * seeded Gaussian block.  Uses T_{2k} = 2 T_k^2 - T_0 and
 * T_{2k+1} = 2 T_{k+1} T_k - T_1 (App. C, Eq. shift).  mu_out: host. */
dacp_status dacp_dos_moments(dacp_ctx ctx, dacp_ham h, double e_bound, int n_moments, int nvec, const double *R,
                             uint64_t seed, double *mu_out);

/* Seeded start states: out[s * b + j] ~ N(0,1) from Philox4x32-10 with counter
 * (s, j, 0, 0) and key (seed_lo, seed_hi); u1, u2 from the top 53 bits of
 * (r0:r1), (r2:r3) plus half an ulp; z = sqrt(-2 ln u1) cos(2 pi u2).
 * out: device [D][b] FP64. */
dacp_status dacp_random_block(dacp_ctx ctx, int64_t D, int b, uint64_t seed, double *out);

/* ---------------------------------------------------------------- filter */

typedef struct {
  double e_bound;    /* E_max of Eq. F; must be >= ||H||                         */
  double a;          /* window half-width, 0 < a < e_bound                       */
  int K;             /* filter order (Sec. II.A uses 18 E_max / a)               */
  int b;             /* block width (number of start states, Sec. III block filter) */
  int precision;     /* DACP_F64, or DACP_F32: first K - fp64_tail steps in FP32 */
  int fp64_tail;     /* FP64 steps after the FP32 part (precision = DACP_F32)    */
  uint64_t seed;     /* used when `start` is NULL                                */
} dacp_filter_params;

/* psi_E = T_K(F) psi, F = (H^2 - E_c) / E_0, E_c = (E_b^2 + a^2)/2,
 * E_0 = (E_b^2 - a^2)/2, every column normalised to 1 (Sec. II.A, Eq. F,
 * Eq. target).  start: device [D][b] FP64 or NULL (seeded Gaussian).
 * psi_out: device [D][b] FP64.  Columns are filtered independently (in groups
 * of 8 (FP64) or 16 (FP32) when L >= 15, so the working set stays cache resident).  With precision DACP_F32 the first
 * K - fp64_tail steps of the same recurrence run in FP32 (FP32 storage and
 * accumulation); the pair (T_{k-1}, T_k) is then converted to FP64 and the
 * last fp64_tail steps run in FP64.  Start and output must not overlap. */
dacp_status dacp_filter(dacp_ctx ctx, dacp_ham h, const dacp_filter_params *p, const double *start, double *psi_out);

/* ----------------------------------------------------------------- basis */

typedef struct {
  double e_bound; /* G = H / e_bound (Sec. II.B, Eq. G2)                       */
  double a;       /* a_r = a / e_bound                                         */
  int n;          /* number of sample pairs; basis width m = b (2n + 1)        */
  int b;          /* block width                                               */
  int group;      /* evolve columns in groups of this width (0 = library     */
                  /* default: 8 when L >= 15 and b > 8, else all b)          */
} dacp_basis_params;

/* Chebyshev evolution T_{k+1} = 2 G T_k - T_{k-1} from psi_E (device [D][b]
 * FP64) up to k_n, storing panels (App. C, Eq. set2)
 *   panel 0 = psi_E, panel 2m-1 = T_{k_m - 1}(G) psi_E, panel 2m = T_{k_m}(G) psi_E,
 * k_m = 2 floor(m pi / (2 a_r)), m = 1..n, panel p in columns [p b, p b + b)
 * of V (device, row-major D x ldv, ldv >= b (2n + 1)).  m_out (host) gets
 * b (2n + 1).  Returns DACP_E_BOUNDS if the evolved norm exceeds the start
 * norm by more than 1e-6 relative (|T_k(G)| <= 1 must hold for e_bound >= ||H||). */
dacp_status dacp_basis(dacp_ctx ctx, dacp_ham h, const dacp_basis_params *p, const double *psi_e, double *V,
                       int64_t ldv, int *m_out);

/* Moment mode (App. C, Eq. shift): S and P of the Chebyshev basis without storing it.  The samples
 * sit on the uniform grid k_m = m Delta, Delta = 2 floor(pi / (2 a_r)) (a_r = a / e_bound), so that
 * sums of sampled orders are sampled too; the panels are
 *   panel 0 = psi_E, panel 2m-1 = T_{k_m - 1}(G) psi_E, panel 2m = T_{k_m}(G) psi_E, m = 1..n.
 * The evolution runs to 2 k_n and records the b x b moments mu_k = psi_E^T T_k(G) psi_E and
 * nu_k = psi_E^T G T_k(G) psi_E at every order x + y, |x - y| of two panel orders; then, with the
 * product identity T_x T_y = (T_{x+y} + T_{|x-y|}) / 2 and H = e_bound G,
 *   S block (p, q) = (mu_{x+y} + mu_{|x-y|}) / 2,
 *   P block (p, q) = e_bound (nu_{x+y} + nu_{|x-y|}) / 2,
 * x, y the orders of panels p, q.  psi_e: device [D][b] FP64, 1 <= b <= 128.  S, P: device m x m,
 * row stride ld >= m = b (2n + 1), both triangles written (symmetric parts of the assembled
 * blocks).  m_out (host, may be NULL) gets m.  Memory besides S and P: three D x g FP64 blocks,
 * G psi_E (D x b) and the moments.  Errors as dacp_basis (DACP_E_BOUNDS when |T_{k_m}(G) psi|
 * exceeds |psi|). */
dacp_status dacp_basis_moments(dacp_ctx ctx, dacp_ham h, const dacp_basis_params *p, const double *psi_e, double *S,
                               double *P, int64_t ld, int *m_out);

/* Stored basis with the moment projection (App. C, Eq. shift): the panels of the uniform grid of
 * dacp_basis_moments are stored in V (device, row-major D x ldv, ldv >= m = b (2n + 1), panel p in
 * columns [p b, p b + b)).  S and P come from b x b moments given by the Gram products of seven
 * anchor panels (orders 0, 1, 2, k_n - 2, k_n - 1, k_n, k_n + 1) and of their images under H with
 * the stored panels: for an anchor of order A and a panel of order x,
 *   (T_A psi)^T (T_x psi) = (mu_{A+x} + mu_{|A-x|}) / 2,              mu_k = psi^T T_k(G) psi,
 *   (H T_A psi)^T (T_x psi) = e_bound (nu_{A+x} + nu_{|A-x|}) / 2,    nu_k = psi^T G T_k(G) psi,
 * so each moment follows from one block and a moment found before it; then
 *   S block (p, q) = (mu_{x+y} + mu_{|x-y|}) / 2,  P block (p, q) = e_bound (nu_{x+y} + nu_{|x-y|}) / 2.
 * The evolution runs to k_n + 1; the Gram products are 2 D (14 b) m flops, in place of the 2 D m^2
 * of V^T V and V^T (H V).  psi_e: device [D][b] FP64, 1 <= b <= 128.  S, P: device m x m, row
 * stride ld >= m, both triangles written (symmetric parts).  m_out (host, may be NULL) gets m.
 * Memory besides V, S and P: three D x g FP64 blocks, the anchors and their images (D x 14b FP64),
 * their Gram product with V (14b x m FP64) and the derived moments (at most 2 (2 k_n + 1) b^2 FP64).  Errors as dacp_basis (DACP_E_BOUNDS when |T_{k_m}(G) psi| exceeds |psi|,
 * DACP_E_NUMERIC for a non-finite state or moment). */
dacp_status dacp_basis_stored_moments(dacp_ctx ctx, dacp_ham h, const dacp_basis_params *p, const double *psi_e,
                                      double *V, int64_t ldv, double *S, double *P, int64_t ld, int *m_out);

/* ------------------------------------------------------------ projection */

/* S = V^T V and P = V^T (H V) (Sec. II.C, Eq. gep) for the first m columns
 * of V (device, row-major D x ldv).  S, P: device m x m row-major with
 * leading dimension ld >= m, both triangles written.  FP64 throughout. */
dacp_status dacp_project(dacp_ctx ctx, dacp_ham h, int m, const double *V, int64_t ldv, double *S, double *P,
                         int64_t ld);

/* Generalised eigenproblem P B = S B Lambda by App. C: S = V_s L_s V_s^T,
 * drop eigenvalues below eps (1e-12 in the paper), U = V~_s L~_s^(-1/2),
 * H~ = U^T P U, H~ = Y Lambda Y^T, B = U Y.  S and P: device m x m (ld),
 * read only.  theta_out: host, r ascending Ritz values; B_out: device r x m
 * row-major (row j = column j of B), may be NULL; r_out: host rank kept. */
dacp_status dacp_rayleigh_ritz(dacp_ctx ctx, int m, const double *S, const double *P, int64_t ld, double eps,
                               double *theta_out, double *B_out, int *r_out);

/* Dense symmetric eigen-decomposition on the GPU (Householder
 * tridiagonalisation; eigenvectors of the tridiagonal by divide and conquer
 * for n >= the "dc" knob (default 96), else implicit QR with the rotations
 * replayed on the GPU; eigenvalues only: implicit QR): A device n x n (ld),
 * destroyed; w host ascending; Zrows device n x n (row j = eigenvector j) or NULL. */
dacp_status dacp_syev(dacp_ctx ctx, int n, double *A, int64_t ld, double *w, double *Zrows);

/* The same decomposition for `count` matrices in one launch, one workgroup per matrix (App. C's
 * two eigen-decompositions for many small subspace problems, the batched-realisation path):
 * Householder tridiagonalisation, the tridiagonal's eigenvalues by bisection, implicit symmetric
 * QR shifted by the nearest of those not yet deflated (else Wilkinson's shift), Householder Q.
 * n[i] (host): 1 <= n[i] <= 2048.  A[i] (host array of device pointers): symmetric n[i] x n[i],
 * row-major, ld n[i], destroyed.  w[i] (host array of host pointers): n[i] eigenvalues ascending.
 * Z[i] (host array of device pointers, entries may be NULL): n[i] x n[i], row j = eigenvector j.
 * Errors: DACP_E_INVALID (sizes, null pointers), DACP_E_CONVERGENCE (QR did not converge). */
dacp_status dacp_syev_batched(dacp_ctx ctx, int count, const int *n, double *const *A, double *const *w,
                              double *const *Z);

/* dacp_syev_batched that allocates nothing, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same arguments,
 * results and errors as dacp_syev_batched (same kernels).  Every device buffer besides A[i] and
 * Z[i] -- the tridiagonal's eigenvectors, the Householder product, w and beta per matrix, the
 * convergence flags, the problem table and the sort permutation -- lives in one fixed workspace of
 * 128 MiB per device, held from the library's first use on that device until the process ends.  A
 * request fits when 2 sum n[i]^2 + 2 sum n[i] doubles plus small tables fit in it (for example 16
 * matrices of n = 1000, or one of n = 2048); a larger one returns DACP_E_INVALID with the sizes in
 * the message, before any device work.  Every call on one device shares that device's workspace
 * and leaves its contents behind (the flags are cleared at the start of each call): calls that
 * overlap on one device, from any context or thread, race and must be serialised by the caller.
 * No hipMalloc, hipFree or allocating library routine is called; host copies of the problem table
 * and the results still synchronise the context's stream. */
dacp_status dacp_syev_batched_noalloc(dacp_ctx ctx, int count, const int *n, double *const *A, double *const *w,
                                      double *const *Z);

/* C = alpha op(A) op(B) + beta C in FP64 on the matrix cores (row-major;
 * op(A) is M x K: A stored M x K when transA = 0, K x M when transA = 1;
 * op(B) is K x N: B stored K x N when transB = 0, N x K when transB = 1). */
dacp_status dacp_gemm(dacp_ctx ctx, int transA, int transB, int64_t M, int64_t N, int64_t K, double alpha,
                      const double *A, int64_t lda, const double *B, int64_t ldb, double beta, double *C, int64_t ldc);

/* ------------------------------------------------------------- end to end */

typedef struct {
  int b;               /* block width (default 64)                                    */
  int group;           /* recurrence column-group width, 0 = library default (above)  */
  double kfac;         /* K = ceil(kfac * E_b / a) (default 18, Sec. II.A)            */
  double window_ratio; /* levels wanted in [-a, a] = ceil(window_ratio * N) (2.2)     */
  double basis_ratio;  /* m = b (2n + 1) ~ basis_ratio * window count (1.5)           */
  double eps;          /* S eigenvalue cut-off (1e-12, App. C)                        */
  double tol_rel;      /* accept |error| <= tol_rel * max(|theta_min|, |theta_max|) of the */
                       /* bound's Lanczos run, an estimate of ||H|| (1e-10)           */
  int lanczos_steps;   /* bound estimator steps (80)                                  */
  int kpm_moments;     /* density moments (256)                                       */
  int kpm_vectors;     /* random vectors for the density (8)                          */
  double e_bound;      /* > 0: use this bound and skip Lanczos                        */
  double a;            /* > 0: use this window and skip the density estimate          */
  int precision;       /* filter precision: DACP_F64 or DACP_F32                      */
  double fp64_tail_frac; /* FP64 tail steps = ceil(frac * K) when precision is FP32  */
  uint64_t seed;       /* start-state seed                                            */
  int max_retries;     /* window retries on DACP_E_WINDOW (1)                         */
  int moment_mode;     /* 1: moment mode (App. C, Eq. shift; see dacp_basis_moments): S  */
                       /* and P from moments, no stored basis; the candidates' Ritz vectors */
                       /* from a second evolution (D x (N + max(64, N/8)) FP64 on device)   */
                       /* for the residual acceptance.  2: the uniform-grid basis stored, S */
                       /* and P from the anchors' moments (dacp_basis_stored_moments), the  */
                       /* Ritz vectors from V as in 0; if the certified core falls short   */
                       /* of N, S and P of the same basis are then formed explicitly and   */
                       /* solved again before any retry.  0 (default): the basis is stored */
                       /* and S = V^T V, P = V^T (H V) are formed.  The batched calls     */
                       /* store every basis and take 2 as here, 1 as 0.                   */
  int sectors;         /* 1: when H commutes with the global spin flip                  */
                       /* P = prod_i sigma^x_i (every Pauli string has an even number of */
                       /* Z and Y factors), half the start columns are projected onto   */
                       /* P = +1 and half onto P = -1; H keeps each column in its sector */
                       /* and every Ritz vector is an eigenvector of P (b >= 2).         */
                       /* 0 (default): plain Gaussian start columns                       */
} dacp_opts;

typedef struct {
  double e_bound, a, a_r;
  int K, n, b, m, rank, n_candidates, n_accepted, retries;
  int64_t evol_steps;       /* recurrence steps of the evolution (per column group) */
  int64_t evol_launches;    /* evolution kernel launches                            */
  double t_bound_ms, t_filter_ms, t_evol_ms, t_project_ms, t_gep_ms, t_accept_ms, t_total_ms;
  double evol_kernel_ms;    /* HIP-event time of the evolution launches only        */
  double max_err_est;       /* largest accepted error estimate                      */
  int evol_group;           /* column-group width the evolution ran with            */
  int n_ghost;              /* candidates whose residual reaches the window edge   */
  int model_used;           /* dacp_central_eigs_learned: 1 = bound and window from the network */
  int model_fallback;       /* 1 = the network's window failed and Lanczos / KPM redid the call */
  int n_clusters_at_b;      /* returned runs of >= b values, each within 2 tol of the next: a level
                               of multiplicity b; b start states resolve at most b copies of one
                               level (Sec. III, block filter), so its multiplicity may be larger */
} dacp_report;

/* Fill `opts` with the defaults listed above. */
void dacp_default_opts(dacp_opts *opts);

/* The N eigenvalues of H nearest 0, ascending (host eigs_out[N]); err_out
 * (host, may be NULL) gets the residual error estimate of each (the estimate of
 * dacp_accept_rule: the residual norm, or the block quadratic residual bound of a
 * cluster of neighbouring Ritz values over its distance to the rest of the
 * spectrum, whichever is smaller); n_out gets N on success or, on DACP_E_WINDOW,
 * the number accepted.  report may be NULL. */
dacp_status dacp_central_eigs(dacp_ctx ctx, dacp_ham h, int N, const dacp_opts *opts, double *eigs_out,
                              double *err_out, int *n_out, dacp_report *report);

/* dacp_central_eigs that also returns the eigenvectors: the Ritz vectors phi = A b of the N
 * returned values (Sec. II.C: the basis A times the subspace solution), each scaled to unit norm.
 *   vecs_out  device, D x N block, row stride ldvec >= N: vecs_out[s * ldvec + i] is component s
 *             of the vector of eigs_out[i].  Written only when the call returns DACP_OK.
 * Forming them is one extra FP64 GEMM of D x N x m after the acceptance.  The angle between
 * phi_i and the exact eigenvector is at most ||H phi_i - theta_i phi_i|| / gap_i, gap_i being the
 * distance from theta_i to every other eigenvalue, so vectors of near-degenerate levels are only
 * determined as a subspace.  Returns DACP_E_INVALID for a null vecs_out or ldvec < N. */
dacp_status dacp_central_eigpairs(dacp_ctx ctx, dacp_ham h, int N, const dacp_opts *opts, double *eigs_out,
                                  double *err_out, double *vecs_out, int64_t ldvec, int *n_out,
                                  dacp_report *report);

/* dacp_central_eigs for `count` independent realisations (disorder samples, possibly of
 * different L, every L <= 14) with the same N and options.  Bounds, densities and windows are
 * set per realisation; then ONE persistent launch runs the filter and the evolution of every
 * start column of every realisation: each workgroup keeps one 2^L column on chip (the vector
 * being applied in LDS, the recurrence terms in registers) and writes only the sampled panels
 * of its basis (Sec. II.A, II.B on many small problems at once).  Projection, subspace solve
 * and acceptance follow per realisation, spread over host worker threads with their own
 * streams.  The realisations whose accepted core falls short are redone together, in one more
 * batched call, with a 1.5x wider window, a basis ratio 0.2 higher and new start blocks (up to
 * opts.max_retries times).
 *   hams[count]              Hamiltonian handles (distinct or repeated)
 *   eigs_out[count * N]      host; row r = the N values of realisation r, ascending
 *   err_out[count * N]       host, may be NULL; error estimates as for dacp_central_eigs
 *   n_out[count]             host; N, or the number accepted for a realisation that fell short
 *   reports[count]           host, may be NULL; per realisation (t_evol_ms is the time of the
 *                            shared launch, t_filter_ms is 0: the filter runs inside it)
 * Device buffers of the call come from a per-device block cache that keeps freed blocks (up to
 * 32 GB) for later calls until the process ends; reuse is ordered by events on the streams.
 * Returns DACP_E_INVALID for L > 14, DACP_E_BOUNDS if a bound is below ||H||, DACP_E_WINDOW
 * if some realisation stays short after its retries (the others are still filled in). */
dacp_status dacp_central_eigs_batched(dacp_ctx ctx, int count, const dacp_ham *hams, int N, const dacp_opts *opts,
                                      double *eigs_out, double *err_out, int *n_out, dacp_report *reports);

/* The parameters dacp_central_eigs picks for one attempt (Sec. II.A, II.B, III), host code with no
 * device or context: the window holds N_w = min(D, ceil(window_ratio' N)) estimated levels, with
 * window_ratio' = window_ratio * 1.5^attempt; a_r = a / E_b from the density's Chebyshev moments
 * (or opts->a); K = ceil(kfac / a_r); the block width b; n = ceil((basis_ratio N_w / b - 1) / 2)
 * evolution samples per start state, m = b (2n + 1); sampled orders k_j = 2 floor(j pi / (2 a_r)).
 *   D, N, e_bound  state length, wanted values, spectral bound E_b > 0
 *   mu[n_mu]       host, density moments as from dacp_dos_moments (unused when opts->a > 0)
 *   opts           host, may be NULL (defaults); attempt = 0 for the first window
 *   fout[3]        host: N_w, a_r, a
 *   iout[4]        host: K, b, n, m
 *   k_samples      host, may be NULL: the first min(n, max_samples) sampled orders
 * Returns DACP_E_INVALID for D < 1, N outside [1, D], E_b <= 0, attempt < 0, null outputs, or
 * missing moments. */
dacp_status dacp_plan(int64_t D, int N, double e_bound, const double *mu, int n_mu, const dacp_opts *opts,
                      int attempt, double *fout, int *iout, int64_t *k_samples, int max_samples);

/* The acceptance rule of dacp_central_eigs (Sec. II.C: the residual of a Ritz pair bounds its error;
 * here with the quadratic form of that bound), host code with no device or context.  Candidates are
 * the first n_sel Ritz values in the order of (|theta|, theta).
 *   - A candidate is a "ghost" when its residual is at least a - |theta|: a unit vector made only of
 *     eigenvectors outside the window [-a, a] has at least that residual, so a ghost may approximate
 *     no level.  Below it, Weyl's bound places a level within the residual of theta, inside [-a, a].
 *   - Estimate: the smaller of ||r|| and the block quadratic residual bound sum_C ||r||^2 / delta_C,
 *     minimised over every run C of at most 8 consecutive non-ghost candidates (in ascending theta)
 *     that contains the candidate; delta_C is the distance from C to the nearest non-ghost Ritz value
 *     outside C (less that value's own residual when it is a candidate) or to the window edge.
 *     Accepted: estimate <= tol.
 *   - The core walks the candidates outward in |theta| while |theta| <= a; the first ghost or
 *     unaccepted candidate ends it.
 *   theta[r]        host, ascending Ritz values
 *   rnorm[n_sel]    host, residual norms of the unit Ritz vectors, in the (|theta|, theta) order
 *   a, tol          window half-width (> 0) and accepted error (>= 0)
 *   core_out        host: the core's size
 *   core_pos[n_sel] host, may be NULL: the core's positions in that order
 *   est_out[n_sel]  host, may be NULL: estimates (infinite for a ghost)
 *   n_ghost_out     host, may be NULL: the number of ghosts
 * Returns DACP_E_INVALID for n_sel outside [0, r], unsorted theta, a <= 0, tol < 0 or null inputs. */
dacp_status dacp_accept_rule(int r, const double *theta, int n_sel, const double *rnorm, double a, double tol,
                             int *core_out, int *core_pos, double *est_out, int *n_ghost_out);

/* Level statistics of a computed spectrum (the paper's motivation, Sec. I): the gap ratios
 * r_i = min(s_i, s_{i+1}) / max(s_i, s_{i+1}) of consecutive spacings s_i = eigs[i+1] - eigs[i].
 * Host code, no device or context needed.
 *   eigs[n]       host, ascending (n >= 3), e.g. the output of dacp_central_eigs
 *   r_out[n - 2]  host, may be NULL; NaN where both spacings are zero (three equal levels)
 *   mean_out      host, may be NULL; mean of the finite ratios (NaN if there is none)
 * Returns DACP_E_INVALID for n < 3, a null eigs, or values not ascending (or NaN). */
dacp_status dacp_spacing_ratios(const double *eigs, int n, double *r_out, double *mean_out);

/* Autotuner of the evolution recurrence for this Hamiltonian and block width b: times `steps`
 * evolution steps of one column group for every group width (powers of two up to min(b, 16)),
 * workgroup size (512, 1024), fused tile (4096, 8192 elements; also 1024 and 2048 below 2^19
 * rows) and high-tile row count
 * (automatic, 1, 2), at the real state length, and keeps the fastest in ctx (the "group",
 * "rec_threads", "rec_tile", "rec_hi_w" knobs).  best_group and best_us_per_column_step (host,
 * may be NULL) get the winner's group width and its time per column and step. */
dacp_status dacp_autotune(dacp_ctx ctx, dacp_ham h, int b, int steps, int *best_group, double *best_us_per_column_step);

/* Autotuner of the batched schedule: runs dacp_central_eigs_batched on a sample of the realisations
 * (every sample_every-th one, plus the first of each L present; sample_every = 1 times the whole
 * set) for each candidate window ratio (2.2, 2.5, 2.8), basis ratio (1.3, 1.5) and filter factor
 * kfac (12, 18), with the caller's window retries (opts_in->max_retries), and keeps the fastest
 * candidate whose every sampled realisation reached N.  A wider window costs larger subspace
 * problems but redoes fewer realisations whose certified core falls short; kfac trades filter
 * length against the core.  best (host) gets opts_in (may be NULL: defaults) with those three
 * fields replaced; best_s (host, may be NULL) the sample's time with that schedule.
 * Returns DACP_E_WINDOW if no candidate reached N everywhere. */
dacp_status dacp_autotune_batched(dacp_ctx ctx, int count, const dacp_ham *hams, int N, const dacp_opts *opts_in,
                                  int sample_every, dacp_opts *best, double *best_s);

/* ------------------------------------------------------- learned window */

/* A small regression network (multilayer perceptron: `layers` tanh hidden layers of width
 * `hidden`, linear output; loss 0.5 mean |y - t|^2) trained and evaluated on the GPU in FP32
 * by the library's own forward, backward and Adam kernels.  The learned window uses
 * n_in = DACP_WINDOW_FEATURES inputs and 2 outputs.  Parameters: one flat FP32 vector, layer
 * by layer, W (n_out x n_in row-major) then b; initial weights Glorot-uniform from `seed`. */
typedef struct dacp_mlp_s *dacp_mlp;
dacp_status dacp_mlp_create(dacp_ctx ctx, int n_in, int hidden, int layers, int n_out, uint64_t seed, dacp_mlp *out);
void dacp_mlp_free(dacp_mlp m);
/* Copy the parameters out (get, host, may be NULL) and/or in (set, host, may be NULL; resets
 * the Adam state); n_params (may be NULL) gets their number. */
dacp_status dacp_mlp_params(dacp_ctx ctx, dacp_mlp m, float *get, const float *set, int *n_params);
/* Loss and gradient of the network as it stands on n samples X (host n x n_in), T (host
 * n x n_out), without standardisation; grad (host, n_params, may be NULL). */
dacp_status dacp_mlp_loss_grad(dacp_ctx ctx, dacp_mlp m, int n, const double *X, const double *T, double *loss,
                               double *grad);
/* Adam training on standardised columns (means and deviations fixed by the first call's data
 * and kept with the network): `epochs` passes in shuffled mini-batches of `batch`, learning
 * rate lr; final_loss (host, may be NULL) gets the loss of the standardised targets. */
dacp_status dacp_mlp_train(dacp_ctx ctx, dacp_mlp m, int n, const double *X, const double *Y, int epochs, int batch,
                           double lr, uint64_t seed, double *final_loss);
/* Y (host n x n_out) = network(X) in the units of the training targets. */
dacp_status dacp_mlp_predict(dacp_ctx ctx, dacp_mlp m, int n, const double *X, double *Y);

#define DACP_WINDOW_FEATURES 8
/* Coupling statistics of H (host, no GPU work): L / 20, log sigma (sigma^2 = sum c^2 = tr H^2 / D),
 * the diagonal share of sigma^2, its two-body part, the single-spin-flip share, max |c| / sigma,
 * sum |c| / (sigma sqrt(n_strings)), log(n_strings) / log(L (L + 1) / 2 + 2 L). */
dacp_status dacp_window_features(dacp_ham h, double *features);
/* Targets of the learned window from the method's own estimators (Sec. III): per realisation
 * labels[2 r] = log(E_b / (sigma sqrt(2 L ln 2))) from the Lanczos bound (sigma sqrt(2 L ln 2) is
 * the extreme-value scale of 2^L levels of spread sigma, which keeps the target flat in L) and
 * labels[2 r + 1] =
 * log(rho(0) sqrt(2 pi) sigma / D), with rho(0) the kernel-polynomial level density at E = 0
 * (levels per unit energy, averaged over |E| <= 0.02 E_b).  Realisations with L <= 14 run as one
 * batched launch per estimator, the others one by one.  opts (may be NULL) supplies the Lanczos steps, moments,
 * vectors and seed. */
dacp_status dacp_window_labels(dacp_ctx ctx, int count, const dacp_ham *hams, const dacp_opts *opts, double *labels);
/* dacp_central_eigs with the bound and the window predicted by `model` (trained on
 * dacp_window_features -> dacp_window_labels): E_b = (1 + bound_margin) sigma sqrt(2 L ln 2) exp(y0), clamped to
 * sum |c|; a from rho(0) = D exp(y1) / (sqrt(2 pi) sigma) as the half-width holding
 * ceil(window_ratio N) levels.  If the call then fails with DACP_E_BOUNDS (E_b below ||H||),
 * DACP_E_NUMERIC (a filter overflow from such a bound) or DACP_E_WINDOW (too few accepted
 * values), it is redone with the Lanczos / KPM estimates
 * (report->model_fallback = 1): the method's own estimators are both the fallback and the check. */
dacp_status dacp_central_eigs_learned(dacp_ctx ctx, dacp_ham h, dacp_mlp model, double bound_margin, int N,
                                      const dacp_opts *opts, double *eigs_out, double *err_out, int *n_out,
                                      dacp_report *report);

/* dacp_central_eigs_batched with every realisation's bound and window predicted by `model` (one
 * forward pass over all realisations, the formulas of dacp_central_eigs_learned) instead of the
 * batched Lanczos / KPM launches.  Tolerances are relative to each predicted bound / (1 +
 * bound_margin).  A realisation whose predicted bound proves below ||H|| (the evolution's norm
 * guard) or whose accepted core falls short of N is redone alone with the Lanczos / KPM estimates
 * (reports[r].model_fallback = 1).  reports[r].t_bound_ms is the prediction time.  Arguments,
 * outputs and errors otherwise as dacp_central_eigs_batched. */
dacp_status dacp_central_eigs_batched_learned(dacp_ctx ctx, int count, const dacp_ham *hams, dacp_mlp model,
                                              double bound_margin, int N, const dacp_opts *opts, double *eigs_out,
                                              double *err_out, int *n_out, dacp_report *reports);

#ifdef __cplusplus
}
#endif
#endif /* DACP_H */
