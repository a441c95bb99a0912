/*
 * fds.h -- C ABI of the MI355X proxy-surface fast direct solver for 2D
 * time-harmonic elastic scattering by traction-free cavities (Galerkin P1,
 * Burton-Miller formulation).
 *
 * Method: Matsumoto & Maruyama, "Linearly scalable fast direct solver based
 * on proxy surface method for two-dimensional elastic wave scattering by
 * cavity".  Section references below are to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Complex numbers are complex128 stored as interleaved (re, im) doubles.
 * - Geometry (Section 4): one or more closed polygons, vertices in
 *   counter-clockwise order, closed implicitly.  Nodes are numbered
 *   consecutively over the curves in input order.  The normal of each
 *   element points into the cavity (Section 2).
 * - Unknowns: index 2 t + i holds displacement component u_{i+1} at global
 *   node t; N_unk = 2 * (total nodes).  A DOF list is an array of such
 *   indices.
 * - Time factor exp(-i omega t); Hankel functions of the first kind.
 * - Device pointers are HIP device memory (e.g. torch tensor data_ptr());
 *   host pointers are plain host memory.  ``stream`` is a hipStream_t
 *   (NULL = default stream).  Calls are asynchronous with respect to the
 *   host unless stated otherwise; every entry point that returns results on
 *   the host synchronises ``stream`` first.
 * - Matrices passed as device pointers are column-major with a leading
 *   dimension ``ld``.
 * - Every entry point returns an fds_status; on error the out-parameters
 *   are left untouched and nothing leaks.
 */
#ifndef FDS_H
#define FDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fds_factor_s* fds_factor;    /* opaque; owned by the library until fds_destroy */
typedef struct { double re, im; } fds_c64;

typedef enum {
  FDS_OK = 0,
  FDS_EINVAL = 1,     /* bad argument: null pointer, size < 1, ld too small, omega <= 0, mu <= 0,
                         lambda + mu <= 0, rho <= 0, tol outside (0, 1) */
  FDS_EGEOM = 2,      /* a curve with fewer than 8 nodes, a zero-length element, clockwise curve; in
                         fds_build also an element longer than 5 / k_T (the quadrature rules below hold
                         up to k_T h = 5, about 1.3 elements per transverse wavelength) */
  FDS_ENOMEM = 3,     /* device or host allocation failed */
  FDS_EHIP = 4,       /* a HIP runtime call failed */
  FDS_ESINGULAR = 5,  /* zero or non-finite pivot in an LU factorisation */
  FDS_ENOCONV = 6     /* iterative refinement did not reach its tolerance */
} fds_status;

typedef struct {
  int32_t n_curves;
  const int32_t* n_nodes;   /* host, [n_curves] */
  const double* xy;         /* host, [2 * sum(n_nodes)]: x0, y0, x1, y1, ... ; copied by the library */
} fds_geometry;

typedef struct {
  int32_t leaf_nodes;       /* nodes per leaf cell (Section 5.1); default 64 */
  int32_t n_proxy;          /* smallest proxy polygon (Section 7.1); default 64.  A cell whose proxy circle
                               has radius rho gets max(n_proxy, ceil(2 k_T rho) + 40) vertices: an outgoing
                               field on the circle carries Fourier modes up to about k_T rho */
  int32_t root_level;       /* level l0 at which the compressed system is solved (Section 7.3); default 1 */
  int32_t solve_graph;      /* 1: run the solve sweeps as a hipGraph captured once per nrhs on a library
                               stream (the caller's stream is synchronised first); default 0 */
  double proxy_ratio;       /* proxy radius / cell radius; default 1.5 */
  fds_c64 alpha;            /* Burton-Miller coupling; {0,0} selects i / (mu k_T) */
  int32_t use_alpha;        /* 0: alpha = i/(mu k_T); 1: use ``alpha`` as given (0 allowed) */
  int32_t precision;        /* FDS_PREC_FP64 (default): every step in complex FP64.
                               FDS_PREC_MIXED: assembly, IDs and the root LU in FP64; the per-cell LUs,
                               A_i^{-1} U_i, V_i X_i, A~_i and the solve sweeps in complex FP32; each
                               solve refined iteratively against the FP64 compressed operator A_c */
  int32_t ir_max_iter;      /* mixed form: refinement steps allowed per solve; default 10 */
  int32_t proxy_fixed;      /* 1: every proxy polygon has exactly n_proxy vertices (no growth with k_T rho;
                               for comparisons); default 0 */
  double ir_rtol;           /* mixed form: stop when every column has ||f - A_c x|| <= ir_rtol ||f||
                               (default 1e-8) ... */
  double ir_dtol;           /* ... and its last correction ||delta|| <= ir_dtol ||x|| (default 1e-6; the
                               correction measures the error of the previous iterate, which the step
                               then reduces by the contraction factor of the FP32 solve) */
  int32_t rank_mode;        /* FDS_RANK_ADAPTIVE (default): every ID by the pivoted QR of its interaction
                               matrix (Sections 7.1, 7.2).  FDS_RANK_LEARNED: the rank predictor pre-sizes a
                               randomized ID (sketch of ceil(k_pred) + oversample rows); its result is kept
                               when the sketch reveals the rank (taken at tol / 10, with 4 rows to spare)
                               and the residual judge passes (every residual column within tol of the
                               largest column of the interaction matrix itself), else the cell falls back
                               to the pivoted QR; the predictor abstains for cells whose standardised
                               inputs lie beyond 4 of its training sigma */
  int32_t oversample;       /* learned form: extra sketch rows; default 10 */
  uint64_t seed;            /* learned form: seed of the sketches (SplitMix64); default 0x5EED */
  const float* predictor;   /* learned form: host, FDS_MLP_BLOB floats (see fds_mlp_forward); copied */
  int32_t autotune;         /* 1 (default): during the build, time the candidate launch shapes of the solve
                               sweeps (right-hand-side columns per workgroup of the block LU solves: 1, 2,
                               4, ..., 32; GEMM output tiles of 64 x 64 or 64 x 16) on the leaf level of
                               the factor itself, for 1, 8, 32 and 128 right-hand sides, and keep
                               the fastest per class of nrhs (1 | 2-8 | 9-32 | 33+); the choice is cached per
                               device and leaf shape for later factorisations in the process; every shape
                               gives bitwise identical results.  0: fixed shapes */
  int32_t mfma_sweeps;      /* 1 (default): plain FP64 factors run the upward solve sweep on the FP64
                               matrix cores for 16 or more right-hand sides, one launch per level (LU solve by
                               16-row blocks with inverted 16 x 16 diagonal blocks, then f~ = (A~_i V_i) g with
                               A~_i V_i formed once per factor), for levels whose cells have at most 256
                               unknowns and 192 skeleton unknowns; fewer right-hand sides take the LU-solve
                               kernel and a GEMM with A~_i V_i; the downward sweep and larger levels use the
                               LU-solve and GEMM kernels.  0: those kernels for every level */
} fds_options;

enum { FDS_PREC_FP64 = 0, FDS_PREC_MIXED = 1 };
enum { FDS_RANK_ADAPTIVE = 0, FDS_RANK_LEARNED = 1 };

/* Defaults listed above. */
int fds_options_default(fds_options* opt);

/* Factor the Galerkin Burton-Miller system of the given scatterer (Sections
 * 6 and 7; algorithm summary of Section 7.3): per-level proxy compression by
 * column-pivoted-QR interpolative decompositions, the inverse-free upward
 * elimination A~_i = (V_i A_i^{-1} U_i)^{-1}, and an LU of the compressed
 * system at level l0.  ``tol`` is the ID truncation tolerance (Section 8.1).
 * Entries (Section 5.2; the paper gives no quadrature) by element pairs:
 * tensor Gauss-Legendre with 4, 6 or 10 points per element for a gap of at
 * least 8 h, at least 2 h, or less (h the longer element), at least 6
 * points when k_T h > 0.5 and 10 when k_T h > 2.5; coincident pairs by a
 * graded rule across the diagonal (20 offsets, 30 when k_T h > 0.5) and
 * adjacent pairs by Duffy maps about the shared vertex (12 x 12 points per
 * triangle, 24 x 24 when k_T h > 0.5).
 * Synchronous: returns when the factor is complete.  The factor lives in
 * device memory until fds_destroy.  opt == NULL selects the defaults. */
int fds_build(const fds_geometry* geom, double omega, double lambda, double mu, double rho,
              double tol, const fds_options* opt, void* stream, fds_factor* out);

/* Number of complex unknowns 2 N: both displacement components at each of the
 * N nodes of the polygons (Section 4), numbered as stated at the top. */
int fds_size(fds_factor f, int64_t* n_unknowns);

/* Galerkin load vectors f^s_i = int psi^s (u^I_i + alpha (T u^I)_i) ds
 * (Section 5.2) for unit plane waves: kind[k] = 0 for a P-wave
 * u^I = d exp(i k_L d.x), 1 for an S-wave u^I = (J d) exp(i k_T d.x),
 * d = (cos angle[k], sin angle[k]).  kind, angle: host [nrhs].
 * rhs: device, column k at rhs + k * ld, ld >= N_unk. */
int fds_rhs_plane(fds_factor f, int32_t nrhs, const int32_t* kind, const double* angle,
                  fds_c64* rhs, int64_t ld, void* stream);

/* x = A_c^{-1} rhs for nrhs right-hand sides, A_c the compressed operator:
 * upward sweep, root solve, downward sweep (Sections 6.2, 6.3, 7.3).
 * rhs, x: device, column-major with leading dimensions ld_rhs, ld_x
 * (>= N_unk).  rhs is not modified.  Only one solve per factor may run at a
 * time.
 * Mixed form: x_0 from the FP32 sweeps, then x_{j+1} = x_j + delta_j with
 * delta_j the FP32 sweeps applied to f - A_c x_j, the product with A_c
 * taken in FP64 through the compressed (nested U, V, diagonal-block) form;
 * ends when the ir_rtol / ir_dtol rule holds for every column, else after
 * ir_max_iter steps with FDS_ENOCONV (x is written either way; the stats
 * hold the residual).  Synchronises the stream once per step. */
int fds_solve(fds_factor f, int32_t nrhs, const fds_c64* rhs, int64_t ld_rhs,
              fds_c64* x, int64_t ld_x, void* stream);

/* fds_solve without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same sweeps and kernels as fds_solve, and
 * bitwise the same x, with the level vectors of the sweeps in a
 * file-scope device array of 128 MiB (one per device, held until the
 * process ends) instead of the factor's workspace.  Plain FP64 factors
 * only (the mixed form needs refinement buffers: FDS_EINVAL).  The scratch
 * needed is sum over the compressed levels of (B_l + 2 R_l) * nrhs * 16
 * bytes (B_l the level's active unknowns, R_l its skeleton unknowns; about
 * 19 MiB per right-hand side for the 131072-node ellipse at tol 1e-8);
 * more than 128 MiB is refused with FDS_EINVAL (solve fewer right-hand
 * sides per call).  Asynchronous: returns once the work is queued on
 * ``stream`` (no host synchronisation, no allocation, no memset).  Every
 * call on a device shares that device's scratch and leaves its contents
 * behind: calls that overlap on one device (different streams, or other
 * host threads) race, so the caller orders them.  Arguments and errors
 * otherwise as fds_solve. */
int fds_solve_noalloc(fds_factor f, int32_t nrhs, const fds_c64* rhs, int64_t ld_rhs, fds_c64* x, int64_t ld_x,
                      void* stream);

/* y = A_c x with the FP64 compressed operator (Section 6.1: block-diagonal
 * part plus U (skeleton interactions) V, nested over the levels; Section
 * 6.2 for the parents' blocks), for a factor built with FDS_PREC_MIXED (the
 * plain form does not keep U_i and the unfactored blocks: FDS_EINVAL).
 * x, y: device, column-major, ld_x, ld_y >= N_unk.  Synchronous. */
int fds_apply(fds_factor f, int32_t nrhs, const fds_c64* x, int64_t ld_x, fds_c64* y, int64_t ld_y,
              void* stream);

/* Displacement at points of the solid from boundary solutions, by the
 * integral representation of Section 3:
 *   u_i(x) = u^I_i(x) - int_Gamma T^{n_y}_{jk} G_ik(x - y) u_j(y) ds(y),
 * u the piecewise-linear interpolant of each solution's nodal values
 * (Section 4).  geom, omega, lambda, mu, rho: the scatterer and material the
 * solutions belong to (as for fds_build).  x: device, solution r at
 * x + r * ld_x (ld_x >= N_unk), e.g. as written by fds_solve.
 * targets: device, n_target points as (x1, x2) pairs.  kind, angle: host
 * [nrhs], the plane wave of each solution (as for fds_rhs_plane), whose
 * field is added; both NULL: the scattered part only.  out: device,
 * out[r * ld_out + 2 m + i] = u_{i+1} at target m for solution r
 * (ld_out >= 2 n_target).  n_near: host, optional: the number of targets
 * closer to some element than 1/64 of its length.
 * Quadrature per (target, element) by the distance d to the element and its
 * length h: 4-, 6- or 10-point Gauss-Legendre for d >= 8h, 2h, h; for
 * d < h the element is split into min(64, ceil(h/d)) 10-point panels.
 * Targets counted in n_near get less accuracy; the representation does not
 * hold on Gamma itself, and inside a cavity it gives (approximately) zero.
 * nrhs == 0 or n_target == 0: nothing to do (FDS_OK).  Errors: FDS_EINVAL
 * (sizes, pointers, kind not 0/1, only one of kind/angle given, nrhs >
 * 65535, leading dimensions above 2^31 - 1), FDS_EGEOM, FDS_ENOMEM,
 * FDS_EHIP.  Device scratch, for a chunk of targets at a time: the
 * evaluation matrix (2 N_unk complex numbers per target) and the partial
 * products of the matrix-core product over slabs of 1024 unknowns
 * (2 ceil(N_unk / 1024) nrhs complex numbers per target when N_unk > 1024),
 * together at most FDS_FIELD_CHUNK_MB (environment, default 2048) MiB
 * unless one 32-target chunk needs more.  Results do not depend on the
 * chunk size.
 * Synchronous. */
int fds_field(const fds_geometry* geom, double omega, double lambda, double mu, double rho, int32_t nrhs,
              const fds_c64* x, int64_t ld_x, int64_t n_target, const double* targets, const int32_t* kind,
              const double* angle, fds_c64* out, int64_t ld_out, int64_t* n_near, void* stream);

typedef struct {
  int32_t levels;           /* depth L of the tree */
  int32_t root_level;       /* l0 */
  int64_t n_unknowns;
  int64_t root_size;        /* order of the compressed system at l0 */
  int32_t max_rank;         /* largest per-component skeleton size */
  int32_t max_proxy;        /* largest proxy polygon (vertices) of any compressed cell */
  double factor_seconds;    /* wall time of fds_build */
  double assembly_seconds;  /* GPU time in the entry-assembly kernels during the build */
  double id_seconds;        /* GPU time in the pivoted QR / ID kernels */
  double merge_seconds;     /* GPU time in LU / solves / GEMMs of the elimination */
  double root_seconds;      /* GPU time of the root LU */
  int64_t factor_bytes;     /* device bytes held by the factor */
  int64_t kernel_evals;     /* quadrature-point kernel evaluations during the build */
  /* per quadrature class of element pairs: 0 regular pairs with 2, 3 or 4
   * Gauss points on the test element (and 2, 3, 4 or 6 on the trial
   * element), 1 regular pairs with 6 on the test element, 2 the 10-point
   * pairs, 3 coincident, 4/5 adjacent (two orientations) */
  double class_seconds[6];  /* GPU time of that class's integration kernels, summed over launches */
  int64_t class_evals[6];   /* kernel evaluations (quadrature points) of that class */
  int64_t class_launches[6];  /* assembly batches in which the class had pairs */
  /* mixed form, last solve: refinement steps taken, and the largest column
   * values of ||f - A_c x|| / ||f|| and ||delta|| / ||x|| at exit */
  int32_t precision;
  int32_t ir_iterations;
  double ir_residual;
  double ir_correction;
  /* IDs: cells of all compressed levels; learned form: cells whose IDs came
   * from the sketch, and cells that fell back to the pivoted QR because the
   * sketch did not reveal a rank or because the judge rejected it */
  int32_t rank_mode;
  int32_t reserved2;
  int64_t cells_compressed;
  int64_t cells_sketched;
  int64_t cells_fallback_rank;
  int64_t cells_fallback_judge;
  double predict_seconds;   /* host time spent waiting for the rank predictions (launched ahead of each
                               level's assembly) */
  /* autotuner: chosen columns per workgroup of the LU solves and GEMM tile
   * width for nrhs classes 1 | 2-8 | 9-32 | 33+, and its wall time */
  int32_t tune_chunk[4];
  int32_t tune_gemm_cols[4];
  double tune_seconds;
  /* the twelve pair-integration kernels of an assembly batch, in launch
   * order: regular pairs with 2, 3, 4, 6 points on the test element (each
   * general, then series-only), 10-point pairs, coincident, adjacent next,
   * adjacent previous: GPU time summed over launches, quadrature points,
   * launches that had pairs */
  double pair_kernel_seconds[12];
  int64_t pair_kernel_evals[12];
  int64_t pair_kernel_launches[12];
} fds_stats;

int fds_get_stats(fds_factor f, fds_stats* s);

/* Per-cell ranks: for cell c (heap index, Section 5.1) of every compressed
 * level, out[4 c + 0..3] = (k_row comp 1, k_col comp 1, k_row comp 2,
 * k_col comp 2) as found by the IDs at tolerance (before pairing); -1 for
 * cells that were not compressed.  out: host [4 * (2^(L+1) - 1)]. */
int fds_get_ranks(fds_factor f, int32_t* out, int64_t n_out);

/* Skeleton DOF lists of one cell (global unknown indices, component-major,
 * in pivot order).  rows/cols: host, capacity cap; n_out receives the count. */
int fds_get_skeleton(fds_factor f, int32_t cell, int64_t* rows, int64_t* cols, int64_t cap, int64_t* n_out);

/* One record per cell of every compressed level, in the order the levels
 * were compressed (leaves first): the predictor's training data.
 * feat: log(k_T d), log(k_L d) (d = 2 R, R the cell radius used for its
 * proxy circle), level (root 0), log(active DOFs per component), log(rows of
 * the proxy-plus-near interaction matrix), -log10(tol).  rank: (k_row comp 1, k_col comp 1, k_row comp 2,
 * k_col comp 2) at tolerance.  k_pred: the learned form's prediction (-1 in
 * the adaptive form, or when the predictor abstained).  fallback: 0 none,
 * 1 rank not revealed by the sketch, 2 judge rejected, 3 not sketched
 * (predictor abstained, or the sketch would not be smaller than the
 * interaction matrices).  out: host, capacity cap records; n_out receives the count
 * (records beyond cap are not written). */
typedef struct {
  int32_t cell, level;
  int32_t rank[4];
  int32_t k_pred, fallback;
  double feat[6];
} fds_rank_record;

int fds_get_rank_log(fds_factor f, fds_rank_record* out, int64_t cap, int64_t* n_out);

void fds_destroy(fds_factor f);

/* Device memory: the library takes its device buffers from a process-wide
 * cache of blocks, so that a factorisation after the first reuses the
 * blocks of earlier (destroyed) factors instead of calling hipMalloc and
 * hipFree.  A freed block is handed out again at once for work on the
 * stream that freed it, and for another stream only after that stream has
 * passed the free.  At most FDS_CACHE_LIMIT_MB (environment, default
 * 65536) MiB are kept per device.  The pinned host blocks that stage the
 * factorisation's uploads are kept the same way (at most 512 MiB).
 * fds_release_cache hands every cached device block and every cached pinned
 * host block back to the runtime (blocks held by live factors are not
 * touched); fds_cached_bytes gives the device bytes currently held by the
 * cache.  Both are safe to call at any time from the host. */
void fds_release_cache(void);
int64_t fds_cached_bytes(void);

/* Device memory from the caller instead of the cache (so that, e.g.,
 * PyTorch's caching allocator owns every buffer of the library; the
 * interface asks for PyTorch as the provider of device memory):
 *   alloc(bytes, device, stream, ctx) returns a device pointer of at least
 *     ``bytes`` bytes on HIP device ``device``, to be used on ``stream``
 *     (a hipStream_t), or NULL on failure (the entry point then returns
 *     FDS_ENOMEM);
 *   free_fn(ptr, bytes, device, stream, ctx) takes it back; ``stream`` is the
 *     one named at allocation.  Work queued on that stream may still use the
 *     block: the allocator may reuse it for later work on that stream (stream
 *     order) but not on another stream before that work has finished (the
 *     library synchronises any other stream that used the block before the
 *     call).
 * Both callbacks may run on any host thread, during any entry point.
 * alloc == free_fn == NULL restores the library's cache.  The setting is
 * process-wide.  Returns FDS_EINVAL if exactly one callback is NULL, or
 * while the library holds device blocks (live factors; their blocks must go
 * back to the allocator that made them): call it before the first
 * fds_build or after every factor has been destroyed.  On success the
 * cache is emptied, so fds_cached_bytes() stays 0 while the callbacks are
 * set. */
typedef void* (*fds_alloc_fn)(size_t bytes, int32_t device, void* stream, void* ctx);
typedef void (*fds_free_fn)(void* ptr, size_t bytes, int32_t device, void* stream, void* ctx);
int fds_set_allocator(fds_alloc_fn alloc, fds_free_fn free_fn, void* ctx);

const char* fds_strerror(int code);
/* Text of the last error raised on the calling thread (empty if none). */
const char* fds_last_error(void);

/* ------------------------------------------------------------------ steps
 * Step-level entry points used to check each part of the path on its own.
 */

/* Galerkin entries A(rows, cols) of D + I0/2 + alpha N (Section 5.2) for
 * arbitrary DOF lists of the given geometry, computed by the GPU assembly
 * kernels.  rows, cols: host int64 [nr], [nc].  out: device, column-major
 * nr x nc, leading dimension ld >= nr.  Synchronous. */
int fds_entries(const fds_geometry* geom, double omega, double lambda, double mu, double rho,
                const fds_options* opt, int64_t nr, const int64_t* rows, int64_t nc,
                const int64_t* cols, fds_c64* out, int64_t ld, void* stream);

/* Special functions on the GPU (equation of the fundamental solution): for
 * each x[k] > 0 (device double [n]) writes out[4 k + 0..3] = J0, J1, Y0, Y1
 * at x, and with a = x[k], b = beta a the combinations
 * E = (a H1(a) - b H1(b)) / a^2 and chi = H2(a) - beta^2 H2(b):
 * outc[2 k] = E, outc[2 k + 1] = chi.  out: device double [4 n];
 * outc: device fds_c64 [2 n].  Synchronous. */
int fds_special_eval(int64_t n, const double* x, double beta, double* out, fds_c64* outc, void* stream);

/* Batched column-pivoted QR interpolative decomposition (Section 7.1):
 * for problem p, the m[p] x n[p] column-major matrix at a + off[p] (leading
 * dimension m[p]) is overwritten by its partial QR; after at most kmax[p]
 * steps (stopping early at the first |R_jj| <= tol |R_11| when stop_at_tol
 * is set) piv (device int32, n[p] entries at pivoff[p]) holds the column
 * order and rank[p] (device int32) the number of steps taken.  Pivot rule:
 * largest exactly recomputed remaining column norm, ties within a relative
 * 1e-12 going to the lowest original column.  All size/offset arrays are
 * host int64 [np].  Synchronous. */
int fds_cpqr_batched(int32_t np, fds_c64* a, const int64_t* off, const int64_t* m, const int64_t* n,
                     int32_t* piv, const int64_t* pivoff, const int64_t* kmax, double tol,
                     int32_t stop_at_tol, int32_t* rank, void* stream);

/* Interpolation matrices of finished column IDs (Section 7.1): for problem
 * p with rank k = rank[p] > 0 (host int32 [np]), the matrix at a + off[p]
 * (device, m[p] x n[p], leading dimension m[p]) holding the partial QR and
 * piv + pivoff[p] the pivots written by fds_cpqr_batched, writes
 * W = [I, R11^{-1} R12] P^T (k x n[p], column-major, leading dimension k)
 * at w + woff[p] (device), so that M ~ M(:, piv[0..k)) W.  R12 is
 * overwritten by R11^{-1} R12.  Problems of rank 0 are skipped.  Ranks up
 * to 64 stage R11 in LDS; larger ranks solve one column per thread.  Host
 * int64 arrays [np].  Synchronous. */
int fds_interp_batched(int32_t np, fds_c64* a, const int64_t* off, const int64_t* m, const int64_t* n,
                       const int32_t* piv, const int64_t* pivoff, const int32_t* rank, fds_c64* w,
                       const int64_t* woff, void* stream);

/* Batched LU with partial pivoting (the factorisation of the diagonal
 * blocks A_i and of the compressed system, Sections 6.2, 6.3): for matrix p
 * the n[p] x n[p] column-major matrix at a + off[p] (device, ld n[p]) is
 * overwritten by L (unit lower, below the diagonal) and U; piv (device int32,
 * n[p] entries at pivoff[p]) records that row k was swapped with row piv[k]
 * at step k (0-based).  Pivot: largest modulus in the column, lowest row on
 * ties.  Matrices up to 384 rows are factored by one workgroup each with the
 * panel in LDS (except those above 128 rows in a batch of at most 8),
 * larger ones by the multi-workgroup blocked form (panels of 32 or 16
 * columns in LDS when they fit, else in memory).  info (host int32 [np]):
 * 0, or 1 + the first step with a zero or non-finite pivot (that column
 * keeps its row).  Synchronous. */
int fds_lu_batched(int32_t np, fds_c64* a, const int64_t* off, const int64_t* n, int32_t* piv,
                   const int64_t* pivoff, int32_t* info, void* stream);

/* Randomized column ID with residual judge (learned form of the IDs of
 * Sections 7.1, 7.2): for problem p with the m[p] x n[p] column-major matrix
 * M at a + off[p] (device, ld m[p]; not modified), Y = Omega M with Omega
 * s[p] x m[p], entry (i, l) = (+-1) + i (+-1) from bits 0 and 1 of
 * SplitMix64(seed) output number (gid[p] << 44) | (i << 24) | l; pivoted QR
 * of Y (pivot rule of fds_cpqr_batched) to the first
 * |R_jj| <= sketch_tol |R_11| (the learned factorisation uses tol / 10),
 * giving rank[p] and piv (host int32, n[p] entries at pivoff[p], the first
 * rank[p] being the skeleton); revealed[p] = rank[p] + 4 <= s[p] or
 * s[p] >= n[p]; ratio[p] = max_j |M(:,j) - M(:,J) W(:,j)| / max_j |M(:,j)|
 * with J, W the ID of rank[p] from the sketch.  1 <= s[p] <= m[p],
 * n[p] <= 4096 (sketches of up to 64 rows and 128 columns by the LDS
 * kernel, larger ones by GEMM, as in the learned factorisation).  Host
 * arrays are int64 [np] unless stated.  Synchronous. */
int fds_rid_batched(int32_t np, const fds_c64* a, const int64_t* off, const int64_t* m, const int64_t* n,
                    const int64_t* s, const int64_t* gid, uint64_t seed, double sketch_tol, int32_t* piv,
                    const int64_t* pivoff, int32_t* rank, int32_t* revealed, double* ratio, void* stream);

/* Rank predictor: 6-64-64-64-1 perceptron with ReLU.  A predictor is a
 * float blob of FDS_MLP_BLOB entries: W1 (64 x 6, row-major, row j = hidden
 * unit j), b1 (64), W2 (64 x 64), b2, W3 (64 x 64), b3, w4 (64), b4 (1) --
 * the FDS_MLP_PARAMS trainable entries -- then mu (6), sigma (6), y_scale.
 * The prediction for features x is y_scale * (w4 . h3 + b4) with
 * h1 = relu(W1 (x - mu) / sigma + b1), h2 = relu(W2 h1 + b2),
 * h3 = relu(W3 h2 + b3). */
#define FDS_MLP_PARAMS 8833
#define FDS_MLP_BLOB 8846

/* A fresh predictor for training data x (device float n x 6 row-major),
 * y (device float [n]): mu, sigma = mean and population standard deviation
 * of each feature (sigma 1 where it is 0), y_scale = max(1, max y); weights
 * He-uniform, entry p (flat index in the blob) = lim (2 u - 1) with
 * u = (SplitMix64(seed) output p >> 11) 2^-53 and lim = sqrt(6 / fan_in);
 * biases 0.  blob: host [FDS_MLP_BLOB], written.  Synchronous. */
int fds_mlp_init(float* blob, int64_t n, const float* x, const float* y, uint64_t seed, void* stream);

/* Predictions for n feature rows.  blob: host; x: device float n x 6
 * row-major; y: device float [n].  bf16 = 1 rounds weights, inputs and
 * activations to bfloat16 (FP32 accumulation), as the learned factor does;
 * 0 computes in FP32.  Synchronous. */
int fds_mlp_forward(const float* blob, int64_t n, const float* x, float* y, int32_t bf16, void* stream);

/* Mean squared error L = mean_k (net(x_k) - y_k / y_scale)^2 over all n
 * rows and its gradient with respect to the trainable parameters (FP32,
 * deterministic).  blob, grad (FDS_MLP_PARAMS), loss: host; x, y: device.
 * Synchronous. */
int fds_mlp_loss_grad(const float* blob, int64_t n, const float* x, const float* y, float* grad, float* loss,
                      void* stream);

/* Train on the GPU: ``steps`` Adam steps (beta1 0.9, beta2 0.999, eps 1e-8,
 * learning rate lr) on minibatches of ``batch`` rows drawn with replacement
 * (row SplitMix64(seed) output (step << 32) | slot, mod n, step 1-based);
 * batch = 0 uses all rows every step.  blob: host, updated in place (only the
 * trainable entries change); loss_hist: host [steps] or NULL, the minibatch
 * loss before each step.  Synchronous. */
int fds_mlp_train(float* blob, int64_t n, const float* x, const float* y, int32_t steps, int64_t batch, float lr,
                  uint64_t seed, float* loss_hist, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* FDS_H */
