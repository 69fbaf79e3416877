/*
 * h2.h - C ABI of libh2mi, an accuracy-controlled H^2 direct solver for AMD
 * MI355X (gfx950).
 *
 * The solver implements the level-by-level factorization of a general
 * H^2-matrix of Ma & Jiao, "Accuracy Directly Controlled Fast Direct
 * Solutions of General H^2-Matrices and Its Application to Electrically
 * Large Integral-Equation-Based Electromagnetic Analysis" (arXiv:1703.06155):
 * at every tree level each cluster's basis is updated with the fill-ins to a
 * prescribed accuracy (Sec. III-A-2, eqs. 16-18 / 25-27), zeros are
 * introduced with [V_perp V]^H from both sides (eqs. 5-8 / 30), a partial LU
 * of the rank-sized diagonal block is taken and its Schur complement is
 * applied to the coupled blocks (eqs. 9-15 / 31-32), level after level up to
 * the coarsest admissible level l0 (Alg. 1); the factors Z = L U of eq. 34
 * are then applied by the substitution sweeps of Sec. IV (Algs. 5-6).
 *
 * The matrix is the one of a volume integral equation on N cells:
 *   A_ij = k^2 chi_j h^3 e^{-jkr_ij} / (4 pi r_ij)   (i != j),
 *   A_ii = 1 + chi_i ((1 + jka) e^{-jka} - 1),  a = (3 / (4 pi))^{1/3} h.
 * A = Z D with D = diag(k^2 h^3 chi) and Z complex symmetric; the library
 * factors Z, whose single cluster basis per cluster serves rows and columns
 * as the paper's eqs. 2, 5, 7-8 and 16 require, and solves A x = b as
 * Z y = b, x = D^-1 y.
 *
 * Conventions for every call:
 *   - complex vectors are interleaved (re, im) doubles ("c128"), column-major
 *     with leading dimension ld >= n, in the caller's point order;
 *   - vector arguments (b, x, g, lam, y) are DEVICE pointers; points and
 *     contrast are HOST pointers, copied during the call;
 *   - hip_stream is a hipStream_t (NULL = the default stream); all device work
 *     of a call is enqueued on it;
 *   - no call throws; every call returns an h2_status and, on failure, sets a
 *     thread-local message readable with h2_last_error();
 *   - arguments are validated before any device work, so argument errors are
 *     reported without touching a GPU;
 *   - a handle is not thread-safe, and successive calls on one handle must be
 *     ordered on the device (the same stream, or the caller synchronises
 *     between streams); distinct handles are independent.
 */
#ifndef H2MI_H
#define H2MI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct h2_ctx* h2_handle;

typedef enum {
  H2_OK = 0,
  H2_ERR_ARG = 1,       /* invalid argument (null pointer, size, range, non-finite) */
  H2_ERR_OOM = 2,       /* device allocation failed */
  H2_ERR_SINGULAR = 3,  /* zero pivot in a partial or final LU */
  H2_ERR_STATE = 4,     /* call out of order (e.g. solve before factor) */
  H2_ERR_DEVICE = 5,    /* no usable gfx950 device, or a HIP runtime error */
  H2_ERR_NOCONV = 6,    /* refinement did not reach tol within max_iter, or its residual is not finite */
  H2_ERR_INTERNAL = 7   /* size beyond a kernel limit, or an internal invariant broke */
} h2_status;

enum { H2_FP64 = 0, H2_MIXED = 1 };
enum { H2_ORDER_COLOR = 0 };

typedef struct {
  size_t struct_size;          /* sizeof(h2_options); guards ABI growth */
  int32_t precision;           /* H2_FP64 (default) or H2_MIXED (complex64 Schur and
                                  projection GEMMs, FP64 everything else) */
  int32_t order;               /* H2_ORDER_COLOR: clusters of one colour of a level's
                                  inadmissible graph are eliminated together */
  double eps_fill;             /* Step 0 truncation (eqs. 17, 26); <= 0: use eps */
  const int32_t* forced_ranks; /* optional host array pinning rank decisions, layout in
                                  h2_forced_ranks_layout(); NULL: decide from eps */
  int64_t forced_ranks_len;    /* number of int32 entries behind forced_ranks */
  /* Optional device allocator (both or neither; Python passes PyTorch's caching
   * allocator).  Every device buffer the handle owns then comes from alloc(bytes,
   * stream, alloc_ctx), where stream is the hipStream_t of the call that needs it,
   * and goes back through free(p, stream, alloc_ctx) after the library has waited
   * for all of its device work.  alloc returning NULL makes the call fail with
   * H2_ERR_OOM; the handle stays usable (a failed h2_factor leaves it unfactored).
   * Buffers grow on demand and are kept by the handle until h2_destroy, so calls
   * after the first factorization and solve of a given size allocate nothing.
   * The functions may be called from the library's batch threads.  NULL: the
   * library uses hipMalloc / hipFree. */
  void* (*alloc)(size_t bytes, void* stream, void* ctx);
  void (*free)(void* p, void* stream, void* ctx);
  void* alloc_ctx;
  int32_t stop_level;          /* last level factored (Sec. III-C, closing remark): levels
                                  L..stop_level take Steps 0-3, and the matrix merged to
                                  level stop_level - 1 is factored by a dense LU; 0: the
                                  coarsest admissible level l0 (Alg. 1); otherwise it must
                                  lie in [l0, L] (H2_ERR_ARG) */
} h2_options;

typedef struct {
  int32_t iterations;          /* refinement steps taken (0 for a plain solve) */
  double rel_residual;         /* ||b - A_H2 x|| / ||b|| after the last step (column max) */
  double rel_residual_first;   /* the same after the first solve */
} h2_solve_info;

/* Build the H^2 representation of Z (Sec. II, eqs. 1-3) on the device.
 *   points   host, n x 3 row-major cell centres (distinct);
 *   k, h     wavenumber and cell edge (> 0);
 *   contrast host, n real values, each finite and > 0;
 *   leaf     maximum leaf cluster size (>= 1); eta >= 0 admissibility
 *            parameter of eq. 1; eps in (0,1) truncation of the nested bases
 *            (sigma_j > eps * sigma_1 of each far-field block row).
 * The cluster tree bisects every cluster at the midpoint of its bounding
 * box's longest side until all leaves hold <= leaf points; eq. 1 is tested on
 * cell-support boxes (centres +- h/2).  On success *out owns all device
 * memory of the problem; release it with h2_destroy.  Synchronises the stream. */
h2_status h2_build(const double* points, int64_t n, double k, double h, const double* contrast,
                   int32_t leaf, double eta, double eps, const h2_options* opt,
                   void* hip_stream, h2_handle* out);

/* Replace the per-cell contrast (host array of n values, each finite and
 * > 0, caller order).  Only the diagonal of Z = A D^-1 depends on the
 * contrast, so the nested bases and couplings are kept and the inadmissible
 * leaf blocks are recomputed; the result equals a fresh h2_build with the new
 * contrast.  The handle becomes unfactored.  Synchronises the stream. */
h2_status h2_set_contrast(h2_handle H, const double* contrast, void* hip_stream);

/* Select the arithmetic of the next h2_factor: H2_FP64, or H2_MIXED where the
 * Schur updates (eq. 12) and the zero-introducing projections (eqs. 5/30) run
 * on complex FP32 matrix cores with FP32 accumulation while Step 0, the
 * partial LU and the refinement residual stay FP64.  A change of precision
 * leaves the handle unfactored. */
h2_status h2_set_precision(h2_handle H, int32_t precision);

/* Replay the forward/backward sweeps of h2_solve and h2_solve_adjoint from HIP
 * graphs (enable != 0): the first solve with a given right-hand-side count and
 * direction after each factorization captures the sweep's launches on a
 * private stream; later solves launch the graph on the caller's stream.
 * Results are identical to the direct launches.  Default: off. */
h2_status h2_set_sweep_graph(h2_handle H, int32_t enable);

/* Change the stop level of later factorizations (the meaning of
 * h2_options.stop_level; 0 = l0).  The handle becomes unfactored. */
h2_status h2_set_stop_level(h2_handle H, int32_t level);

/* Schur flush splitting at a level (level = -1: every level): a colour's flush
 * whose tasks, kept whole, would make fewer than below_wgs 64 x 64 tile
 * workgroups splits every task of more than 10 terms into chunks (partial
 * tiles summed in a fixed order by a second kernel); a larger flush keeps
 * every task whole.  below_wgs = -1 restores the default (8192), 0 never
 * splits.  The choice depends on sizes only, so results stay deterministic for
 * given settings; it changes the order in which a block's updates are summed,
 * hence the rounding.  The handle becomes unfactored. */
h2_status h2_set_schur_split(h2_handle H, int32_t level, int64_t below_wgs);

/* Mixed form: the Schur flush kernel of a level (level = -1: every level).
 * mode 1: terms of clusters whose panels show no growth run on FP32 matrix
 * cores, the others in FP64; 0: every term in FP64 (only the projections stay
 * mixed at that level); -1: the default rule (FP32 routing where the level's
 * clusters eliminate 32 or more unknowns on average).  The handle becomes
 * unfactored when it is in the mixed form. */
h2_status h2_set_mixed_flush(h2_handle H, int32_t level, int32_t mode);

/* Terms per chunk of a split Schur task at a level (level = -1: every level;
 * terms = -1: the default, 10): a colour's flush that splits (h2_set_schur_split)
 * cuts every task of more pending terms into chunks of at most this many.
 * Rebuilds the level's flush lists; the handle becomes unfactored.  Changes
 * the order in which a block's updates are summed, hence the rounding. */
h2_status h2_set_schur_chunk(h2_handle H, int32_t level, int32_t terms);

#define H2_TUNING_MAX_LEVELS 64

/* Measured settings of a handle (h2_tune). */
typedef struct h2_tuning {
  int32_t stop_level;        /* chosen stop level (0 when no block is admissible) */
  int32_t from_cache;        /* 1: taken from the process-wide cache, only the final factorization ran */
  int64_t split_below[H2_TUNING_MAX_LEVELS]; /* per level l: the Schur split threshold (-1: not factored) */
  int32_t mixed_flush[H2_TUNING_MAX_LEVELS]; /* per level l, mixed form: the flush mode (-1: not factored or FP64 form) */
  int32_t schur_chunk[H2_TUNING_MAX_LEVELS]; /* per level l: terms per chunk of split Schur tasks (-1: not factored) */
  double factor_ms;          /* factorization time with the chosen settings */
} h2_tuning;

/* Autotuner: chooses the stop level (as h2_tune_stop_level, with the default
 * split and flush rules) and then, per factored level, the Schur split
 * threshold among {0, 2048, 8192, 32768, unlimited}, in the mixed form the
 * flush mode among {0, 1}, and the terms per chunk of split tasks among
 * {5, 10, 20}, by one factorization per candidate (the candidate
 * on every level at once; each level keeps the candidate under which its own
 * time was lowest).  The result is stored in a process-wide cache
 * keyed by the cluster tree (every cluster's size), eta, eps, the form, the
 * forced ranks and max_final; a later call on any handle with the same key
 * applies the cached settings and factors once.  The handle is left factored
 * with the chosen settings.  Synchronises the stream.  Thread-safe. */
h2_status h2_tune(h2_handle H, int64_t max_final, void* hip_stream, h2_tuning* out);

/* Empty the autotuner's cache. */
h2_status h2_tune_cache_clear(void);

/* The stop level in force (*level = 0 when no block is admissible). */
h2_status h2_stop_level(h2_handle H, int32_t* level);

/* Choose the stop level by measurement: factor with the stop at l0, l0 + 1, ...
 * (HIP-event time of each whole factorization, ms[e] for the stop l0 + e when
 * ms is not NULL, n_ms entries, -1 where not tried) and keep the fastest.  A
 * run stopped at l knows the kept unknowns of level l + 1, i.e. the dense block
 * a stop at l + 1 would leave; the search ends before that block would exceed
 * max_final unknowns.  The handle is left factored with the chosen level
 * (*chosen).  Synchronises the stream. */
h2_status h2_tune_stop_level(h2_handle H, int64_t max_final, void* hip_stream, int32_t* chosen, double* ms,
                             int32_t n_ms);

/* Factor Z = L U in the product form of eq. 34 (Alg. 1 with Steps 0-3 per
 * cluster, Algs. 2-4; coupling/transfer updates eqs. 20-23 / 33; final LU of
 * the block merged to the level above the stop level, l0 - 1 by default; an
 * early stop adds to it the blocks of coarser admissible pairs expanded
 * through the transfer matrices, eqs. 2-3).  Synchronises once per level to size the next
 * level's storage.  H2_ERR_SINGULAR leaves the handle unfactored. */
h2_status h2_factor(h2_handle H, void* hip_stream);

/* x = M^-1 b for nrhs columns (forward sweep Alg. 5, backward sweep Alg. 6;
 * eqs. 37, 41), where M = L U D approximates A.  With tol > 0 iterative
 * refinement x += M^-1 (b - A_H2 x) runs until the relative residual against
 * the H^2-represented matrix A_H2 = Z_H2 D (the accuracy measure of the
 * paper's Sec. VI-B) is <= tol for every column, at most max_iter steps
 * (H2_ERR_NOCONV otherwise, x holding the last iterate).  b and x may alias.
 * Without refinement the call is asynchronous; info may be NULL. */
h2_status h2_solve(h2_handle H, const void* b, void* x, int32_t nrhs, int64_t ld, double tol,
                   int32_t max_iter, void* hip_stream, h2_solve_info* info);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): x = M^-1 b
 * exactly as h2_solve with tol = 0 computes it (the same kernels, identical
 * results), with every work buffer of the sweeps - the per-level vectors, the
 * final-block vectors and the backward gather's partial sums - carved from a
 * fixed 64 MiB device array that the library holds on each device it runs on
 * until the process ends.  The call allocates nothing (no hipMalloc, no
 * allocator callback); H must be factored.  Sizes whose work space exceeds
 * 64 MiB (e.g. more than one right-hand side at N = 262144) are rejected with
 * H2_ERR_ARG before any device work.  All calls on one device share that
 * array and keep its last contents: calls that overlap on one device (other
 * streams, other threads) race and must be serialised by the caller.  b and x
 * are device pointers (ld >= n) and may alias.  Asynchronous. */
h2_status h2_solve_noalloc(h2_handle H, const void* b, void* x, int32_t nrhs, int64_t ld, void* hip_stream);

/* lam = M^-H g: the conjugate transposes of the sweeps of eq. 35 applied in
 * reverse order over the same factors (the exact adjoint of the computed
 * solve).  With tol > 0 the result is refined against A_H2^H = D conj(Z_H2)
 * exactly as h2_solve refines against A_H2.  g and lam may alias.  Without
 * refinement the call is asynchronous; info may be NULL. */
h2_status h2_solve_adjoint(h2_handle H, const void* g, void* lam, int32_t nrhs, int64_t ld, double tol,
                           int32_t max_iter, void* hip_stream, h2_solve_info* info);

/* Gradient of a real loss with respect to the per-cell contrast through
 * x = A^-1 b, given x (nrhs columns), g = dL/d conj(x) in PyTorch's convention
 * and lam = A^-H g from h2_solve_adjoint: column j of A equals
 * chi_j (k^2 h^3 G e_j + c e_j) + e_j (c the self term of the diagonal), so
 * grad_chi[j] = sum over columns of Re(conj(lam_j - g_j) x_j) / chi_j.
 * x, g, lam: device, column-major with leading dimension ld; grad_chi: device,
 * n doubles, overwritten, in the caller's point order.  Exact for the exact
 * inverse; with the factorization's lam the error is of the order of the
 * solve's residual.  Asynchronous. */
h2_status h2_contrast_gradient(h2_handle H, const void* x, const void* g, const void* lam, int32_t nrhs,
                               int64_t ld, double* grad_chi, void* hip_stream);

/* y = A_H2 x (conj_transpose = 0) or y = A_H2^H x (conj_transpose = 1), with
 * the inadmissible leaf blocks and V_t S_ts V_s^T (eq. 2) applied through the
 * nested bases (eq. 3).  x and y must not alias.  Asynchronous. */
h2_status h2_matvec(h2_handle H, const void* x, void* y, int32_t nrhs, int64_t ld,
                    int32_t conj_transpose, void* hip_stream);

/* Factor `count` independent handles together (h2_factor_batch_mode with
 * H2_BATCH_FUSED). */
h2_status h2_factor_batch(h2_handle* hs, int32_t count, void* hip_stream);

/* Batch schedules of h2_factor_batch_mode. */
#define H2_BATCH_FUSED 0   /* one launch per (level step, colour index, stage) for all problems */
#define H2_BATCH_STREAMS 1 /* one stream per handle, driven by up to eight host threads */

/* Factor `count` independent handles together; each handle's factors are
 * bit-identical to those of h2_factor.  Handles must be distinct; each may use
 * its own precision, stop level, forced ranks and allocator.
 * H2_BATCH_FUSED: the problems advance in lockstep, level by level from each
 *   one's finest level (Alg. 1), on hip_stream; every stage of colour index c
 *   (Schur flush, Step 0 Gram and eigenvectors, projections, partial LU,
 *   panels) is a single launch whose workgroups cover the work items of every
 *   problem that has colour c (problems whose sizes select another kernel
 *   variant go to a second launch of that variant).  Host synchronisation: once
 *   per level step for all problems.  Timings of the handles (h2_timing,
 *   h2_level_timing) then cover the whole batch up to that handle's end, and
 *   per-kernel times are not measured.  The shared launches' work item table
 *   lives in hs[0] (allocated through its allocator, kept for later batches).
 * H2_BATCH_STREAMS: each handle works on a stream of its own (default
 *   priority, created on first use) and up to eight host threads drive them;
 *   all start after the work already queued on hip_stream, and hip_stream
 *   waits for all of them.
 * Returns the first failure ("batch item k: ..."); the other items are still
 * factored.  H2_ERR_ARG for an unknown mode. */
h2_status h2_factor_batch_mode(h2_handle* hs, int32_t count, void* hip_stream, int32_t mode);

/* x[k] = M_k^-1 b[k] for every handle k as h2_solve does (nrhs columns,
 * leading dimension ld[k], refinement to tol when tol > 0, infos[k] when infos
 * is not NULL): h2_solve_batch_mode with H2_BATCH_FUSED.  b[k], x[k] are device
 * pointers; b[k] and x[k] may alias. */
h2_status h2_solve_batch(h2_handle* hs, int32_t count, const void* const* b, void* const* x, int32_t nrhs,
                         const int64_t* ld, double tol, int32_t max_iter, void* hip_stream, h2_solve_info* infos);

/* Batched solves (Algs. 5-6, refined as h2_solve).  H2_BATCH_FUSED: on hip_stream,
 * the problems' sweeps run in lockstep, every stage of a colour (forward local
 * products and gathers, backward partial sums and local products) one launch
 * over all problems that have that colour; merges, final blocks and the
 * refinement residuals per problem; one host synchronisation per refinement
 * step for all problems; problems leave the refinement as they converge.
 * H2_BATCH_STREAMS: a stream per handle driven by up to eight host threads.
 * Results equal h2_solve's bit for bit in both modes.  A failing problem
 * (H2_ERR_NOCONV) is reported ("batch item k: ...") after the others finish;
 * infos[k] is filled for every problem. */
h2_status h2_solve_batch_mode(h2_handle* hs, int32_t count, const void* const* b, void* const* x, int32_t nrhs,
                              const int64_t* ld, double tol, int32_t max_iter, void* hip_stream, h2_solve_info* infos,
                              int32_t mode);

/* Release every resource of H (NULL is ignored). */
void h2_destroy(h2_handle H);

/* Message describing the last failure on the calling thread ("" if none). */
const char* h2_last_error(void);

/* Host-only structure query (no device is touched): builds the cluster tree,
 * block partition and colouring exactly as h2_build does.  counts receives 8
 * int64 values: N, L, l0 (-1 if no admissible block), leaves, leaf_min,
 * leaf_max, admissible pairs at the leaf level, inadmissible pairs at the
 * leaf level.  perm (nullable, n entries) receives the tree order of the
 * points; colours (nullable, leaves entries) the leaf colours. */
h2_status h2_structure(const double* points, int64_t n, double h, int32_t leaf, double eta,
                       int64_t* counts, int64_t* perm, int32_t* colours);

/* Host-only query of the deferred Schur updates of one tree level (no device is
 * touched; Sec. III-A, eq. 12).  Eliminating cluster i updates every block
 * (a, b) with a and b in i's inadmissible list; the library keeps each update
 * pending until a or b is next processed or the level ends, and sums a block's
 * pending updates in one pass.  The updates are written to out as records of four
 * int64: event, a, b, i (event c < *ncolours: the flush before colour c is
 * eliminated; event *ncolours: the flush at the level's end; a <= b the block's
 * clusters, i the eliminated cluster), in flush order and, within a block, in
 * the order they are summed.  *count receives the number of records and
 * *ncolours the level's colours.  With out == NULL only those two are written;
 * H2_ERR_ARG if cap < 4 * records or level lies outside [l0, L] of the tree
 * h2_structure describes. */
h2_status h2_schur_schedule(const double* points, int64_t n, double h, int32_t leaf, double eta, int32_t level,
                            int32_t* ncolours, int64_t* out, int64_t cap, int64_t* count);

/* Host-only query of how the blocks of one tree level are merged into the blocks
 * of its parent level (Sec. III-A, eq. 23; no device is touched).  Each ordered
 * child pair (a, b) that holds a block (inadmissible, admissible, or filled in by
 * Schur updates) is written to out as seven int64: parent row cluster, parent
 * column cluster, ci = a & 1, dj = b & 1 (the child's position in the parent
 * block), kind (0 inadmissible, 1 admissible, 2 fill-in), a, b.  Parent blocks
 * are stored for parent row <= parent column, so pairs below the parent diagonal
 * are not written, except at level l0, whose blocks all go into the final dense
 * block (parent clusters of level l0 - 1).  *count receives the number of
 * records; with out == NULL only *count is written; H2_ERR_ARG if cap < 7 *
 * records or level lies outside [l0, L]. */
h2_status h2_merge_schedule(const double* points, int64_t n, double h, int32_t leaf, double eta, int32_t level,
                            int64_t* out, int64_t cap, int64_t* count);

/* Per-level statistics after h2_factor, written as rows of int64:
 *   level, clusters, sum n, max n, sum k, max k, sum k~, max k~, min k~, eliminated.
 * rows_cap is the number of rows out can hold; *rows receives the count.
 * The final dense block is reported as one more row with level = l0 - 1. */
h2_status h2_stats(h2_handle H, int64_t* out, int32_t rows_cap, int32_t* rows);

/* Milliseconds of each factored level of the last h2_factor (its Steps 0-3 for
 * every colour, the flush of its pending Schur updates and its merge into the
 * parent level, eqs. 20-23), one value per row of h2_stats in the same order,
 * the final dense LU last; HIP events on the factorization's stream.  cap is
 * the number of doubles ms can hold (ms may be NULL to query *count). */
h2_status h2_level_timing(h2_handle H, double* ms, int32_t cap, int32_t* count);

/* Rank decisions of the last build/factor as (level, cluster, k, k~) int32
 * quadruples for every nonempty cluster of every factored level, finest level
 * first; this array (length 4 * *count) is also the forced_ranks format:
 * passing it back pins both the construction rank k and the factor rank k~
 * of each listed cluster.  cap is in quadruples. */
h2_status h2_forced_ranks_layout(h2_handle H, int32_t* out, int64_t cap, int64_t* count);

/* Timing (milliseconds) of the phases of the last h2_factor, measured with
 * HIP events on its stream: out[0] total, out[1] basis update and
 * projection (Steps 0-2), out[2] partial LU and panels, out[3] Schur
 * updates (eq. 12), out[4] level merges, out[5] final LU; n_out >= 6.
 * With n_out >= 10 the algorithmic ledger follows, computed from the actual
 * ranks: out[6] Schur flops (4 r ((sum m_a)^2 + sum m_a^2) per eliminated
 * cluster: the blocks (a, b) with a <= b of its partners, complex), out[7] number of Schur launches (updates are deferred and flushed
 * into a block just before its row or column cluster is processed, and at the
 * end of the level), out[8] flops of the whole factorization, out[9] Schur
 * bytes (each flushed block read and written once per flush, each panel slice
 * read once per update term).  The ledger is computed on the first call after
 * a factorization. */
h2_status h2_factor_timing(h2_handle H, double* out, int32_t n_out);

/* Per-kernel timing of later factorizations (enable != 0): the factorization
 * records HIP events around each kernel family of every colour on its stream
 * (a few hundred extra events per factorization, so leave it off where the
 * factorization itself is timed).  Default: off.  Diagnostics only. */
h2_status h2_set_kernel_timing(h2_handle H, int32_t enable);

/* Roofline ledger per kernel family of the last h2_factor, from its actual
 * ranks (complex multiply-add = 8 flops; bytes count what the operation must
 * move through HBM, each operand read and each result written once).
 * Families f = 0..7: Step 0 Gram of the fill-ins (eq. 16), Step 0 complement,
 * eigenvectors and Q~ (eqs. 17-19; latency-bound), Step 2 projections
 * (eqs. 5-8), partial LU with the triangular inverses (eqs. 9-11), the C and R
 * panels (eqs. 12-13), Schur updates (eq. 12), level merges (eqs. 20-23),
 * final dense LU.  out[3f] = milliseconds (summed HIP event intervals; -1 when
 * the factorization ran without h2_set_kernel_timing; the Schur, merge and
 * final LU intervals are always measured), out[3f+1] = flops,
 * out[3f+2] = bytes.  out[24] = bytes one right-hand side's forward and
 * backward sweeps must read (Q~ twice, L^-1 P, U^-1, the C and R panels, the
 * final block's L and U factors); out[25] = bytes one H^2 matvec must read (near blocks,
 * expanded bases, couplings).  out[26] (when n_out >= 27) = the fraction of
 * the Schur flops whose cluster passed the mixed form's FP32 test (0 for
 * FP64; a flush still runs a block's FP32-safe terms in FP64 when they carry
 * fewer than 64 contraction columns).  n_out >= 26; H2_ERR_STATE before
 * h2_factor. */
h2_status h2_kernel_ledger(h2_handle H, double* out, int32_t n_out);

#ifdef __cplusplus
}
#endif

#endif /* H2MI_H */
