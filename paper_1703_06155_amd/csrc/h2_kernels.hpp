// Device-side data views and kernel launchers (host interface of h2_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <utility>
#include <vector>

namespace h2 {

// Operand access modes: element (i, k) of op(A) / (k, j) of op(B).
enum Op : int { OP_N = 0, OP_T = 1, OP_C = 2, OP_R = 3 };  // R = conjugate, not transposed
// Epilogue of a tile: C = acc, C += acc, C -= acc.
enum ProjSel { PJ_ALL = 0, PJ_OFFDIAG = 1, PJ_DIAG = 2 };  // which blocks a projection launch handles
enum StoreMode : int { ST_SET = 0, ST_ADD = 1, ST_SUB = 2 };

// Geometry and kernel constants of the VIE matrix Z = A D^-1 (tree order).
struct GeomView {
  const double* pts;       // N x 3, tree order
  const double* chi;       // N, tree order
  const int32_t* leafid;   // N: leaf cluster of each tree-ordered point
  int64_t N;
  int L;
  double k, h;
  double diag_re_c, diag_im_c;  // self term c = (1 + jka) e^{-jka} - 1
  double k2h3;                  // k^2 h^3
};

// One factorization level; every array is indexed by cluster (nc entries),
// slot, or partner-list position.  Dimensions written during the level (kt)
// are read back by later kernels of the same level on the device.
struct LevelView {
  int nc;
  const int32_t* n;        // current size n_i
  const int32_t* k;        // basis columns k_i
  int32_t* kt;             // k~_i (Step 0 result)
  const int32_t* colour;
  const double* nu;        // construction sigma_1
  const int32_t* forced;   // forced k~ or -1 (nullable)
  double eps_fill;
  // blocks ("slots"): inadmissible pairs and fill-receiving admissible pairs
  const int64_t* slot_off;
  const int32_t* slot_a;
  const int32_t* slot_b;
  double2* slots;
  int nnear;               // slots [0, nnear) are inadmissible blocks, the rest fill-receiving blocks;
                           // one slot per unordered pair (slot_a <= slot_b), block (b, a) = its transpose
  const int32_t* diag_slot;
  // inadmissible partners N+(i) (incl. i), CSR
  const int32_t* np_ptr;
  const int32_t* np_cl;
  const int32_t* np_srow;  // code of block (i, a): slot, or ~slot when stored as (a, i)
  const int32_t* np_scol;  // code of block (a, i)
  const int32_t* np_off;   // offset of a inside the panels (sum of n over earlier partners)
  // fill partners (admissible / ancestor-admissible pairs reached by fill-ins), CSR
  const int32_t* fp_ptr;
  const int32_t* fp_cl;
  const int32_t* fp_srow;  // code of block (i, b)
  // per-cluster storage
  const int64_t* q_off;  double2* Q;     // Q~ (n x n), kept-first: [B B_add B~perp]
  const int64_t* b_off;  double2* B;     // B (n x k)
  const int64_t* bp_off; double2* Bp;    // B_perp (n x (n-k))
  const int64_t* lu_off; double2* LU;    // L^-1 P (rmax x rmax) then U^-1 (rmax x rmax)
  const int64_t* cp_off; double2* CP;    // C panel (prow x rmax)
  const int64_t* rp_off; double2* RP;    // R panel (rmax x prow)
  const int32_t* prow;                   // sum of n_a over N+(i)
  const int64_t* w_off;  double2* W;     // workspace: H (n x n), X (n x d), G' (d x d), U' (d x d)
  int32_t* flags;                        // [0]: 1 + cluster of a zero pivot
  double* margins;                       // per cluster (sigma_p / tau, sigma_{p+1} / tau)
  unsigned long long* pmax;              // 4 per cluster: max |C|, max |R|, max |input block| (double bits), unused
};

// Per-colour task lists (device arrays).
struct ColourTasks {
  const int32_t* cl; int ncl;            // clusters of the colour
  const int32_t* pj_slot; const int64_t* pj_toff; int npj;   // projection slots, temp offsets
  const int32_t* sc_slot; const int32_t* sc_cptr; const int32_t* sc_i; const int32_t* sc_ja;
  const int32_t* sc_jb; int nsc;          // Schur targets and their contributions
  const int32_t* sc_sp;                   // per task {chunk, chunks, chunks of earlier groups, group}
  const int32_t* sc_gtask; int ngrp;      // split groups: first task of each
  const int32_t* sc_gbase;                // split groups: first 64 x 64 partial tile of each
  double2* sc_part;                       // partial tiles of split tasks
  const int32_t* pn_i; const int32_t* pn_ja; int npn;          // panel tasks (i, partner pos)
  const int32_t* sv_cl; const int32_t* sv_cptr; const int32_t* sv_i; const int32_t* sv_ja;
  int nsv;                                // solve gather targets and contributions
  int colour;
  int tiles;                              // 64-wide tiles per block side (ceil(max n / 64))
};

// One problem's share of a launch that serves several independent problems: the
// launch's workgroups are dealt to the entries in order, entry e taking
// gx * gy * gz workgroups from `first` on, laid out as the grid (gx, gy, gz) the
// problem's own launch would use.  buf / aux / i0 carry the kernel's per-problem
// arguments (work space pointer and stride, phase, side or size bound).
struct BatchEntry {
  LevelView v;
  ColourTasks c;
  double2* buf;
  int64_t aux;
  int32_t i0;
  int32_t gx, gy, gz;
  int32_t first;
};

// Kernels that run as one launch over several problems' entries (the same
// bodies as the problems' own launches; the entries' grids and arguments follow
// the matching single-problem launcher).
enum BatchKernel : int {
  BK_SCHUR_FP64, BK_SCHUR_MIXED, BK_SCHUR_REDUCE, BK_GRAM_FILL, BK_GRAM_FILL_REDUCE, BK_XFORM,
  BK_STEP0_1, BK_STEP0_2, BK_STEP0_4, BK_STEP0_8, BK_PROJ, BK_PROJ_MIXED, BK_PROJ_FUSED, BK_PROJ_FUSED_MIXED,
  BK_LU_REG, BK_LU_BIG, BK_PANELS
};
// entries: device array of ne entries sorted by `first`; blocks = total workgroups
void launch_batched(int kernel, const BatchEntry* entries, int ne, int blocks, hipStream_t st);
// The stages of one colour of a level, in launch order (each depends on the previous).
enum BatchStage : int {
  BS_SCHUR, BS_SCHUR_REDUCE, BS_GRAM, BS_GRAM_REDUCE, BS_XFORM0, BS_XFORM1, BS_STEP0, BS_XFORM2, BS_PROJ0,
  BS_PROJ1, BS_LU, BS_PANELS, BS_COUNT
};
// Appends the (kernel, entry) pairs one problem contributes to a stage (mixed: the
// mixed form's projections; mixed_flush: its FP32-routing Schur flush): buf / aux
// are its work space and stride (Gram partials, eigen-solver, projection temp or
// LU scratch), i0 its largest eliminated dimension (Step 0, LU); the grids follow
// the single-problem launchers.
void batch_stage_entries(int stage, const LevelView& v, const ColourTasks& c, bool mixed, bool mixed_flush,
                         double2* buf, int64_t aux, int i0, std::vector<std::pair<int, BatchEntry>>& out);

// One problem's share of a shared sweep launch (forward or backward sweep of one
// colour, Algs. 5-6): the per-problem arguments of the single-problem kernels and
// the same local grid, placed at workgroup `first` of the shared grid.
struct SweepEntry {
  LevelView v;
  ColourTasks c;
  double2* vec;
  const int64_t* voff;
  int64_t ldv;
  double2* part;
  double2* scratch;
  int32_t nrhs, adj, nsplit;
  int32_t gx, gy, gz;
  int32_t first;
};
enum SweepKernel : int {
  SK_SW_FWD_LOCAL, SK_SW_FWD_GATHER, SK_SW_BWD_PARTIAL, SK_SW_BWD_LOCAL,
  SK_SV_FWD_LOCAL, SK_SV_FWD_GATHER, SK_SV_BWD_PARTIAL, SK_SV_BWD_LOCAL
};
// stages of one colour: forward local then gather; backward partial sums then local
enum SweepStage : int { SS_FWD_LOCAL, SS_FWD_GATHER, SS_BWD_PARTIAL, SS_BWD_LOCAL };
// The (kernel, entry) pairs one problem's colour contributes to a sweep stage; grids
// as launch_sweep_fwd / launch_sweep_bwd.
void sweep_stage_entries(int stage, const LevelView& v, const ColourTasks& c, double2* vec, const int64_t* voff,
                         int64_t ldv, int nrhs, int adj, double2* part, int nsplit, double2* scratch,
                         std::vector<std::pair<int, SweepEntry>>& out);
void launch_sweep_batched(int kernel, const SweepEntry* entries, int ne, int blocks, hipStream_t st);

// Generic host-resolved batched GEMM task: C (op)= op(A) op(B).
struct GemmTask {
  const double2* A;
  const double2* B;
  double2* C;
  int64_t lda, ldb, ldc;
  int32_t m, n, K;
  int32_t opA, opB, mode;
};

// ---- construction ----
void launch_near_blocks(const GeomView& g, const int32_t* pr, const int32_t* pc, const int64_t* off,
                        const int64_t* rs, const int32_t* rn, const int64_t* cs, const int32_t* cn,
                        int npairs, double2* out, hipStream_t st);
void launch_leaf_gram(const GeomView& g, const uint32_t* mask, int ncl, int level, const int64_t* cstart,
                      const int32_t* csize, int64_t kchunk, int nchunks, double2* part, int64_t stride,
                      const int64_t* goff, int ntr, hipStream_t st);
void launch_gram_reduce(const double2* part, double2* out, const int64_t* off, const int32_t* sz,
                        int ncl, int nchunks, int64_t stride, hipStream_t st);
void launch_proj_rows(const GeomView& g, const uint32_t* mask, int level, int nch, const int64_t* cstart,
                      const int32_t* csize, const int32_t* ck, const int64_t* voff, const double2* V,
                      const int64_t* yoff, const int32_t* yld, double2* Y, int64_t col0, int ncols,
                      int ntr, hipStream_t st);
void launch_gram_acc(int ncl, const int32_t* dim, const int64_t* yoff, const double2* Y, int ncols,
                     const int64_t* goff, double2* G, int ntr, hipStream_t st);
void launch_coupling_x(const GeomView& g, int npairs, int ntr, int ntc, const int32_t* pt, const int32_t* ps,
                       const int64_t* tstart, const int32_t* tsz, const int32_t* tk, const int64_t* voff,
                       const double2* V, const int64_t* xoff, double2* X, hipStream_t st);
// one GEMM task passed by value: a tile per workgroup, no host synchronisation
void launch_gemm_one(const GemmTask& T, hipStream_t st);
void launch_gemm_batched(const GemmTask* tasks, const int32_t* tile_task, const int32_t* tile_rc,
                         int ntiles, hipStream_t st);
void launch_transpose_copy(const GemmTask* tasks, int ntasks, hipStream_t st);

// Batched Hermitian eigensolver (cyclic Jacobi): G (d x d, ld d) per problem at
// goff; writes eigenvalues descending (lam at loff) and eigenvectors (U at uoff,
// ld d).  rel != 0: rotate until |g_pq| <= 4e-16 sqrt(|g_pp g_qq|) (relative
// accuracy), else until |g_pq| <= 1e-15 ||G||_F.
void launch_jacobi(int nprob, const int32_t* dims, const int64_t* goff, double2* G, const int64_t* uoff,
                   double2* U, const int64_t* loff, double* lam, int rel, double2* scratch,
                   const int64_t* soff, hipStream_t st);

// ---- factorization ----
constexpr int GRAM_SPLIT = 64;  // partial sums of the Step 0 Gram (several workgroups per CU at ~13 clusters a colour)
// Mixed form: a cluster's Schur terms run in FP32 when sqrt(r) max|C| max|R| is
// at most this multiple of the largest entry of the blocks they were formed from.
constexpr double F32_KAPPA = 8.0;
constexpr int STEP0_DMAX = 512;  // largest cluster complement n - k (Step 0, Step 1, partial LU)
constexpr int SCHUR_CHUNK_TERMS = 10;  // Schur tasks with more terms are split along the contraction
constexpr int LU_LDS_MAX = 96;  // Step 3a keeps F in LDS up to this many rows, else in scratch
void launch_householder_perp(const LevelView& v, int nc, hipStream_t st);
void launch_gram_fill(const LevelView& v, const ColourTasks& c, double2* part, int64_t pstride, hipStream_t st);
void launch_xform(const LevelView& v, const ColourTasks& c, int phase, hipStream_t st);
void launch_step0_eig(const LevelView& v, const ColourTasks& c, double2* scratch, int dm, hipStream_t st);
void launch_proj(const LevelView& v, const ColourTasks& c, double2* temp, int side, bool mixed, hipStream_t st);
void launch_proj_fused(const LevelView& v, const ColourTasks& c, bool mixed, hipStream_t st);
void launch_lu(const LevelView& v, const ColourTasks& c, double2* scratch, int rm, hipStream_t st);
void launch_panels(const LevelView& v, const ColourTasks& c, hipStream_t st);
void launch_schur(const LevelView& v, const ColourTasks& c, bool mixed, hipStream_t st);

// Level end: parent blocks from children (copy of kept k~ x k~ parts, padded
// couplings plus fills, carried fills).
struct MergeTask {
  int64_t dst;         // element offset of the destination sub-block origin
  int64_t ldd;
  int32_t kind;        // 0 near slot, 1 admissible (coupling + optional fill), 2 fill slot
  int32_t slot;        // source slot (kinds 0, 2) or fill slot / -1 (kind 1)
  int32_t ca, cb;      // child clusters
  int64_t soff;        // coupling offset (kind 1)
  int32_t ska, skb;    // coupling dims (construction ranks)
  int32_t tr;          // source slot holds (cb, ca): read transposed
};
void launch_zero(double2* p, int64_t n, hipStream_t st);
// One piece of a staged host array: `bytes` (a multiple of 4, at most STAGE_PIECE)
// at offset `src` of the staging buffer go to `dst`; src and dst are 16-byte aligned.
constexpr int64_t STAGE_PIECE = 16384;
struct CopySeg {
  int64_t src;
  int64_t bytes;
  void* dst;
};
void launch_scatter_segments(const char* base, const CopySeg* segs, int nseg, hipStream_t st);
void launch_copy_blocks(const double2* src, const int64_t* src_off, double2* dst, const int64_t* dst_off,
                        const int64_t* len, int nb, hipStream_t st);
void launch_merge(const LevelView& v, const MergeTask* t, int nt, const double2* S, double2* dst,
                  hipStream_t st);
void launch_parent_basis(int np, const int32_t* pn, const int32_t* pk, const int32_t* k1,
                         const int32_t* k2, const int32_t* off1, const int64_t* toff, const double2* T,
                         const int64_t* boff, double2* B, hipStream_t st);

// Dense LU with partial pivoting of one panel (rows j0.., 64 columns) of an
// n x n column-major matrix: factorizes in place, records pivots, swaps rows
// across the whole matrix, writes the explicit inverse of the unit-lower
// diagonal block (64 x 64, ld 64) to linv.
void launch_dense_panel(double2* A, int64_t n, int64_t j0, int32_t* piv, double2* linv, int32_t* flag,
                        hipStream_t st);
void launch_tri_inv_upper(const double2* A, int64_t n, int w, double2* Uinv, hipStream_t st);
void launch_apply_perm_cols(double2* X, int64_t n, const int32_t* piv, hipStream_t st);
// Solves with the final block's LU factors: row gather / scatter by a permutation
// (nrhs columns, leading dimension ld) and one 64-row block step of a
// right-looking triangular solve (mode 0: L forward, 1: U backward, 2: U^H
// forward, 3: L^H backward; D = the inverse of the block's diagonal block; the
// block's result goes to y, the other rows of x are updated in place).
void launch_dense_perm(const double2* in, double2* out, const int32_t* perm, int64_t n, int nrhs, int64_t ld,
                       int scatter, hipStream_t st);
void launch_dense_trsv_step(const double2* A, int64_t n, int64_t j0, int w, const double2* D, double2* x,
                            double2* y, int64_t ld, int nrhs, int mode, hipStream_t st);

// ---- sweeps (nrhs columns; per-level vectors with leading dimension ldv) ----
constexpr int BWD_SPLIT = 8;   // partial sums of the backward gather (many right-hand sides)
constexpr int SV_SPLIT = 32;   // partial sums of the backward gather (matrix-vector sweeps)
constexpr int SMALL_RHS = 4;   // up to this many right-hand sides the sweeps use matrix-vector kernels
void launch_sweep_fwd(const LevelView& v, const ColourTasks& c, double2* vec, const int64_t* voff, int64_t ldv,
                      int nrhs, int adj, double2* scratch, hipStream_t st);
void launch_sweep_bwd(const LevelView& v, const ColourTasks& c, double2* vec, const int64_t* voff, int64_t ldv,
                      int nrhs, int adj, double2* part, int nsplit, double2* scratch, hipStream_t st);
void launch_dense_apply(const double2* M, int64_t n, const double2* x, double2* y, int64_t ld, int nrhs,
                        int conj_trans, hipStream_t st);
void launch_vmerge(int np, const int32_t* kt, const int64_t* cvoff, const int64_t* pvoff, int64_t ldc,
                   int64_t ldp, int nrhs, double2* cvec, double2* pvec, int up, const int32_t* nonempty,
                   hipStream_t st);
void launch_permute_in(const double2* x, int64_t ldx, const int64_t* perm, const double* scale,
                       int conj_in, int64_t N, int nrhs, double2* out, int64_t ldo, hipStream_t st);
void launch_permute_out(const double2* in, int64_t ldi, const int64_t* perm, const double* scale,
                        int conj_out, int64_t N, int nrhs, double2* y, int64_t ldy, int accumulate,
                        hipStream_t st);
void launch_dense_gemv(const double2* M, int64_t n, const double2* x, double2* y, int64_t ld, int nrhs,
                       int conj_trans, hipStream_t st);

// ---- fixed device scratch of the allocation-free solve ----
// 64 MiB per device, held from the first use until the process ends.
constexpr int64_t NOALLOC_SCRATCH_ELEMS = (int64_t(64) << 20) / 16;
// Device address of the scratch array on the current device (looked up once per
// device with hipGetSymbolAddress); NULL with *err set when the lookup fails.
double2* noalloc_scratch(hipError_t* err);

// ---- H^2 matrix-vector product ----
void launch_near_mv(int nc, const int32_t* rptr, const int32_t* rcol, const int64_t* boff,
                    const double2* blocks, const int64_t* cstart, const int32_t* csize, const double2* x,
                    double2* y, int64_t ld, int nrhs, hipStream_t st);
void launch_basis_mv(int nc, const int32_t* rows, const int32_t* cols, const int64_t* moff,
                     const double2* M, const int64_t* xoff, const double2* x, const int64_t* yoff,
                     double2* y, int64_t ldx, int64_t ldy, int nrhs, int trans, int accumulate,
                     hipStream_t st);
void launch_coupling_mv(int nc, const int32_t* rptr, const int32_t* rcol, const int64_t* soff,
                        const int32_t* kr, const int32_t* kc, const double2* S, const int64_t* xoff,
                        const double2* x, const int64_t* yoff, double2* y, int64_t ld, int nrhs,
                        hipStream_t st);

// ---- refinement helpers ----
void launch_residual(const double2* b, int64_t ldb, const double2* ax, int64_t lda, double2* r, int64_t ldr,
                     int64_t N, int nrhs, hipStream_t st);
void launch_axpy_cols(const double2* d, int64_t ldd, double2* x, int64_t ldx, int64_t N, int nrhs,
                      hipStream_t st);
void launch_col_norms(const double2* x, int64_t ld, int64_t N, int nrhs, double* out, hipStream_t st);
void launch_contrast_grad(const double2* x, const double2* g, const double2* lam, int64_t ld, int nrhs,
                          const double* chi, int64_t N, double* grad, hipStream_t st);

}  // namespace h2
