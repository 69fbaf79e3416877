// Host orchestration and C ABI of libh2mi.
//
// h2_build: structure (tree, partition, colouring), task plans, and the H^2
//   construction on the device (far-field Grams -> Hermitian eigensolver ->
//   nested bases, couplings, inadmissible leaf blocks).
// h2_factor: Alg. 1 level by level; within a level clusters of one colour
//   take Steps 0-3 together; one host synchronisation per level reads the
//   ranks k~ that size the next level.
// h2_solve / h2_solve_adjoint / h2_matvec: the sweeps of Sec. IV, their
//   adjoint, and the H^2 product, all on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <array>
#include <climits>
#include <iterator>
#include <limits>
#include <tuple>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <atomic>
#include <exception>
#include <system_error>
#include <memory>
#include <mutex>
#include <thread>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/h2.h"
#include "h2_kernels.hpp"
#include "h2_structure.hpp"

namespace h2 {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

struct Fail {
  h2_status st;
  std::string msg;
};

[[noreturn]] static void fail(h2_status st, const std::string& m) { throw Fail{st, m}; }

#define HIPCHK(x)                                                                      \
  do {                                                                                 \
    hipError_t e_ = (x);                                                               \
    if (e_ != hipSuccess) {                                                            \
      if (e_ == hipErrorOutOfMemory) fail(H2_ERR_OOM, std::string("device allocation: ") + #x); \
      fail(H2_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_));             \
    }                                                                                  \
  } while (0)

// ---------------------------------------------------------------------------
// device memory
// ---------------------------------------------------------------------------
// Where device memory comes from: the caller's allocator when h2_build was given
// one (h2_options.alloc / free / alloc_ctx), else hipMalloc / hipFree.  Every call
// on a handle runs with that handle's allocator and stream installed for the
// calling thread (AllocScope), so buffers allocated anywhere inside the call take
// it; each buffer remembers the allocator it came from.
struct DevAllocator {
  void* (*alloc)(size_t bytes, void* stream, void* ctx) = nullptr;
  void (*free)(void* p, void* stream, void* ctx) = nullptr;
  void* ctx = nullptr;
};
static thread_local const DevAllocator* t_alloc = nullptr;
static thread_local hipStream_t t_stream = nullptr;
static thread_local bool t_device_idle = false;  // set while h2_destroy frees after one device-wide wait

struct AllocScope {
  const DevAllocator* prev_a;
  hipStream_t prev_s;
  AllocScope(const DevAllocator* a, hipStream_t s) : prev_a(t_alloc), prev_s(t_stream) {
    t_alloc = (a && a->alloc && a->free) ? a : nullptr;
    t_stream = s;
  }
  ~AllocScope() {
    t_alloc = prev_a;
    t_stream = prev_s;
  }
};

template <typename T>
struct DArr {
  T* p = nullptr;
  size_t n = 0;    // elements in use
  size_t cap = 0;  // elements allocated
  const DevAllocator* from = nullptr;  // caller's allocator that provided p (NULL: hipMalloc)
  DArr() = default;
  DArr(const DArr&) = delete;
  DArr& operator=(const DArr&) = delete;
  DArr(DArr&& o) noexcept : p(o.p), n(o.n), cap(o.cap), from(o.from) {
    o.p = nullptr;
    o.n = o.cap = 0;
    o.from = nullptr;
  }
  DArr& operator=(DArr&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      cap = o.cap;
      from = o.from;
      o.p = nullptr;
      o.n = o.cap = 0;
      o.from = nullptr;
    }
    return *this;
  }
  ~DArr() { release(); }
  void release() {
    if (p) {
      if (from) {
        // the caller's allocator may hand the memory out again at once: the handle's
        // work on it must be done.  Calls on one handle are ordered on the device (the
        // same stream, or the caller synchronises), so the current stream covers them;
        // a device-wide wait here would also stall every other handle of a batch.
        if (!t_device_idle) (void)hipStreamSynchronize(t_stream);
        from->free(p, t_stream, from->ctx);
      } else {
        (void)hipFree(p);
      }
    }
    p = nullptr;
    from = nullptr;
    n = cap = 0;
  }
  // Keeps the existing allocation when it is large enough: buffers that live
  // in the handle are reused by the next factorization instead of being
  // mapped again (mapping tens of GB costs seconds).  Contents are undefined.
  void alloc(size_t cnt) {
    if (cnt == 0) cnt = 1;
    if (p && cap >= cnt) {
      n = cnt;
      return;
    }
    release();
    if (t_alloc) {
      p = static_cast<T*>(t_alloc->alloc(cnt * sizeof(T), t_stream, t_alloc->ctx));
      if (!p) fail(H2_ERR_OOM, "the caller's allocator returned NULL for " + std::to_string(cnt * sizeof(T)) + " bytes");
      from = t_alloc;
      n = cap = cnt;
      return;
    }
    const hipError_t e = hipMalloc((void**)&p, cnt * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      size_t fr = 0, tot = 0;
      (void)hipGetLastError();
      (void)hipMemGetInfo(&fr, &tot);
      fail(e == hipErrorOutOfMemory ? H2_ERR_OOM : H2_ERR_DEVICE,
           "device allocation of " + std::to_string(cnt * sizeof(T) >> 20) + " MiB failed (" +
               std::to_string(fr >> 20) + " of " + std::to_string(tot >> 20) + " MiB free)");
    }
    n = cap = cnt;
  }
  // blocking: the host vector may be a temporary.  An allocation that is large
  // enough is reused, so device pointers taken from it stay valid.
  void upload(const std::vector<T>& v, hipStream_t st) {
    alloc(v.size());
    if (!v.empty()) {
      HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));
    }
  }
};

// Small host arrays of one factorization step (offsets, sizes, task lists) gathered
// in one pinned buffer, copied to the device at once and spread to their arrays by
// one kernel: no host wait per array.  Owned by a handle, grown on demand.  The
// pinned buffer is rewritten only after the copy out of it has finished.
struct Stager {
  std::vector<char> buf;
  std::vector<CopySeg> segs;
  char* host = nullptr;
  size_t host_cap = 0;
  DArr<char> dev;
  hipEvent_t copied = nullptr;
  Stager() = default;
  Stager(const Stager&) = delete;
  Stager& operator=(const Stager&) = delete;
  ~Stager() {
    if (copied) {
      (void)hipEventSynchronize(copied);
      (void)hipEventDestroy(copied);
    }
    if (host) (void)hipHostFree(host);
  }
  static size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }
  // d is sized for v now; its contents arrive with the next flush()
  template <typename T>
  void put(DArr<T>& d, const std::vector<T>& v) {
    static_assert(sizeof(T) % 4 == 0, "staged elements are whole 4-byte words");
    d.alloc(v.size());
    if (v.empty()) return;
    const size_t off = align16(buf.size()), bytes = v.size() * sizeof(T);
    if (reinterpret_cast<uintptr_t>(d.p) % 16 != 0) fail(H2_ERR_INTERNAL, "staged device array not 16-byte aligned");
    buf.resize(off + bytes);
    std::memcpy(buf.data() + off, v.data(), bytes);
    for (size_t o = 0; o < bytes; o += STAGE_PIECE)
      segs.push_back({(int64_t)(off + o), (int64_t)std::min<size_t>(STAGE_PIECE, bytes - o),
                      reinterpret_cast<char*>(d.p) + o});
  }
  void flush(hipStream_t st) {
    if (segs.empty()) return;
    const size_t toff = align16(buf.size()), total = toff + segs.size() * sizeof(CopySeg);
    buf.resize(total);
    std::memcpy(buf.data() + toff, segs.data(), segs.size() * sizeof(CopySeg));
    if (copied) HIPCHK(hipEventSynchronize(copied));
    else HIPCHK(hipEventCreateWithFlags(&copied, hipEventDisableTiming));
    if (total > host_cap) {
      if (host) HIPCHK(hipHostFree(host));
      host = nullptr;
      host_cap = 0;
      const size_t cap = std::max(total, (size_t)1 << 20);
      if (hipHostMalloc((void**)&host, cap, hipHostMallocDefault) != hipSuccess || !host) {
        host = nullptr;
        (void)hipGetLastError();
        fail(H2_ERR_OOM, "pinned host allocation of " + std::to_string(cap) + " bytes failed");
      }
      host_cap = cap;
    }
    std::memcpy(host, buf.data(), total);
    dev.alloc(total);
    HIPCHK(hipMemcpyAsync(dev.p, host, total, hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(copied, st));
    launch_scatter_segments(dev.p, reinterpret_cast<const CopySeg*>(dev.p + toff), (int)segs.size(), st);
    buf.clear();
    segs.clear();
  }
};

// ---------------------------------------------------------------------------
// plans
// ---------------------------------------------------------------------------
struct ColourPlan {
  std::vector<int32_t> cl, pj_slot, sc_slot, sc_cptr, sc_i, sc_ja, sc_jb, pn_i, pn_ja, sv_cl, sv_cptr, sv_i,
      sv_ja;
  // Schur tasks with many terms are split along the contraction into chunks of at
  // most SCHUR_CHUNK_TERMS terms (or the level's setting): per task {chunk, chunks, chunks of earlier groups,
  // group} ({-1, 1, 0, 0} when whole); nps chunks and ngrp groups in all
  std::vector<int32_t> sc_sp, sc_gtask;
  std::vector<int32_t> sc_gbase;  // per group, set per factorization: first 64 x 64 partial tile
  int nps = 0, ngrp = 0;
  // the same flush unsplit (one task per block), used when the partial tiles do not fit
  std::vector<int32_t> sc_slot_u, sc_cptr_u, sc_sp_u;
  DArr<int32_t> d_cl, d_pj_slot, d_sc_slot, d_sc_cptr, d_sc_i, d_sc_ja, d_sc_jb, d_pn_i, d_pn_ja, d_sv_cl,
      d_sv_cptr, d_sv_i, d_sv_ja, d_sc_sp, d_sc_gtask, d_sc_slot_u, d_sc_cptr_u, d_sc_sp_u, d_sc_gbase;
  DArr<int64_t> d_pj_toff;
  std::vector<int64_t> pj_toff;
  int64_t temp_elems = 0;
};

struct MergeSrc {  // rank-independent part of a merge task
  int32_t pslot;   // parent slot (or parent pair index for the final dense block)
  int32_t ci, dj;  // which child of the parent row / column cluster
  int32_t kind, slot, adm;  // kind 0 near / 1 admissible (adm = pair index) / 2 fill
  int32_t ca, cb;
  int32_t tr;      // the source slot stores (cb, ca): read it transposed
};

struct LevelPlan {
  int l = 0, nc = 0, ncol = 0, nnear = 0, nslot = 0;
  std::vector<int32_t> colour, nonempty, slot_a, slot_b, diag_slot;
  std::vector<int32_t> np_ptr, np_cl, np_srow, np_scol;
  std::vector<int32_t> fp_ptr, fp_cl, fp_srow;
  std::vector<int32_t> near_src;  // near slot -> index in S.near[l]
  std::vector<ColourPlan> cols;
  ColourPlan fin;                 // Schur updates still pending when the level ends
  std::vector<MergeSrc> merge;  // into level l-1 (slots) or the final dense block
  // device copies of the static lists
  DArr<int32_t> d_colour, d_nonempty, d_slot_a, d_slot_b, d_diag_slot, d_np_ptr, d_np_cl, d_np_srow, d_np_scol,
      d_fp_ptr, d_fp_cl, d_fp_srow;
  // row-wise slot lookup: for cluster a, (b, slot) sorted by b
  std::vector<int32_t> rl_ptr, rl_b, rl_slot;
  // Code of block (a, b): the slot index when stored as (a, b) (a <= b), or
  // ~slot when it is the transpose of the stored block (b, a).
  // INT32_MIN when the pair has no slot.
  int slot_code(int a, int b) const {
    const int s = (a <= b) ? slot_of(a, b) : slot_of(b, a);
    if (s < 0) return INT32_MIN;
    return (a <= b) ? s : ~s;
  }
  int slot_of(int a, int b) const {
    auto beg = rl_b.begin() + rl_ptr[a], end = rl_b.begin() + rl_ptr[a + 1];
    auto it = std::lower_bound(beg, end, b);
    if (it == end || *it != b) return -1;
    return rl_slot[it - rl_b.begin()];
  }
};

// construction data of one level (l0 <= l <= L)
struct BuildLevel {
  std::vector<int32_t> k;       // ranks
  std::vector<double> nu;       // sigma_1 of the far-field row
  std::vector<double> margin;   // per cluster (sigma_k/thr, sigma_{k+1}/thr)
  std::vector<int64_t> boff;    // basis (leaf V: #t x k; non-leaf T: (k1+k2) x k)
  DArr<double2> basis;
  std::vector<int64_t> voff;    // expanded basis #t x k
  DArr<double2> V;
  std::vector<int64_t> soff;    // couplings for S.adm[l] (k_t x k_s)
  DArr<double2> S;
  DArr<int64_t> d_voff, d_soff;
  DArr<int32_t> d_k, d_rows;    // k per cluster, #t per cluster
  DArr<int32_t> d_cptr, d_ccol; // admissible CSR by row cluster (into S.adm order)
  DArr<int64_t> d_cstart, d_xoff;  // cluster starts (tree order), xhat offsets
  DArr<double> d_nu;
  DArr<double2> mv_x, mv_y;     // matvec work: x_hat, y_hat (ktot x nrhs)
  int64_t ktot = 0;             // sum of k
};

// factor data of one level (kept for the sweeps)
struct FactorLevel {
  std::vector<int32_t> n, kt, k;  // sizes, factor ranks k~, construction ranks
  int64_t ntot = 0;
  DArr<int32_t> d_n, d_k, d_kt, d_forced, d_np_off, d_prow, d_flags;
  DArr<int64_t> d_slot_off, d_q_off, d_b_off, d_bp_off, d_lu_off, d_cp_off, d_rp_off, d_w_off, d_voff;
  DArr<double> d_margins;
  DArr<double2> d_pmax;   // 4 unsigned 64-bit maxima per cluster (mixed form)
  DArr<double2> Q, LU, CP, RP, B;
  std::vector<int64_t> voff;
  LevelView view{};
  int tiles = 1;
  bool mixed_flush = false;  // the level's Schur flushes routed FP32-safe terms to FP32
};

}  // namespace h2

struct h2_ctx {
  h2::DevAllocator allocator;              // first member: outlives every buffer it provided
  h2::Structure S;
  int64_t N = 0;
  double k = 0, h = 0, eta = 0, eps = 0, eps_fill = 0;
  int leaf = 0, precision = H2_FP64;
  std::vector<double> chi_tree;
  std::vector<int32_t> forced_k, forced_kt;  // flattened per level: offset lvl_base[l]
  std::vector<int64_t> lvl_base;
  bool has_forced = false;
  // device geometry
  h2::DArr<double> d_pts, d_chi, d_scale_solve, d_scale_mat, d_chi_user;
  h2::DArr<int32_t> d_leafid;
  h2::DArr<int64_t> d_perm;
  h2::GeomView geom{};
  // plans and construction
  std::vector<h2::LevelPlan> plans;        // index L - l
  std::vector<h2::BuildLevel> build;       // index L - l
  h2::DArr<double2> near_orig;             // inadmissible leaf blocks (S.near[L] order)
  std::vector<int64_t> near_off;
  h2::DArr<int64_t> d_near_off, d_leaf_start;
  h2::DArr<int32_t> d_near_ptr, d_near_col, d_leaf_size, d_near_pr, d_near_pc;
  // factorization
  bool factored = false;
  std::vector<h2::FactorLevel> flev;       // index L - l
  h2::DArr<double2> slot_buf[2];           // block arenas of even / odd levels (index L - l)
  h2::DArr<double2> ws_bp, ws_w, ws_temp, ws_lu, ws_eig, ws_gram;  // per-level work space
  h2::DArr<double2> ws_scp;                                          // partial tiles of split Schur tasks
  h2::DArr<h2::MergeTask> ws_merge;
  int64_t nf = 0;
  std::vector<int32_t> final_off;          // per cluster of level l0-1
  h2::DArr<int64_t> d_final_off;           // the same (without the total), on the device
  // the sweeps as captured graphs, keyed by (nrhs, adjoint); they run on vtmp3 in place
  bool use_graph = false;
  hipStream_t cap_stream = nullptr;
  hipStream_t own_stream = nullptr;        // the handle's stream inside batched calls
  std::map<std::pair<int, int>, hipGraphExec_t> sweep_graphs;
  void drop_graphs() {
    for (auto& g : sweep_graphs) (void)hipGraphExecDestroy(g.second);
    sweep_graphs.clear();
  }
  ~h2_ctx() {
    drop_graphs();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (own_stream) (void)hipStreamDestroy(own_stream);
  }
  h2::DArr<double2> Zf;                    // final dense block, overwritten by its LU factors
  h2::DArr<double2> dl_linv, dl_uinv;       // inverses of the final LU's 64 x 64 diagonal blocks
  h2::DArr<int32_t> dl_piv, dl_flag, dl_perm;
  std::vector<double> timing;
  std::vector<double> ledger;              // [6] Schur flops, [7] Schur launches, [8] factor flops, [9] Schur bytes
  bool ledger_valid = false;
  // per kernel family of the last factorization: ms (HIP events), flops, bytes
  bool kernel_timing = false;
  std::vector<double> kernel_ms;           // 8 families (see h2_kernel_ledger); -1 = not measured
  std::vector<double> kernel_led;          // 3 per family + sweep bytes + matvec bytes
  double merge_elems = 0;                  // elements of the parent blocks the merges wrote
  // sweep workspace
  std::vector<h2::DArr<double2>> vbuf;
  h2::DArr<double2> vtmp, vtmp2, vtmp3, sw_scratch, sw_part;
  int vbuf_nrhs = 0;
  h2::DArr<double> d_norms;
  h2::DArr<double2> mv_in, mv_out;         // h2_matvec work vectors
  h2::DArr<double2> rf_b0, rf_r, rf_ax, rf_vt;  // refinement work vectors
  h2::DArr<double> rf_nb;
  h2::DArr<h2::GemmTask> gm_tasks;         // task lists of run_gemms (final dense LU)
  h2::DArr<int32_t> gm_tt, gm_rc;
  h2::DArr<int32_t> lv_k1, lv_k2, lv_off1; // per-level uploads of factor_impl
  h2::DArr<int64_t> lv_toff, lv_so, lv_do, lv_len;
  int stop = -1;                           // last factored level (l0 unless stopped early, Sec. III-C)
  std::vector<int64_t> split_below;        // per level: Schur flush split threshold in workgroups (-1: default)
  std::vector<int32_t> mixed_flush;        // per level, mixed form: 1 FP32-routing flush, 0 FP64 flush, -1 default rule
  std::vector<int32_t> schur_chunk;        // per level: terms per chunk of a split Schur task (<= 0: SCHUR_CHUNK_TERMS)
  h2::DArr<double2> fb_X, fb_Y;            // early stop: expanded bases and their products with couplings
  h2::DArr<int32_t> fb_n, fb_k, fb_k1, fb_k2, fb_off1;
  h2::DArr<int64_t> fb_toff, fb_xoff;
  h2::DArr<h2::BatchEntry> batch_entries;  // work items of shared launches when this handle leads a batch
  h2::DArr<h2::SweepEntry> sweep_entries;  // work items of shared sweep launches when it leads a batched solve
  h2::Stager stage;                        // per-level host arrays on their way to the device
  std::vector<std::vector<int64_t>> stats_rows;
  std::vector<double> level_ms;            // per stats row: ms of that level (Steps 0-3 and its merge) / final LU
};

namespace h2 {

static void build_plan_level(h2_ctx* H, int l, LevelPlan& P) {
  const Structure& S = H->S;
  P.l = l;
  P.nc = S.nclusters(l);
  const int nc = P.nc;
  P.colour.assign(S.colour[l].begin(), S.colour[l].end());
  P.ncol = S.ncolours[l];
  P.nonempty.resize(nc);
  for (int t = 0; t < nc; ++t) P.nonempty[t] = S.size[l][t] > 0;
  // near lists
  P.np_ptr.assign(nc + 1, 0);
  for (const Pair& p : S.near[l]) P.np_ptr[p.first + 1]++;
  for (int t = 0; t < nc; ++t) P.np_ptr[t + 1] += P.np_ptr[t];
  P.np_cl.resize(S.near[l].size());
  {
    std::vector<int32_t> fillp(P.np_ptr.begin(), P.np_ptr.end() - 1);
    for (const Pair& p : S.near[l]) P.np_cl[fillp[p.first]++] = p.second;
  }
  // Blocks are stored once per unordered pair {a, b} (a <= b): every state of
  // the factorization is complex symmetric (Z is, the projections act as a
  // congruence with Q~^H, and Schur complements of symmetric matrices stay
  // symmetric), so block (b, a) is the transpose of block (a, b).
  // Near slots: the pairs of S.near with a <= b, in S.near order.
  P.near_src.clear();
  std::vector<int64_t> nearkeys;
  for (size_t e = 0; e < S.near[l].size(); ++e) {
    const Pair& p = S.near[l][e];
    if (p.first > p.second) continue;
    P.near_src.push_back((int32_t)e);
    nearkeys.push_back((int64_t)p.first * nc + p.second);
  }
  P.nnear = (int)P.near_src.size();
  // Blocks touched by some cluster's Schur update: (a, b), a <= b, both near a
  // common cluster i.  Near is symmetric, so row a collects N(i) over i in N(a);
  // the rows come out in order and each row is sorted, so the keys are sorted.
  std::vector<int64_t> keys;
  {
    std::vector<char> mark(nc, 0);
    std::vector<int32_t> row;
    for (int a = 0; a < nc; ++a) {
      row.clear();
      for (int x = P.np_ptr[a]; x < P.np_ptr[a + 1]; ++x) {
        const int i = P.np_cl[x];
        for (int y = P.np_ptr[i]; y < P.np_ptr[i + 1]; ++y) {
          const int b = P.np_cl[y];
          if (b >= a && !mark[b]) {
            mark[b] = 1;
            row.push_back(b);
          }
        }
      }
      std::sort(row.begin(), row.end());
      for (int b : row) {
        keys.push_back((int64_t)a * nc + b);
        mark[b] = 0;
      }
    }
  }
  // remove near pairs from keys -> fill pairs
  std::vector<int64_t> nearsorted(nearkeys);
  std::sort(nearsorted.begin(), nearsorted.end());
  std::vector<int64_t> fillkeys;
  std::set_difference(keys.begin(), keys.end(), nearsorted.begin(), nearsorted.end(),
                      std::back_inserter(fillkeys));
  P.nslot = P.nnear + (int)fillkeys.size();
  P.slot_a.resize(P.nslot);
  P.slot_b.resize(P.nslot);
  for (int e = 0; e < P.nnear; ++e) {
    P.slot_a[e] = (int32_t)(nearkeys[e] / nc);
    P.slot_b[e] = (int32_t)(nearkeys[e] % nc);
  }
  for (size_t e = 0; e < fillkeys.size(); ++e) {
    P.slot_a[P.nnear + e] = (int32_t)(fillkeys[e] / nc);
    P.slot_b[P.nnear + e] = (int32_t)(fillkeys[e] % nc);
  }
  // row lookup
  P.rl_ptr.assign(nc + 1, 0);
  for (int s = 0; s < P.nslot; ++s) P.rl_ptr[P.slot_a[s] + 1]++;
  for (int t = 0; t < nc; ++t) P.rl_ptr[t + 1] += P.rl_ptr[t];
  {
    std::vector<std::pair<int32_t, int32_t>> tmp(P.nslot);
    std::vector<int32_t> fillp(P.rl_ptr.begin(), P.rl_ptr.end() - 1);
    for (int s = 0; s < P.nslot; ++s) tmp[fillp[P.slot_a[s]]++] = {P.slot_b[s], s};
    for (int t = 0; t < nc; ++t) std::sort(tmp.begin() + P.rl_ptr[t], tmp.begin() + P.rl_ptr[t + 1]);
    P.rl_b.resize(P.nslot);
    P.rl_slot.resize(P.nslot);
    for (int s = 0; s < P.nslot; ++s) {
      P.rl_b[s] = tmp[s].first;
      P.rl_slot[s] = tmp[s].second;
    }
  }
  P.np_srow.resize(P.np_cl.size());
  P.np_scol.resize(P.np_cl.size());
  P.diag_slot.assign(nc, -1);
  for (int i = 0; i < nc; ++i)
    for (int x = P.np_ptr[i]; x < P.np_ptr[i + 1]; ++x) {
      const int a = P.np_cl[x];
      P.np_srow[x] = P.slot_code(i, a);
      P.np_scol[x] = P.slot_code(a, i);
      if (a == i) P.diag_slot[i] = P.np_srow[x];
    }
  // fill partner lists: row i, non-near b, in either stored orientation
  P.fp_ptr.assign(nc + 1, 0);
  for (int s = P.nnear; s < P.nslot; ++s) {
    P.fp_ptr[P.slot_a[s] + 1]++;
    P.fp_ptr[P.slot_b[s] + 1]++;
  }
  for (int t = 0; t < nc; ++t) P.fp_ptr[t + 1] += P.fp_ptr[t];
  P.fp_cl.resize(P.fp_ptr[nc]);
  P.fp_srow.resize(P.fp_ptr[nc]);
  {
    std::vector<int32_t> fillp(P.fp_ptr.begin(), P.fp_ptr.end() - 1);
    for (int s = P.nnear; s < P.nslot; ++s) {
      const int a = P.slot_a[s], b = P.slot_b[s];
      int e = fillp[a]++;
      P.fp_cl[e] = b;
      P.fp_srow[e] = s;  // block (a, b) as stored
      e = fillp[b]++;
      P.fp_cl[e] = a;
      P.fp_srow[e] = ~s;  // block (b, a): the stored block transposed
    }
  }
  // colours
  P.cols.clear();
  P.cols.resize(P.ncol);
  for (int i = 0; i < nc; ++i)
    if (P.colour[i] >= 0) P.cols[P.colour[i]].cl.push_back(i);
  for (int s = 0; s < P.nslot; ++s) {
    const int cx = P.colour[P.slot_a[s]], cy = P.colour[P.slot_b[s]];
    P.cols[cx].pj_slot.push_back(s);
    if (cy != cx) P.cols[cy].pj_slot.push_back(s);
  }
  // Schur updates are deferred: the contribution of an eliminated cluster i to
  // a block (a, b) stays pending until a or b is processed (its rows/columns
  // are then needed and change coordinates) or the level ends.  Every block is
  // therefore written at most three times per level, with all contributions of
  // an interval summed in one pass.
  //
  // A block is processed only by the colours of its two clusters, so a term added
  // while colour c is eliminated is flushed by the first of those colours after c,
  // or at the level's end (event ncol, the plan `fin`).  Flush `e` visits its
  // blocks in slot order and each block's terms in the order they were added
  // (colour, cluster, then partner pair).  Two passes over the terms: count per
  // (slot, event), then place.
  // terms per chunk of a split task at this level (h2_set_schur_chunk, h2_tune)
  const int chunk_terms =
      (l < (int)H->schur_chunk.size() && H->schur_chunk[l] > 0) ? H->schur_chunk[l] : SCHUR_CHUNK_TERMS;
  const int ncol = P.ncol;
  std::vector<int32_t> tc0(P.nslot), tc1(P.nslot);  // the colours processing each slot, ascending
  for (int s2 = 0; s2 < P.nslot; ++s2) {
    const int ca = P.colour[P.slot_a[s2]], cb = P.colour[P.slot_b[s2]];
    tc0[s2] = std::min(ca, cb);
    tc1[s2] = std::max(ca, cb);
  }
  // event of a term added to slot s2 at colour c, as 0/1 (tc0, tc1) or 2 (level end)
  auto event_of = [&](int s2, int c) -> int { return tc0[s2] > c ? 0 : (tc1[s2] > c ? 1 : 2); };
  std::vector<int32_t> cnt3((size_t)3 * P.nslot, 0);
  std::vector<int32_t> term_slot;
  for (int c = 0; c < ncol; ++c)
    for (int i : P.cols[c].cl)
      for (int x = P.np_ptr[i]; x < P.np_ptr[i + 1]; ++x)
        for (int y = P.np_ptr[i]; y < P.np_ptr[i + 1]; ++y)
          if (P.np_cl[x] <= P.np_cl[y]) {
            const int s2 = P.slot_of(P.np_cl[x], P.np_cl[y]);
            term_slot.push_back(s2);
            cnt3[(size_t)3 * s2 + event_of(s2, c)]++;
          }
  // task layout of every flush; woff3 = where each (slot, event) run of terms starts
  std::vector<int32_t> woff3((size_t)3 * P.nslot, 0);
  auto layout = [&](ColourPlan& C, const std::vector<int32_t>& slots, int ev) {
    C.sc_slot.clear();
    C.sc_cptr.assign(1, 0);
    C.sc_sp.clear();
    C.sc_gtask.clear();
    C.nps = C.ngrp = 0;
    C.sc_slot_u.clear();
    C.sc_cptr_u.assign(1, 0);
    C.sc_sp_u.clear();
    int32_t pos = 0;
    for (int s2 : slots) {
      const int j = ev < 0 ? 2 : (tc0[s2] == ev ? 0 : 1);
      const int T = cnt3[(size_t)3 * s2 + j];
      if (T == 0) continue;
      woff3[(size_t)3 * s2 + j] = pos;
      const int np = (T + chunk_terms - 1) / chunk_terms;
      for (int ch = 0; ch < np; ++ch) {
        const int t1 = (int)((int64_t)T * (ch + 1) / np);
        C.sc_slot.push_back(s2);
        C.sc_cptr.push_back(pos + t1);
        if (np == 1) {
          C.sc_sp.insert(C.sc_sp.end(), {-1, 1, 0, 0});
        } else {
          C.sc_sp.insert(C.sc_sp.end(), {ch, np, C.nps, C.ngrp});
        }
      }
      if (np > 1) {
        C.sc_gtask.push_back((int32_t)C.sc_slot.size() - np);
        C.nps += np;
        C.ngrp += 1;
      }
      pos += T;
      C.sc_slot_u.push_back(s2);
      C.sc_cptr_u.push_back(pos);
      C.sc_sp_u.insert(C.sc_sp_u.end(), {-1, 1, 0, 0});
    }
    C.sc_i.assign(pos, 0);
    C.sc_ja.assign(pos, 0);
    C.sc_jb.assign(pos, 0);
  };
  for (int c = 0; c < ncol; ++c) {
    ColourPlan& C = P.cols[c];
    std::vector<int32_t> touched(C.pj_slot.begin(), C.pj_slot.end());
    std::sort(touched.begin(), touched.end());
    layout(C, touched, c);
  }
  {
    std::vector<int32_t> all(P.nslot);
    for (int s2 = 0; s2 < P.nslot; ++s2) all[s2] = s2;
    layout(P.fin, all, -1);
  }
  {
    size_t q = 0;
    for (int c = 0; c < ncol; ++c)
      for (int i : P.cols[c].cl)
        for (int x = P.np_ptr[i]; x < P.np_ptr[i + 1]; ++x)
          for (int y = P.np_ptr[i]; y < P.np_ptr[i + 1]; ++y)
            if (P.np_cl[x] <= P.np_cl[y]) {
              const int s2 = term_slot[q++];
              const int j = event_of(s2, c);
              ColourPlan& C = j == 2 ? P.fin : P.cols[j == 0 ? tc0[s2] : tc1[s2]];
              const int32_t w = woff3[(size_t)3 * s2 + j]++;
              C.sc_i[w] = i;
              C.sc_ja[w] = x;
              C.sc_jb[w] = y;
            }
  }
  for (int c = 0; c < P.ncol; ++c) {
    ColourPlan& C = P.cols[c];
    // panels and solve gathers
    std::vector<std::array<int32_t, 3>> sv;
    for (int i : C.cl)
      for (int x = P.np_ptr[i]; x < P.np_ptr[i + 1]; ++x) {
        C.pn_i.push_back(i);
        C.pn_ja.push_back(x);
        sv.push_back({P.np_cl[x], i, x});
      }
    std::sort(sv.begin(), sv.end());
    C.sv_cptr.push_back(0);
    for (size_t e = 0; e < sv.size(); ++e) {
      if (e == 0 || sv[e][0] != sv[e - 1][0]) {
        if (e) C.sv_cptr.push_back((int32_t)e);
        C.sv_cl.push_back(sv[e][0]);
      }
      C.sv_i.push_back(sv[e][1]);
      C.sv_ja.push_back(sv[e][2]);
    }
    C.sv_cptr.push_back((int32_t)sv.size());
    if (C.sv_cl.empty()) C.sv_cptr.assign(1, 0);
  }
}

// Plans of several levels, one host thread per level (each writes only its own
// plan); a level whose thread cannot be started is built on the calling thread.
static void build_plan_levels(h2_ctx* H, const std::vector<int>& levels) {
  std::vector<std::exception_ptr> err(levels.size());
  auto work = [H, &levels, &err](size_t e) {
    try {
      build_plan_level(H, levels[e], H->plans[H->S.L - levels[e]]);
    } catch (...) {
      err[e] = std::current_exception();
    }
  };
  std::vector<std::thread> th;
  th.reserve(levels.size());
  for (size_t e = 0; e < levels.size(); ++e) {
    try {
      th.emplace_back(work, e);
    } catch (const std::system_error&) {
      work(e);
    }
  }
  for (auto& t : th) t.join();
  for (auto& e : err)
    if (e) std::rethrow_exception(e);
}

// merge plan from level l (plan P) into level l-1 (plan Pp, or the final block when l == l0).
// Ordered child pairs (a, b) are placed at (a & 1, b & 1) of the parent block
// (a / 2, b / 2).  Parent levels store pairs with a / 2 <= b / 2 (full blocks on
// the diagonal), so ordered pairs below the parent diagonal are skipped; the
// final dense block takes every ordered pair.
static void build_merge(h2_ctx* H, LevelPlan& P, const LevelPlan* Pp) {
  const Structure& S = H->S;
  const int l = P.l;
  const int npar = S.nclusters(l - 1);
  P.merge.clear();
  auto parent_pos = [&](int a, int b) -> int {
    if (Pp) return (a / 2 <= b / 2) ? Pp->slot_of(a / 2, b / 2) : -2;  // -2: below the parent diagonal
    return (a / 2) * npar + (b / 2);  // final dense block: pair index
  };
  std::vector<char> is_adm_fill(P.nslot, 0);
  for (size_t e = 0; e < S.adm[l].size(); ++e) {
    const Pair& p = S.adm[l][e];
    const int code = P.slot_code(p.first, p.second);
    const int fs = code == INT32_MIN ? -1 : (code < 0 ? ~code : code);
    if (fs >= 0) is_adm_fill[fs] = 1;
    const int pp = parent_pos(p.first, p.second);
    if (pp == -2) continue;
    if (pp < 0) fail(H2_ERR_INTERNAL, "admissible pair without an inadmissible parent");
    P.merge.push_back({pp, p.first & 1, p.second & 1, 1, fs, (int32_t)e, p.first, p.second, code < 0 ? 1 : 0});
  }
  for (int s = 0; s < P.nslot; ++s) {
    if (s >= P.nnear && is_adm_fill[s]) continue;
    const int kind = s < P.nnear ? 0 : 2;
    for (int o = 0; o < 2; ++o) {
      const int a = o ? P.slot_b[s] : P.slot_a[s], b = o ? P.slot_a[s] : P.slot_b[s];
      if (o && a == b) continue;
      const int pp = parent_pos(a, b);
      if (pp == -2) continue;
      if (pp < 0) {
        if (kind == 0) fail(H2_ERR_INTERNAL, "inadmissible pair without an inadmissible parent");
        if (!Pp) fail(H2_ERR_INTERNAL, "fill-in outside the final block");
        fail(H2_ERR_INTERNAL, "carried fill-in without a parent slot");
      }
      P.merge.push_back({pp, a & 1, b & 1, kind, s, -1, a, b, o});
    }
  }
}

static void upload_plan(LevelPlan& P, hipStream_t st) {
  P.d_colour.upload(P.colour, st);
  P.d_nonempty.upload(P.nonempty, st);
  P.d_slot_a.upload(P.slot_a, st);
  P.d_slot_b.upload(P.slot_b, st);
  P.d_diag_slot.upload(P.diag_slot, st);
  P.d_np_ptr.upload(P.np_ptr, st);
  P.d_np_cl.upload(P.np_cl, st);
  P.d_np_srow.upload(P.np_srow, st);
  P.d_np_scol.upload(P.np_scol, st);
  P.d_fp_ptr.upload(P.fp_ptr, st);
  P.d_fp_cl.upload(P.fp_cl, st);
  P.d_fp_srow.upload(P.fp_srow, st);
  for (ColourPlan& C : P.cols) {
    C.d_cl.upload(C.cl, st);
    C.d_pj_slot.upload(C.pj_slot, st);
    C.d_sc_slot.upload(C.sc_slot, st);
    C.d_sc_cptr.upload(C.sc_cptr, st);
    C.d_sc_i.upload(C.sc_i, st);
    C.d_sc_ja.upload(C.sc_ja, st);
    C.d_sc_jb.upload(C.sc_jb, st);
    C.d_sc_sp.upload(C.sc_sp, st);
    C.d_sc_gtask.upload(C.sc_gtask, st);
    C.d_sc_slot_u.upload(C.sc_slot_u, st);
    C.d_sc_cptr_u.upload(C.sc_cptr_u, st);
    C.d_sc_sp_u.upload(C.sc_sp_u, st);
    C.d_pn_i.upload(C.pn_i, st);
    C.d_pn_ja.upload(C.pn_ja, st);
    C.d_sv_cl.upload(C.sv_cl, st);
    C.d_sv_cptr.upload(C.sv_cptr, st);
    C.d_sv_i.upload(C.sv_i, st);
    C.d_sv_ja.upload(C.sv_ja, st);
  }
  P.fin.d_sc_slot.upload(P.fin.sc_slot, st);
  P.fin.d_sc_cptr.upload(P.fin.sc_cptr, st);
  P.fin.d_sc_i.upload(P.fin.sc_i, st);
  P.fin.d_sc_ja.upload(P.fin.sc_ja, st);
  P.fin.d_sc_jb.upload(P.fin.sc_jb, st);
  P.fin.d_sc_sp.upload(P.fin.sc_sp, st);
  P.fin.d_sc_gtask.upload(P.fin.sc_gtask, st);
  P.fin.d_sc_slot_u.upload(P.fin.sc_slot_u, st);
  P.fin.d_sc_cptr_u.upload(P.fin.sc_cptr_u, st);
  P.fin.d_sc_sp_u.upload(P.fin.sc_sp_u, st);
}

// ---------------------------------------------------------------------------
// batched GEMM helper (host-resolved tasks)
// ---------------------------------------------------------------------------
// Task lists live in handle-owned grow-only buffers; the call waits for its
// launch before the lists are reused.
static void run_gemms(h2_ctx* H, const std::vector<GemmTask>& tasks, hipStream_t st) {
  if (tasks.empty()) return;
  std::vector<int32_t> tt, rc;
  for (size_t i = 0; i < tasks.size(); ++i) {
    const int tr = (tasks[i].m + 63) / 64, tc = (tasks[i].n + 63) / 64;
    for (int a = 0; a < tr; ++a)
      for (int b = 0; b < tc; ++b) {
        tt.push_back((int32_t)i);
        rc.push_back(a | (b << 16));
      }
  }
  DArr<GemmTask>& dt = H->gm_tasks;
  DArr<int32_t>& dtt = H->gm_tt;
  DArr<int32_t>& drc = H->gm_rc;
  dt.alloc(tasks.size());
  HIPCHK(hipMemcpyAsync(dt.p, tasks.data(), tasks.size() * sizeof(GemmTask), hipMemcpyHostToDevice, st));
  dtt.upload(tt, st);
  drc.upload(rc, st);
  launch_gemm_batched(dt.p, dtt.p, drc.p, (int)tt.size(), st);
  HIPCHK(hipStreamSynchronize(st));
}

static bool sync_debug() {
  static const bool on = [] {
    const char* e = std::getenv("H2MI_SYNC_CHECK");
    return e && e[0] == '1';
  }();
  return on;
}

// After a group of launches: report launch errors; with H2MI_SYNC_CHECK=1 also
// wait for the device and report execution errors at the group that caused them.
static void check_launch(const char* where = "") {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) fail(H2_ERR_DEVICE, std::string("kernel launch ") + where + ": " + hipGetErrorString(e));
  if (sync_debug()) {
    e = hipDeviceSynchronize();
    if (e != hipSuccess) fail(H2_ERR_DEVICE, std::string("kernel execution ") + where + ": " + hipGetErrorString(e));
  }
}

// ---------------------------------------------------------------------------
// construction (Sec. II): nested bases from the far-field block rows
// ---------------------------------------------------------------------------
static std::vector<uint32_t> near_mask(const Structure& S, int l) {
  const int64_t nc = S.nclusters(l);
  std::vector<uint32_t> m((size_t)((nc * nc + 31) / 32), 0u);
  for (const Pair& p : S.near[l]) {
    const int64_t bit = (int64_t)p.first * nc + p.second;
    m[bit >> 5] |= 1u << (bit & 31);
  }
  return m;
}

static int forced_k_of(h2_ctx* H, int l, int t) {
  if (!H->has_forced) return -1;
  return H->forced_k[H->lvl_base[l] + t];
}

constexpr int CONSTRUCT_PASSES = 2;  // Gram passes of the construction eigen-decomposition

static void construct(h2_ctx* H, hipStream_t st) {
  const Structure& S = H->S;
  const int L = S.L, l0 = S.l0;
  const int nlev = L - l0 + 1;
  H->build.clear();
  H->build.resize(nlev);
  const GeomView& g = H->geom;
  for (int l = L; l >= l0; --l) {
    BuildLevel& B = H->build[L - l];
    const int nc = S.nclusters(l);
    B.k.assign(nc, 0);
    B.nu.assign(nc, 0.0);
    B.margin.assign(2 * nc, 0.0);
    // Gram dimensions
    std::vector<int32_t> dim(nc, 0);
    for (int t = 0; t < nc; ++t) {
      if (l == L)
        dim[t] = (int32_t)S.size[l][t];
      else
        dim[t] = H->build[L - l - 1].k[2 * t] + H->build[L - l - 1].k[2 * t + 1];
      if (S.size[l][t] == 0) dim[t] = 0;
    }
    std::vector<int64_t> goff(nc + 1, 0);
    int dmax = 0;
    for (int t = 0; t < nc; ++t) {
      goff[t + 1] = goff[t] + (int64_t)dim[t] * dim[t];
      dmax = std::max(dmax, dim[t]);
    }
    const int64_t gtot = goff[nc];
    DArr<double2> G;
    G.alloc(gtot);
    DArr<int64_t> d_goff;
    d_goff.upload(goff, st);
    std::vector<uint32_t> mask = near_mask(S, l);
    DArr<uint32_t> d_mask;
    d_mask.upload(mask, st);
    const int ntr = std::max(1, (dmax + 63) / 64);
    if (l == L) {
      std::vector<int64_t> cstart(S.start[l].begin(), S.start[l].end());
      std::vector<int32_t> csize(nc);
      for (int t = 0; t < nc; ++t) csize[t] = (int32_t)S.size[l][t];
      DArr<int64_t> d_cs;
      DArr<int32_t> d_sz;
      d_cs.upload(cstart, st);
      d_sz.upload(csize, st);
      // split the columns so that the partial Grams stay below ~1 GiB
      int64_t kchunk = 2048;
      while ((H->N + kchunk - 1) / kchunk * gtot * 16 > (int64_t)1 << 30 && kchunk < H->N) kchunk *= 2;
      const int nchunks = (int)((H->N + kchunk - 1) / kchunk);
      DArr<double2> part;
      part.alloc((size_t)nchunks * gtot);
      launch_leaf_gram(g, d_mask.p, nc, l, d_cs.p, d_sz.p, kchunk, nchunks, part.p, gtot, d_goff.p, ntr, st);
      check_launch("host.cpp:534");
      launch_gram_reduce(part.p, G.p, nullptr, nullptr, nc, nchunks, gtot, st);
      check_launch("host.cpp:536");
      HIPCHK(hipStreamSynchronize(st));
    } else {
      const BuildLevel& C = H->build[L - l - 1];
      const int ncc = S.nclusters(l + 1);
      // stacked row blocks: child c of parent t writes rows [off, off + k_c) of Y_t (ld dim_t)
      std::vector<int64_t> cstart(S.start[l + 1].begin(), S.start[l + 1].end());
      std::vector<int32_t> csize(ncc), ck(ncc), yld(ncc);
      int kmax = 0;
      for (int c = 0; c < ncc; ++c) {
        csize[c] = (int32_t)S.size[l + 1][c];
        ck[c] = C.k[c];
        yld[c] = dim[c / 2];
        kmax = std::max(kmax, ck[c]);
      }
      std::vector<int64_t> ybase(nc + 1, 0);
      int64_t rowsum = 0;
      for (int t = 0; t < nc; ++t) rowsum += dim[t];
      int64_t chunk = 8192;
      while (chunk > 256 && rowsum * chunk * 16 > ((int64_t)1 << 31)) chunk /= 2;
      chunk = std::min<int64_t>(chunk, H->N);
      for (int t = 0; t < nc; ++t) ybase[t + 1] = ybase[t] + (int64_t)dim[t] * chunk;
      std::vector<int64_t> yoff(ncc);
      for (int c = 0; c < ncc; ++c) yoff[c] = ybase[c / 2] + ((c & 1) ? C.k[c - 1] : 0);
      std::vector<int64_t> ytoff(nc);
      for (int t = 0; t < nc; ++t) ytoff[t] = ybase[t];
      DArr<int64_t> d_cs, d_yoff, d_ytoff;
      DArr<int32_t> d_sz, d_ck, d_yld, d_dim;
      d_cs.upload(cstart, st);
      d_sz.upload(csize, st);
      d_ck.upload(ck, st);
      d_yld.upload(yld, st);
      d_yoff.upload(yoff, st);
      d_ytoff.upload(ytoff, st);
      d_dim.upload(dim, st);
      DArr<double2> Y;
      Y.alloc(std::max<int64_t>(1, ybase[nc]));
      launch_zero(G.p, gtot, st);
      const int ktr = std::max(1, (kmax + 63) / 64);
      for (int64_t c0 = 0; c0 < H->N; c0 += chunk) {
        const int ncols = (int)std::min<int64_t>(chunk, H->N - c0);
        launch_proj_rows(g, d_mask.p, l, ncc, d_cs.p, d_sz.p, d_ck.p, C.d_voff.p, C.V.p, d_yoff.p, d_yld.p, Y.p, c0,
                         ncols, ktr, st);
        check_launch("host.cpp:579");
        launch_gram_acc(nc, d_dim.p, d_ytoff.p, Y.p, ncols, d_goff.p, G.p, ntr, st);
        check_launch("host.cpp:581");
      }
      HIPCHK(hipStreamSynchronize(st));
    }
    // eigen-decomposition of every Gram (relative-accuracy Jacobi)
    std::vector<int64_t> uoff(goff.begin(), goff.end() - 1), loff(nc), soff(nc);
    int64_t lt = 0, stt = 0;
    for (int t = 0; t < nc; ++t) {
      loff[t] = lt;
      lt += dim[t];
      soff[t] = stt;
      if (dim[t] > 64) stt += 2 * (int64_t)(dim[t] + 1) * (dim[t] + 1);
    }
    DArr<double2> U, scratch;
    DArr<double> lam;
    U.alloc(gtot);
    lam.alloc(std::max<int64_t>(1, lt));
    scratch.alloc(std::max<int64_t>(1, stt));
    DArr<int64_t> d_uoff, d_loff, d_soff;
    DArr<int32_t> d_dim;
    d_uoff.upload(uoff, st);
    d_loff.upload(loff, st);
    d_soff.upload(soff, st);
    d_dim.upload(dim, st);
    if (dmax > 255) fail(H2_ERR_INTERNAL, "construction Gram larger than 255 (eigensolver limit)");
    launch_jacobi(nc, d_dim.p, d_goff.p, G.p, d_uoff.p, U.p, d_loff.p, lam.p, 1, scratch.p, d_soff.p, st);
    check_launch("construction eigensolver");
    // Refinement passes.  The Gram W W^H of a far-field row W carries rounding of order
    // u sigma_1^2 in every entry, which moves the eigenvectors of singular values near
    // the truncation threshold by ~u sigma_1^2 / (sigma_k^2 - sigma_{k+1}^2) (1e-7 at
    // eps = 1e-4 with a 5 % gap).  Rotating the rows first, B = U0^H W, and taking the
    // Gram of B again leaves errors of order u sigma_1 (sigma_i + sigma_j) in entry
    // (i, j): its eigenvectors U1 make U = U0 U1 accurate to ~u sigma_1 / (sigma_k -
    // sigma_{k+1}), the accuracy of an SVD of W, and its eigenvalues the sigma_j^2.
    // (A third pass measured no better: 32^3 against the SVD-built oracle, 1.0e-10
    // element-wise with two passes, 2.8e-10 with three - rounding-level noise.)
    for (int pass = 1; pass < CONSTRUCT_PASSES; ++pass) {
      const bool leaf = (l == L);
      std::vector<int64_t> cstart2, ybase2(nc + 1, 0);
      std::vector<int32_t> csize2, ck2, yld2;
      std::vector<int64_t> yoff2;
      const int nch = leaf ? nc : S.nclusters(l + 1);
      int kmax2 = 0;
      if (leaf) {
        cstart2.assign(S.start[l].begin(), S.start[l].end());
        csize2.resize(nc);
        for (int t = 0; t < nc; ++t) csize2[t] = (int32_t)S.size[l][t];
        ck2 = dim;
        yld2 = dim;
        kmax2 = dmax;
      } else {
        const BuildLevel& C = H->build[L - l - 1];
        cstart2.assign(S.start[l + 1].begin(), S.start[l + 1].end());
        csize2.resize(nch);
        ck2.resize(nch);
        yld2.resize(nch);
        for (int c = 0; c < nch; ++c) {
          csize2[c] = (int32_t)S.size[l + 1][c];
          ck2[c] = C.k[c];
          yld2[c] = dim[c / 2];
          kmax2 = std::max(kmax2, ck2[c]);
        }
      }
      int64_t rowsum = 0;
      for (int t = 0; t < nc; ++t) rowsum += dim[t];
      int64_t chunk = 8192;
      while (chunk > 256 && rowsum * chunk * 16 > ((int64_t)1 << 31)) chunk /= 2;
      chunk = std::min<int64_t>(chunk, H->N);
      for (int t = 0; t < nc; ++t) ybase2[t + 1] = ybase2[t] + (int64_t)dim[t] * chunk;
      if (leaf) {
        yoff2.assign(ybase2.begin(), ybase2.end() - 1);
      } else {
        const BuildLevel& C = H->build[L - l - 1];
        yoff2.resize(nch);
        for (int c = 0; c < nch; ++c) yoff2[c] = ybase2[c / 2] + ((c & 1) ? C.k[c - 1] : 0);
      }
      DArr<int64_t> d_cs2, d_yoff2, d_ybase2;
      DArr<int32_t> d_sz2, d_ck2, d_yld2;
      d_cs2.upload(cstart2, st);
      d_sz2.upload(csize2, st);
      d_ck2.upload(ck2, st);
      d_yld2.upload(yld2, st);
      d_yoff2.upload(yoff2, st);
      d_ybase2.upload(std::vector<int64_t>(ybase2.begin(), ybase2.end() - 1), st);
      DArr<double2> Y, Y2;
      Y.alloc(std::max<int64_t>(1, ybase2[nc]));
      if (!leaf) Y2.alloc(std::max<int64_t>(1, ybase2[nc]));
      launch_zero(G.p, gtot, st);
      const int ktr2 = std::max(1, (kmax2 + 63) / 64);
      for (int64_t c0 = 0; c0 < H->N; c0 += chunk) {
        const int ncols = (int)std::min<int64_t>(chunk, H->N - c0);
        if (leaf) {
          // B = U0^H Z[t, far columns] straight from the kernel entries
          launch_proj_rows(g, d_mask.p, l, nc, d_cs2.p, d_sz2.p, d_ck2.p, d_uoff.p, U.p, d_yoff2.p, d_yld2.p, Y.p,
                           c0, ncols, ktr2, st);
          check_launch("construction second pass");
          launch_gram_acc(nc, d_dim.p, d_ybase2.p, Y.p, ncols, d_goff.p, G.p, ntr, st);
        } else {
          const BuildLevel& C = H->build[L - l - 1];
          launch_proj_rows(g, d_mask.p, l, nch, d_cs2.p, d_sz2.p, d_ck2.p, C.d_voff.p, C.V.p, d_yoff2.p, d_yld2.p,
                           Y.p, c0, ncols, ktr2, st);
          check_launch("construction second pass");
          std::vector<GemmTask> rot;
          for (int t = 0; t < nc; ++t) {
            if (dim[t] == 0) continue;
            rot.push_back({U.p + uoff[t], Y.p + ybase2[t], Y2.p + ybase2[t], dim[t], dim[t], dim[t], dim[t], ncols,
                           dim[t], OP_C, OP_N, ST_SET});
          }
          run_gemms(H, rot, st);
          launch_gram_acc(nc, d_dim.p, d_ybase2.p, Y2.p, ncols, d_goff.p, G.p, ntr, st);
        }
        check_launch("construction second pass");
      }
      DArr<double2> U1;
      U1.alloc(gtot);
      launch_jacobi(nc, d_dim.p, d_goff.p, G.p, d_uoff.p, U1.p, d_loff.p, lam.p, 1, scratch.p, d_soff.p, st);
      check_launch("construction eigensolver, second pass");
      // U = U0 U1 (written over the consumed Gram, then moved into U)
      std::vector<GemmTask> prod;
      for (int t = 0; t < nc; ++t) {
        if (dim[t] == 0) continue;
        prod.push_back({U.p + uoff[t], U1.p + uoff[t], G.p + uoff[t], dim[t], dim[t], dim[t], dim[t], dim[t], dim[t],
                        OP_N, OP_N, ST_SET});
      }
      run_gemms(H, prod, st);
      if (gtot > 0) HIPCHK(hipMemcpyAsync(U.p, G.p, gtot * sizeof(double2), hipMemcpyDeviceToDevice, st));
    }
    std::vector<double> hl(std::max<int64_t>(1, lt));
    HIPCHK(hipMemcpyAsync(hl.data(), lam.p, hl.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    // ranks: sigma_j > eps * sigma_1
    B.boff.assign(nc + 1, 0);
    for (int t = 0; t < nc; ++t) {
      int kt = 0;
      double s1 = 0.0;
      if (dim[t] > 0) {
        s1 = std::sqrt(std::max(hl[loff[t]], 0.0));
        const double thr = H->eps * s1;
        if (s1 > 0.0) {
          for (int j = 0; j < dim[t]; ++j)
            if (std::sqrt(std::max(hl[loff[t] + j], 0.0)) > thr) kt = j + 1;
          B.margin[2 * t] = kt > 0 ? std::sqrt(std::max(hl[loff[t] + kt - 1], 0.0)) / thr : 1e300;
          B.margin[2 * t + 1] = kt < dim[t] ? std::sqrt(std::max(hl[loff[t] + kt], 0.0)) / thr : 0.0;
        }
      }
      const int fk = forced_k_of(H, l, t);
      if (fk >= 0) kt = std::min(fk, dim[t]);
      B.k[t] = kt;
      B.nu[t] = s1;
      B.boff[t + 1] = B.boff[t] + (int64_t)dim[t] * kt;
    }
    // basis = leading k columns of the eigenvector matrix (contiguous in column-major)
    B.basis.alloc(B.boff[nc]);
    for (int t = 0; t < nc; ++t)
      if (B.boff[t + 1] > B.boff[t])
        HIPCHK(hipMemcpyAsync(B.basis.p + B.boff[t], U.p + uoff[t], (B.boff[t + 1] - B.boff[t]) * sizeof(double2),
                              hipMemcpyDeviceToDevice, st));
    // expanded bases
    B.voff.assign(nc + 1, 0);
    for (int t = 0; t < nc; ++t) B.voff[t + 1] = B.voff[t] + S.size[l][t] * (int64_t)B.k[t];
    B.V.alloc(B.voff[nc]);
    if (l == L) {
      if (B.voff[nc] > 0)
        HIPCHK(hipMemcpyAsync(B.V.p, B.basis.p, B.voff[nc] * sizeof(double2), hipMemcpyDeviceToDevice, st));
    } else {
      const BuildLevel& C = H->build[L - l - 1];
      std::vector<GemmTask> tasks;
      for (int t = 0; t < nc; ++t) {
        if (B.k[t] == 0 || S.size[l][t] == 0) continue;
        const int k1 = C.k[2 * t], k2 = C.k[2 * t + 1];
        const int64_t n1 = S.size[l + 1][2 * t], n2 = S.size[l + 1][2 * t + 1];
        const int64_t nt = S.size[l][t];
        const double2* T = B.basis.p + B.boff[t];
        if (k1 > 0 && n1 > 0)
          tasks.push_back({C.V.p + C.voff[2 * t], T, B.V.p + B.voff[t], n1, (int64_t)(k1 + k2), nt, (int32_t)n1,
                           B.k[t], k1, OP_N, OP_N, ST_SET});
        if (k2 > 0 && n2 > 0)
          tasks.push_back({C.V.p + C.voff[2 * t + 1], T + k1, B.V.p + B.voff[t] + n1, n2, (int64_t)(k1 + k2), nt,
                           (int32_t)n2, B.k[t], k2, OP_N, OP_N, ST_SET});
      }
      // rows of a child with k = 0 must read as zero
      launch_zero(B.V.p, B.voff[nc], st);
      run_gemms(H, tasks, st);
    }
    B.ktot = 0;
    for (int t = 0; t < nc; ++t) B.ktot += B.k[t];
    B.d_voff.upload(B.voff, st);
    B.d_k.upload(B.k, st);
    HIPCHK(hipStreamSynchronize(st));
  }
  // couplings S_ts = V_t^H Z(t, s) conj(V_s) for admissible pairs (t < s), S_st = S_ts^T
  for (int l = l0; l <= L; ++l) {
    BuildLevel& B = H->build[L - l];
    const auto& adm = S.adm[l];
    B.soff.assign(adm.size() + 1, 0);
    for (size_t e = 0; e < adm.size(); ++e)
      B.soff[e + 1] = B.soff[e] + (int64_t)B.k[adm[e].first] * B.k[adm[e].second];
    B.S.alloc(B.soff[adm.size()]);
    std::unordered_map<int64_t, int32_t> idx;
    const int64_t nc = S.nclusters(l);
    for (size_t e = 0; e < adm.size(); ++e) idx[(int64_t)adm[e].first * nc + adm[e].second] = (int32_t)e;
    std::vector<int32_t> pt, ps;
    std::vector<int64_t> xoff;
    std::vector<size_t> pe;
    int64_t xt = 0;
    int kmax = 0, smax = 0;
    std::vector<int64_t> cstart(S.start[l].begin(), S.start[l].end());
    std::vector<int32_t> csize(nc), ck(nc);
    for (int t = 0; t < nc; ++t) {
      csize[t] = (int32_t)S.size[l][t];
      ck[t] = B.k[t];
    }
    DArr<int64_t> d_cs;
    DArr<int32_t> d_sz, d_ck;
    d_cs.upload(cstart, st);
    d_sz.upload(csize, st);
    d_ck.upload(ck, st);
    DArr<int64_t> d_voff;
    d_voff.upload(B.voff, st);
    auto flush = [&]() {
      if (pt.empty()) return;
      DArr<int32_t> d_pt, d_ps;
      DArr<int64_t> d_xoff;
      DArr<double2> X;
      d_pt.upload(pt, st);
      d_ps.upload(ps, st);
      d_xoff.upload(xoff, st);
      X.alloc(std::max<int64_t>(1, xt));
      const int ntr = std::max(1, (kmax + 63) / 64), ntc = std::max(1, (smax + 63) / 64);
      launch_coupling_x(g, (int)pt.size(), ntr, ntc, d_pt.p, d_ps.p, d_cs.p, d_sz.p, d_ck.p, d_voff.p, B.V.p,
                        d_xoff.p, X.p, st);
      check_launch("host.cpp:712");
      std::vector<GemmTask> tasks, trans;
      for (size_t q = 0; q < pt.size(); ++q) {
        const int t = pt[q], s = ps[q];
        const size_t e = pe[q];
        tasks.push_back({X.p + xoff[q], B.V.p + B.voff[s], B.S.p + B.soff[e], (int64_t)std::max(1, B.k[t]),
                         (int64_t)S.size[l][s], (int64_t)std::max(1, B.k[t]), B.k[t], B.k[s], (int32_t)S.size[l][s],
                         OP_N, OP_R, ST_SET});
        const size_t et = idx[(int64_t)s * nc + t];
        trans.push_back({B.S.p + B.soff[e], nullptr, B.S.p + B.soff[et], (int64_t)std::max(1, B.k[t]), 0,
                         (int64_t)std::max(1, B.k[s]), B.k[t], B.k[s], 0, 0, 0, 0});
      }
      run_gemms(H, tasks, st);
      DArr<GemmTask> dtr;
      dtr.alloc(trans.size());
      HIPCHK(hipMemcpyAsync(dtr.p, trans.data(), trans.size() * sizeof(GemmTask), hipMemcpyHostToDevice, st));
      launch_transpose_copy(dtr.p, (int)trans.size(), st);
      check_launch("host.cpp:729");
      HIPCHK(hipStreamSynchronize(st));
      pt.clear();
      ps.clear();
      xoff.clear();
      pe.clear();
      xt = 0;
      kmax = smax = 0;
    };
    for (size_t e = 0; e < adm.size(); ++e) {
      const int t = adm[e].first, s = adm[e].second;
      if (t >= s) continue;
      if (B.k[t] == 0 || B.k[s] == 0) continue;
      pt.push_back(t);
      ps.push_back(s);
      pe.push_back(e);
      xoff.push_back(xt);
      xt += (int64_t)B.k[t] * S.size[l][s];
      kmax = std::max(kmax, B.k[t]);
      smax = std::max<int>(smax, (int)S.size[l][s]);
      if (xt * 16 > ((int64_t)1 << 30)) flush();
    }
    flush();
    // device views for the H^2 product
    B.d_soff.upload(B.soff, st);
    B.d_nu.upload(B.nu, st);
    std::vector<int32_t> rows(nc);
    for (int t = 0; t < nc; ++t) rows[t] = (int32_t)S.size[l][t];
    B.d_rows.upload(rows, st);
    std::vector<int32_t> cptr(nc + 1, 0), ccol(adm.size());
    for (const Pair& p : adm) cptr[p.first + 1]++;
    for (int t = 0; t < nc; ++t) cptr[t + 1] += cptr[t];
    for (size_t e = 0; e < adm.size(); ++e) ccol[e] = adm[e].second;  // adm sorted by row: CSR order = list order
    B.d_cptr.upload(cptr, st);
    B.d_ccol.upload(ccol, st);
    B.d_cstart.upload(cstart, st);
    std::vector<int64_t> xo(nc);
    int64_t o = 0;
    for (int t = 0; t < nc; ++t) {
      xo[t] = o;
      o += B.k[t];
    }
    B.d_xoff.upload(xo, st);
  }
  // inadmissible leaf blocks
  const auto& nl = S.near[L];
  H->near_off.assign(nl.size() + 1, 0);
  for (size_t e = 0; e < nl.size(); ++e)
    H->near_off[e + 1] = H->near_off[e] + S.size[L][nl[e].first] * S.size[L][nl[e].second];
  H->near_orig.alloc(H->near_off[nl.size()]);
  {
    std::vector<int32_t> pr(nl.size()), pc(nl.size()), sz(S.nclusters(L));
    for (size_t e = 0; e < nl.size(); ++e) {
      pr[e] = nl[e].first;
      pc[e] = nl[e].second;
    }
    for (int t = 0; t < S.nclusters(L); ++t) sz[t] = (int32_t)S.size[L][t];
    std::vector<int64_t> cs(S.start[L].begin(), S.start[L].end());
    H->d_near_pr.upload(pr, st);
    H->d_near_pc.upload(pc, st);
    H->d_leaf_size.upload(sz, st);
    H->d_leaf_start.upload(cs, st);
    H->d_near_off.upload(H->near_off, st);
    launch_near_blocks(g, H->d_near_pr.p, H->d_near_pc.p, H->d_near_off.p, H->d_leaf_start.p, H->d_leaf_size.p,
                       H->d_leaf_start.p, H->d_leaf_size.p, (int)nl.size(), H->near_orig.p, st);
    check_launch("host.cpp:795");
    std::vector<int32_t> nptr(S.nclusters(L) + 1, 0);
    for (const Pair& p : nl) nptr[p.first + 1]++;
    for (int t = 0; t < S.nclusters(L); ++t) nptr[t + 1] += nptr[t];
    H->d_near_ptr.upload(nptr, st);
    H->d_near_col.upload(pc, st);
    HIPCHK(hipStreamSynchronize(st));
  }
}

// ---------------------------------------------------------------------------
// factorization
// ---------------------------------------------------------------------------
struct EventPool {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  hipEvent_t next(hipStream_t st) {
    if (used == ev.size()) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      ev.push_back(e);
    }
    hipEvent_t e = ev[used++];
    HIPCHK(hipEventRecord(e, st));
    return e;
  }
  ~EventPool() {
    for (auto e : ev) (void)hipEventDestroy(e);
  }
};

static float elapsed(hipEvent_t a, hipEvent_t b) {
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, a, b));
  return ms;
}

static void dense_lu_factor(h2_ctx* H, hipStream_t st);

constexpr size_t SCHUR_PART_MAX_BYTES = size_t(8) << 30;
// A colour's Schur flush whose whole tasks make fewer 64 x 64 tile workgroups than
// this splits its long tasks into chunks of SCHUR_CHUNK_TERMS terms (more
// workgroups for a small flush); a larger flush fills the device with whole tasks
// and spares the partial tiles' traffic.  Per level, h2_set_schur_split / h2_tune.
constexpr int64_t SCHUR_SPLIT_BELOW = 8192;
// Mixed form: a level's flushes route FP32-safe terms to FP32 (k_schur_mixed) when
// its clusters' average eliminated dimension is at least this; below, few tasks
// gather enough FP32-safe contraction columns to pay for that kernel's lower
// occupancy, and the FP64 flush runs.  Per level, h2_set_mixed_flush / h2_tune.
constexpr double MIXED_FLUSH_MIN_D = 32.0;

static void release_factor_buffers(h2_ctx* H) {
  H->flev.clear();
  H->slot_buf[0].release();
  H->slot_buf[1].release();
  H->ws_bp.release();
  H->ws_w.release();
  H->ws_temp.release();
  H->ws_lu.release();
  H->ws_eig.release();
  H->ws_gram.release();
  H->ws_scp.release();
  H->ws_merge.release();
  H->Zf.release();
  H->dl_linv.release();
  H->dl_uinv.release();
  H->dl_piv.release();
  H->dl_flag.release();
  H->vbuf.clear();
  H->vbuf_nrhs = 0;
}

// Early stop (Sec. III-C): the final dense block is the matrix merged to level
// pl = ls - 1.  Its pairs that are inadmissible at pl come from the merge; every
// other pair (p, q) lies in an admissible block (p', q') of some level lev <= pl
// (eq. 2), whose entries in the merged coordinates of level pl are
// X_p S_p'q' X_q^T with X_p = B_p E_p: B_p the transfer matrix of p padded with
// zero rows for its children's added columns (eq. 23) and E_p the product of
// the transfer-matrix rows along the path from p up to p' (eq. 3).  The carried
// fill-ins of those pairs were placed by the merge; these products are added.
static void add_far_blocks(h2_ctx* H, int ls, const std::vector<int32_t>& n_par, const std::vector<int32_t>& off1,
                           hipStream_t st) {
  const Structure& S = H->S;
  const int L = S.L, l0 = S.l0, pl = ls - 1;
  const int npar = S.nclusters(pl);
  const int nlv = pl - l0 + 1;  // levels pl, pl - 1, ..., l0
  auto kc = [&](int lev, int t) -> int64_t { return S.size[lev][t] ? H->build[L - lev].k[t] : 0; };
  // X_p^(lev) for every nonempty p of level pl: n_par[p] x k(ancestor at lev), packed
  std::vector<int64_t> xoff((size_t)nlv * npar + 1, 0);
  for (int d = 0; d < nlv; ++d)
    for (int p = 0; p < npar; ++p) {
      const size_t e = (size_t)d * npar + p;
      xoff[e + 1] = xoff[e] + (S.size[pl][p] ? (int64_t)n_par[p] * kc(pl - d, p >> d) : 0);
    }
  H->fb_X.alloc(xoff.back());
  launch_zero(H->fb_X.p, (int64_t)H->fb_X.n, st);
  {
    // level pl: the padded transfer matrices
    const BuildLevel& Bp = H->build[L - pl];
    std::vector<int32_t> pn(npar), pk(npar), k1(npar), k2(npar);
    for (int p = 0; p < npar; ++p) {
      pn[p] = S.size[pl][p] ? n_par[p] : 0;
      pk[p] = (int32_t)kc(pl, p);
      k1[p] = (int32_t)kc(ls, 2 * p);
      k2[p] = (int32_t)kc(ls, 2 * p + 1);
    }
    H->fb_n.upload(pn, st);
    H->fb_k.upload(pk, st);
    H->fb_k1.upload(k1, st);
    H->fb_k2.upload(k2, st);
    H->fb_off1.upload(off1, st);
    H->fb_toff.upload(std::vector<int64_t>(Bp.boff.begin(), Bp.boff.end() - 1), st);
    H->fb_xoff.upload(std::vector<int64_t>(xoff.begin(), xoff.begin() + npar), st);
    launch_parent_basis(npar, H->fb_n.p, H->fb_k.p, H->fb_k1.p, H->fb_k2.p, H->fb_off1.p, H->fb_toff.p,
                        Bp.basis.p, H->fb_xoff.p, H->fb_X.p, st);
    check_launch("far blocks: padded transfer matrices");
  }
  // coarser levels: X_p^(lev) = X_p^(lev+1) T_par[rows of the child on the path]
  for (int d = 1; d < nlv; ++d) {
    const int lev = pl - d;
    const BuildLevel& Bl = H->build[L - lev];
    std::vector<GemmTask> tasks;
    for (int p = 0; p < npar; ++p) {
      if (!S.size[pl][p] || n_par[p] == 0) continue;
      const int c = p >> (d - 1), par = c >> 1;
      const int64_t kchild = kc(lev + 1, c), kpar = kc(lev, par);
      if (kchild == 0 || kpar == 0) continue;
      const int64_t ldt = kc(lev + 1, 2 * par) + kc(lev + 1, 2 * par + 1);
      const int64_t row0 = (c & 1) ? kc(lev + 1, 2 * par) : 0;
      GemmTask t{};
      t.A = H->fb_X.p + xoff[(size_t)(d - 1) * npar + p];
      t.lda = n_par[p];
      t.B = Bl.basis.p + Bl.boff[par] + row0;
      t.ldb = ldt;
      t.C = H->fb_X.p + xoff[(size_t)d * npar + p];
      t.ldc = n_par[p];
      t.m = n_par[p];
      t.n = (int32_t)kpar;
      t.K = (int32_t)kchild;
      t.opA = OP_N;
      t.opB = OP_N;
      t.mode = ST_SET;
      tasks.push_back(t);
    }
    run_gemms(H, tasks, st);
  }
  // every pair not inadmissible at pl: Y = X_p S_p'q', then Z_f(p, q) += Y X_q^T
  std::vector<std::unordered_map<int64_t, int32_t>> adm_index(nlv);
  for (int d = 0; d < nlv; ++d) {
    const int lev = pl - d;
    const int64_t nc = S.nclusters(lev);
    for (size_t e = 0; e < S.adm[lev].size(); ++e)
      adm_index[d][(int64_t)S.adm[lev][e].first * nc + S.adm[lev][e].second] = (int32_t)e;
  }
  std::unordered_map<int64_t, char> near_pl;
  for (const Pair& pr : S.near[pl]) near_pl[(int64_t)pr.first * npar + pr.second] = 1;
  struct Far {
    int p, q, d, e;
  };
  std::vector<Far> far;
  int64_t ytot = 0;
  std::vector<int64_t> yoff;
  for (int p = 0; p < npar; ++p) {
    if (!S.size[pl][p] || n_par[p] == 0) continue;
    for (int q = 0; q < npar; ++q) {
      if (!S.size[pl][q] || n_par[q] == 0) continue;
      if (near_pl.count((int64_t)p * npar + q)) continue;
      int found = -1, fe = -1;
      for (int d = 0; d < nlv && found < 0; ++d) {
        const int64_t nc = S.nclusters(pl - d);
        auto it = adm_index[d].find((int64_t)(p >> d) * nc + (q >> d));
        if (it != adm_index[d].end()) {
          found = d;
          fe = it->second;
        }
      }
      if (found < 0) fail(H2_ERR_INTERNAL, "early stop: a pair covered by no admissible block");
      if (kc(pl - found, p >> found) == 0 || kc(pl - found, q >> found) == 0) continue;
      far.push_back({p, q, found, fe});
      yoff.push_back(ytot);
      ytot += (int64_t)n_par[p] * kc(pl - found, q >> found);
    }
  }
  if (far.empty()) return;
  H->fb_Y.alloc(ytot);
  std::vector<GemmTask> t1, t2;
  for (size_t f = 0; f < far.size(); ++f) {
    const Far& F = far[f];
    const int lev = pl - F.d;
    const BuildLevel& Bl = H->build[L - lev];
    const int64_t kp = kc(lev, F.p >> F.d), kq = kc(lev, F.q >> F.d);
    GemmTask a{};
    a.A = H->fb_X.p + xoff[(size_t)F.d * npar + F.p];
    a.lda = n_par[F.p];
    a.B = Bl.S.p + Bl.soff[F.e];
    a.ldb = kp;
    a.C = H->fb_Y.p + yoff[f];
    a.ldc = n_par[F.p];
    a.m = n_par[F.p];
    a.n = (int32_t)kq;
    a.K = (int32_t)kp;
    a.opA = OP_N;
    a.opB = OP_N;
    a.mode = ST_SET;
    t1.push_back(a);
    GemmTask b{};
    b.A = H->fb_Y.p + yoff[f];
    b.lda = n_par[F.p];
    b.B = H->fb_X.p + xoff[(size_t)F.d * npar + F.q];
    b.ldb = n_par[F.q];
    b.C = H->Zf.p + H->final_off[F.p] + (int64_t)H->final_off[F.q] * H->nf;
    b.ldc = H->nf;
    b.m = n_par[F.p];
    b.n = n_par[F.q];
    b.K = (int32_t)kq;
    b.opA = OP_N;
    b.opB = OP_T;
    b.mode = ST_ADD;
    t2.push_back(b);
  }
  run_gemms(H, t1, st);
  run_gemms(H, t2, st);
}

// One factorization in progress (Alg. 1: per level, Steps 0-3 colour by colour,
// eqs. 16-31, then the merge into the parent level, eq. 23; the matrix left at
// the stop level is factored densely, Sec. III-C).  A single problem drives it
// level by level; a batch drives several in lockstep and launches each colour's
// kernels once for all of them (factor_fused).
struct FactorRun {
  h2_ctx* H;
  hipStream_t st;
  const Structure& S;
  int L, l0, ls = 0, l = 0, j = 0;
  bool own_memory, ktime, mixed, done = false;
  EventPool ev;
  std::vector<std::array<hipEvent_t, 4>> phase_ev;
  // per-kernel intervals when kernel timing is on: {begin, end, family}
  std::vector<std::tuple<hipEvent_t, hipEvent_t, int>> kern_ev;
  hipEvent_t t_begin = nullptr, e_level = nullptr, e_m0 = nullptr, e_m1 = nullptr;
  std::vector<int32_t> n_cur, kk, n_par, off1;
  std::vector<MergeTask> mt;  // kept until the merge's synchronisation
  int dmax = 1;
  int64_t gram_pstride = 0;
  bool split_ok = false;
  int64_t split_below = SCHUR_SPLIT_BELOW;
  bool mixed_flush = false;
  int32_t flags[4] = {0, 0, 0, 0};

  // With the library's own hipMalloc: when device memory is short, start from nothing
  // rather than from the previous factorization's buffers (its factors would sit beside
  // the new arenas).  A caller's allocator keeps what the library frees in its own cache
  // (so the device's free memory says nothing about it) and frees that cache itself when
  // an allocation fails: the handle keeps its buffers.
  bool memory_short() const {
    size_t fr = 0, tot = 0;
    return own_memory && hipMemGetInfo(&fr, &tot) == hipSuccess && (double)fr < 0.35 * (double)tot;
  }
  bool level_pending() const { return !done && l >= ls; }
  LevelPlan& plan() { return H->plans[j]; }
  FactorLevel& flev() { return H->flev[j]; }

  FactorRun(h2_ctx* h, hipStream_t s)
      : H(h), st(s), S(h->S), L(h->S.L), l0(h->S.l0), own_memory(!(h->allocator.alloc && h->allocator.free)),
        ktime(h->kernel_timing), mixed(h->precision == H2_MIXED) {
    H->factored = false;
    // buffers of the previous factorization are reused; nothing of it may still run
    HIPCHK(hipStreamSynchronize(st));
    if (memory_short()) release_factor_buffers(H);
    H->vbuf_nrhs = 0;  // level sizes may change with the ranks: resize the sweep buffers
    H->drop_graphs();
    H->timing.assign(6, 0.0);
    H->stats_rows.clear();
    H->level_ms.clear();
    H->merge_elems = 0;
    H->kernel_ms.assign(8, -1.0);
    t_begin = ev.next(st);
    if (l0 < 0) {
      // no admissible block anywhere: LU of the whole matrix
      H->nf = H->N;
      H->Zf.alloc((size_t)H->N * H->N);
      launch_zero(H->Zf.p, H->N * H->N, st);
      const auto& nl = S.near[L];
      for (size_t e = 0; e < nl.size(); ++e) {
        const int a = nl[e].first, b = nl[e].second;
        HIPCHK(hipMemcpy2DAsync(H->Zf.p + S.start[L][a] + S.start[L][b] * H->N, H->N * sizeof(double2),
                                H->near_orig.p + H->near_off[e], S.size[L][a] * sizeof(double2),
                                S.size[L][a] * sizeof(double2), S.size[L][b], hipMemcpyDeviceToDevice, st));
      }
      hipEvent_t t_m = ev.next(st);
      dense_lu_factor(H, st);
      hipEvent_t t_end = ev.next(st);
      HIPCHK(hipStreamSynchronize(st));
      H->timing[0] = elapsed(t_begin, t_end);
      H->timing[5] = elapsed(t_m, t_end);
      for (int f = 0; f < 7; ++f) H->kernel_ms[f] = 0.0;
      H->kernel_ms[7] = H->timing[5];
      H->ledger_valid = false;
      H->factored = true;
      done = true;
      return;
    }
    ls = H->stop;  // last factored level; the matrix merged to level ls - 1 is factored densely
    H->flev.resize(L - ls + 1);
    // block arenas of consecutive levels alternate between two handle-owned buffers
    n_cur.resize(S.nclusters(L));
    for (int t = 0; t < S.nclusters(L); ++t) n_cur[t] = (int32_t)S.size[L][t];
    l = L;
  }

  // Level l: sizes, offsets and work space, the blocks of the level (leaf blocks
  // or the merged parent blocks), the parent bases (eq. 23) and the complements
  // B_perp of every cluster (Step 0 starts from them).
  void level_begin() {
    j = L - l;
    split_below = (l < (int)H->split_below.size() && H->split_below[l] >= 0) ? H->split_below[l] : SCHUR_SPLIT_BELOW;
    LevelPlan& P = H->plans[j];
    BuildLevel& Bd = H->build[j];
    FactorLevel& F = H->flev[j];
    const int nc = P.nc;
    e_level = ev.next(st);
    F.n = n_cur;
    kk.assign(Bd.k.begin(), Bd.k.end());
    for (int t = 0; t < nc; ++t)
      if (!P.nonempty[t]) kk[t] = 0;
    int nmax = 0;
    dmax = 1;
    for (int t = 0; t < nc; ++t) {
      nmax = std::max(nmax, F.n[t]);
      if (F.n[t] < kk[t]) fail(H2_ERR_INTERNAL, "basis wider than its cluster");
      if (F.n[t] - kk[t] > STEP0_DMAX || kk[t] > STEP0_DMAX)
        fail(H2_ERR_INTERNAL, "level " + std::to_string(l) + " cluster " + std::to_string(t) + ": n = " +
                                  std::to_string(F.n[t]) + ", k = " + std::to_string(kk[t]) +
                                  " beyond the kernel limit of 512");
      dmax = std::max(dmax, F.n[t] - kk[t]);
    }
    if (nmax > 512) fail(H2_ERR_INTERNAL, "cluster dimension above 512 (kernel limit)");
    F.tiles = std::max(1, (nmax + 63) / 64);
    {
      int64_t dsum = 0, ncl = 0;
      for (int t = 0; t < nc; ++t)
        if (P.nonempty[t]) {
          dsum += F.n[t] - kk[t];
          ++ncl;
        }
      const int mf = l < (int)H->mixed_flush.size() ? H->mixed_flush[l] : -1;
      mixed_flush = mixed && (mf >= 0 ? mf != 0 : (ncl > 0 && (double)dsum / ncl >= MIXED_FLUSH_MIN_D));
      F.mixed_flush = mixed_flush;
    }
    // offsets
    std::vector<int64_t> slot_off(P.nslot + 1, 0);
    for (int s = 0; s < P.nslot; ++s)
      slot_off[s + 1] = slot_off[s] + (int64_t)F.n[P.slot_a[s]] * F.n[P.slot_b[s]];
    std::vector<int32_t> np_off(P.np_cl.size()), prow(nc, 0);
    for (int i = 0; i < nc; ++i) {
      int o = 0;
      for (int x = P.np_ptr[i]; x < P.np_ptr[i + 1]; ++x) {
        np_off[x] = o;
        o += F.n[P.np_cl[x]];
      }
      prow[i] = o;
    }
    std::vector<int64_t> q_off(nc + 1, 0), b_off(nc + 1, 0), bp_off(nc + 1, 0), lu_off(nc + 1, 0),
        cp_off(nc + 1, 0), w_off(nc + 1, 0);
    for (int i = 0; i < nc; ++i) {
      const int64_t n = F.n[i], k = kk[i], d = n - k;
      q_off[i + 1] = q_off[i] + n * n;
      b_off[i + 1] = b_off[i] + n * k;
      bp_off[i + 1] = bp_off[i] + n * d;
      lu_off[i + 1] = lu_off[i] + 2 * d * d;
      cp_off[i + 1] = cp_off[i] + (int64_t)prow[i] * d;
      w_off[i + 1] = w_off[i] + n * n + n * d + 2 * d * d;
    }
    // per-colour projection temp offsets
    int64_t temp_max = 0;
    for (ColourPlan& C : P.cols) {
      C.pj_toff.resize(C.pj_slot.size());
      int64_t o = 0;
      for (size_t e = 0; e < C.pj_slot.size(); ++e) {
        C.pj_toff[e] = o;
        const int s = C.pj_slot[e];
        o += (int64_t)F.n[P.slot_a[s]] * F.n[P.slot_b[s]];
      }
      H->stage.put(C.d_pj_toff, C.pj_toff);
      temp_max = std::max(temp_max, o);
    }
    F.ntot = 0;
    F.voff.assign(nc + 1, 0);
    for (int i = 0; i < nc; ++i) F.voff[i + 1] = F.voff[i] + F.n[i];
    F.ntot = F.voff[nc];
    // device arrays
    Stager& sg = H->stage;
    sg.put(F.d_n, F.n);
    sg.put(F.d_k, kk);
    sg.put(F.d_kt, kk);
    {
      std::vector<int32_t> fk(nc, -1);
      if (H->has_forced)
        for (int i = 0; i < nc; ++i) fk[i] = H->forced_kt[H->lvl_base[l] + i];
      sg.put(F.d_forced, fk);
    }
    sg.put(F.d_np_off, np_off);
    sg.put(F.d_prow, prow);
    sg.put(F.d_flags, std::vector<int32_t>(4, 0));
    sg.put(F.d_slot_off, slot_off);
    sg.put(F.d_q_off, q_off);
    sg.put(F.d_b_off, b_off);
    sg.put(F.d_bp_off, bp_off);
    sg.put(F.d_lu_off, lu_off);
    sg.put(F.d_cp_off, cp_off);
    sg.put(F.d_rp_off, cp_off);
    sg.put(F.d_w_off, w_off);
    sg.put(F.d_voff, F.voff);
    F.d_margins.alloc(2 * nc);
    if (mixed) {
      F.d_pmax.alloc(2 * nc);
      launch_zero(F.d_pmax.p, 2 * nc, st);
    }
    F.Q.alloc(q_off[nc]);
    F.LU.alloc(lu_off[nc]);
    F.CP.alloc(cp_off[nc]);
    F.RP.alloc(cp_off[nc]);
    DArr<double2>& slots = H->slot_buf[j & 1];
    DArr<double2>& parent_slots = H->slot_buf[(j + 1) & 1];
    DArr<double2>& Bp = H->ws_bp;
    DArr<double2>& W = H->ws_w;
    DArr<double2>& temp = H->ws_temp;
    DArr<double2>& lu_scr = H->ws_lu;
    DArr<double2>& eig_scr = H->ws_eig;
    DArr<double2>& gram_part = H->ws_gram;
    Bp.alloc(bp_off[nc]);
    W.alloc(w_off[nc]);
    if (F.tiles > 1) temp.alloc(temp_max);  // the one-tile levels project in place
    int maxcl = 1;
    for (ColourPlan& C : P.cols) maxcl = std::max<int>(maxcl, (int)C.cl.size());
    lu_scr.alloc((size_t)maxcl * ((size_t)dmax * dmax + dmax) * (dmax > LU_LDS_MAX ? 1 : 0) + 1);  // k_lu beyond its LDS size
    gram_pstride = (int64_t)maxcl * (F.tiles * 64) * (F.tiles * 64);
    gram_part.alloc((size_t)GRAM_SPLIT * gram_pstride);
    eig_scr.alloc((size_t)maxcl * 4 * dmax * dmax);
    // split Schur tasks: one 64 x 64 partial tile per (chunk, tile) when the level's
    // partial tiles fit in SCHUR_PART_MAX_BYTES, otherwise this level flushes every
    // block whole.  The choice depends on the level's sizes only (never on free
    // device memory), so a problem's arithmetic - the order in which a block's terms
    // are summed and, in the mixed form, which of them run in FP32 - is the same in
    // every run, batched or not; the buffer is kept for later factorizations.
    // A chunk of a split flush of block (a, b) keeps ceil(n_a / 64) ceil(n_b / 64) tiles.
    auto group_bases = [&](ColourPlan& C) -> int64_t {
      C.sc_gbase.resize(C.ngrp);
      int64_t run = 0;
      for (int g = 0; g < C.ngrp; ++g) {
        const int task = C.sc_gtask[g], sl = C.sc_slot[task];
        const int64_t ta = (F.n[P.slot_a[sl]] + 63) / 64, tb = (F.n[P.slot_b[sl]] + 63) / 64;
        C.sc_gbase[g] = (int32_t)run;
        run += (int64_t)C.sc_sp[4 * task + 1] * ta * tb;
      }
      return run;
    };
    int64_t max_tiles = group_bases(P.fin);
    for (ColourPlan& C : P.cols) max_tiles = std::max(max_tiles, group_bases(C));
    const size_t scp_elems = (size_t)std::max<int64_t>(1, max_tiles * 4096);
    split_ok = scp_elems * sizeof(double2) <= SCHUR_PART_MAX_BYTES;
    if (split_ok) {
      H->ws_scp.alloc(scp_elems);
      sg.put(P.fin.d_sc_gbase, P.fin.sc_gbase);
      for (ColourPlan& C : P.cols) sg.put(C.d_sc_gbase, C.sc_gbase);
    }
    // blocks of this level
    if (l == L) {
      slots.alloc(slot_off[P.nslot]);
      launch_zero(slots.p + slot_off[P.nnear], slot_off[P.nslot] - slot_off[P.nnear], st);  // fill blocks
      // inadmissible leaf blocks (a <= b) from the construction's near blocks
      {
        std::vector<int64_t> so(P.nnear), dofs(P.nnear), len(P.nnear);
        for (int e = 0; e < P.nnear; ++e) {
          so[e] = H->near_off[P.near_src[e]];
          dofs[e] = slot_off[e];
          len[e] = slot_off[e + 1] - slot_off[e];
        }
        DArr<int64_t>& d_so = H->lv_so;
        DArr<int64_t>& d_do = H->lv_do;
        DArr<int64_t>& d_len = H->lv_len;
        sg.put(d_so, so);
        sg.put(d_do, dofs);
        sg.put(d_len, len);
        sg.flush(st);
        launch_copy_blocks(H->near_orig.p, d_so.p, slots.p, d_do.p, d_len.p, P.nnear, st);
        check_launch("near block copy");
      }
      F.B.alloc(b_off[nc]);
      if (b_off[nc] > 0)
        HIPCHK(hipMemcpyAsync(F.B.p, Bd.basis.p, b_off[nc] * sizeof(double2), hipMemcpyDeviceToDevice, st));
    } else {
      // parent bases: transfer matrices padded with zero rows (eq. 23)
      const FactorLevel& Fc = H->flev[j - 1];
      const BuildLevel& Bc = H->build[j - 1];
      std::vector<int32_t> k1(nc), k2(nc), off1(nc);
      for (int p = 0; p < nc; ++p) {
        k1[p] = Bc.k[2 * p];
        k2[p] = Bc.k[2 * p + 1];
        off1[p] = H->plans[j - 1].nonempty[2 * p] ? Fc.kt[2 * p] : 0;
      }
      std::vector<int64_t> toff(Bd.boff.begin(), Bd.boff.end() - 1);
      DArr<int32_t>& d_k1 = H->lv_k1;
      DArr<int32_t>& d_k2 = H->lv_k2;
      DArr<int32_t>& d_off1 = H->lv_off1;
      DArr<int64_t>& d_toff = H->lv_toff;
      sg.put(d_k1, k1);
      sg.put(d_k2, k2);
      sg.put(d_off1, off1);
      sg.put(d_toff, toff);
      F.B.alloc(b_off[nc]);
      sg.flush(st);
      launch_parent_basis(nc, F.d_n.p, F.d_k.p, d_k1.p, d_k2.p, d_off1.p, d_toff.p, Bd.basis.p, F.d_b_off.p, F.B.p,
                          st);
      check_launch("host.cpp:997");
      HIPCHK(hipStreamSynchronize(st));
    }
    LevelView& v = F.view;
    v.nc = nc;
    v.n = F.d_n.p;
    v.k = F.d_k.p;
    v.kt = F.d_kt.p;
    v.colour = P.d_colour.p;
    v.nu = Bd.d_nu.p;
    v.forced = H->has_forced ? F.d_forced.p : nullptr;
    v.eps_fill = H->eps_fill;
    v.slot_off = F.d_slot_off.p;
    v.slot_a = P.d_slot_a.p;
    v.slot_b = P.d_slot_b.p;
    v.slots = slots.p;
    v.nnear = P.nnear;
    v.diag_slot = P.d_diag_slot.p;
    v.np_ptr = P.d_np_ptr.p;
    v.np_cl = P.d_np_cl.p;
    v.np_srow = P.d_np_srow.p;
    v.np_scol = P.d_np_scol.p;
    v.np_off = F.d_np_off.p;
    v.fp_ptr = P.d_fp_ptr.p;
    v.fp_cl = P.d_fp_cl.p;
    v.fp_srow = P.d_fp_srow.p;
    v.q_off = F.d_q_off.p;
    v.Q = F.Q.p;
    v.b_off = F.d_b_off.p;
    v.B = F.B.p;
    v.bp_off = F.d_bp_off.p;
    v.Bp = Bp.p;
    v.lu_off = F.d_lu_off.p;
    v.LU = F.LU.p;
    v.cp_off = F.d_cp_off.p;
    v.CP = F.CP.p;
    v.rp_off = F.d_rp_off.p;
    v.RP = F.RP.p;
    v.prow = F.d_prow.p;
    v.w_off = F.d_w_off.p;
    v.W = W.p;
    v.flags = F.d_flags.p;
    v.margins = F.d_margins.p;
    // panel maxima only where the flush routes by them
    v.pmax = mixed_flush ? reinterpret_cast<unsigned long long*>(F.d_pmax.p) : nullptr;
    hipEvent_t e_hp = ktime ? ev.next(st) : nullptr;
    launch_householder_perp(v, nc, st);
    check_launch("host.cpp:1040");
    if (ktime) kern_ev.emplace_back(e_hp, ev.next(st), 1);
  }
  void schur_lists(const ColourPlan& C, ColourTasks& ct) const {
    const int64_t t = H->flev[j].tiles;
    if (split_ok && C.ngrp > 0 && (int64_t)C.sc_slot_u.size() * t * t < split_below) {
      ct.sc_slot = C.d_sc_slot.p;
      ct.sc_cptr = C.d_sc_cptr.p;
      ct.sc_sp = C.d_sc_sp.p;
      ct.nsc = (int)C.sc_slot.size();
      ct.sc_gtask = C.d_sc_gtask.p;
      ct.sc_gbase = C.d_sc_gbase.p;
      ct.ngrp = C.ngrp;
      ct.sc_part = H->ws_scp.p;
    } else {
      ct.sc_slot = C.d_sc_slot_u.p;
      ct.sc_cptr = C.d_sc_cptr_u.p;
      ct.sc_sp = C.d_sc_sp_u.p;
      ct.nsc = (int)C.sc_slot_u.size();
      ct.sc_gtask = nullptr;
      ct.sc_gbase = nullptr;
      ct.ngrp = 0;
      ct.sc_part = nullptr;
    }
  }

  // the task lists of colour c (ct.colour = c: Steps 0-3 of its clusters)
  ColourTasks colour_tasks(int c) {
    ColourPlan& C = plan().cols[c];
    ColourTasks ct{};
    ct.cl = C.d_cl.p;
    ct.ncl = (int)C.cl.size();
    ct.pj_slot = C.d_pj_slot.p;
    ct.pj_toff = C.d_pj_toff.p;
    ct.npj = (int)C.pj_slot.size();
    ct.sc_i = C.d_sc_i.p;
    ct.sc_ja = C.d_sc_ja.p;
    ct.sc_jb = C.d_sc_jb.p;
    schur_lists(C, ct);
    ct.pn_i = C.d_pn_i.p;
    ct.pn_ja = C.d_pn_ja.p;
    ct.npn = (int)C.pn_i.size();
    ct.sv_cl = C.d_sv_cl.p;
    ct.sv_cptr = C.d_sv_cptr.p;
    ct.sv_i = C.d_sv_i.p;
    ct.sv_ja = C.d_sv_ja.p;
    ct.nsv = (int)C.sv_cl.size();
    ct.colour = c;
    ct.tiles = flev().tiles;
    return ct;
  }

  // the updates still pending at the end of the level
  ColourTasks fin_tasks() {
    LevelPlan& P = plan();
    ColourTasks ct{};
    ct.sc_i = P.fin.d_sc_i.p;
    ct.sc_ja = P.fin.d_sc_ja.p;
    ct.sc_jb = P.fin.d_sc_jb.p;
    schur_lists(P.fin, ct);
    ct.colour = P.ncol - 1;
    ct.tiles = flev().tiles;
    return ct;
  }

  // Colour c of the level: the flush of the updates its clusters receive from the
  // colours before it (the blocks as they are before colour c), then Step 0 (the
  // fill-in Gram and its eigenvectors, eqs. 16-17), the projections (eqs. 18-20),
  // the partial LU (eq. 21) and the panels (eqs. 22, 24-26).
  void run_colour(int c) {
    FactorLevel& F = flev();
    LevelView& v = F.view;
    ColourTasks ct = colour_tasks(c);
    ct.colour = c - 1;
    hipEvent_t es = ev.next(st);
    launch_schur(v, ct, mixed_flush, st);
    check_launch("schur");
    ct.colour = c;
    hipEvent_t e0 = ev.next(st);
    launch_gram_fill(v, ct, H->ws_gram.p, gram_pstride, st);
    check_launch("gram_fill");
    hipEvent_t eg = ktime ? ev.next(st) : nullptr;
    if (ktime) kern_ev.emplace_back(e0, eg, 0);
    launch_xform(v, ct, 0, st);
    launch_xform(v, ct, 1, st);
    check_launch("xform");
    launch_step0_eig(v, ct, H->ws_eig.p, dmax, st);
    check_launch("step0_eig");
    launch_xform(v, ct, 2, st);
    hipEvent_t ex = ktime ? ev.next(st) : nullptr;
    if (ktime) kern_ev.emplace_back(eg, ex, 1);
    if (F.tiles == 1) {
      launch_proj_fused(v, ct, mixed, st);
    } else {
      launch_proj(v, ct, H->ws_temp.p, 0, mixed, st);
      launch_proj(v, ct, H->ws_temp.p, 1, mixed, st);
    }
    check_launch("projection");
    hipEvent_t e1 = ev.next(st);
    if (ktime) kern_ev.emplace_back(ex, e1, 2);
    launch_lu(v, ct, H->ws_lu.p, dmax, st);
    check_launch("lu");
    hipEvent_t el = ktime ? ev.next(st) : nullptr;
    launch_panels(v, ct, st);
    check_launch("panels");
    hipEvent_t e2 = ev.next(st);
    if (ktime) {
      kern_ev.emplace_back(e1, el, 3);
      kern_ev.emplace_back(el, e2, 4);
    }
    phase_ev.push_back({es, e0, e1, e2});
  }

  void run_fin() {
    ColourTasks ct = fin_tasks();
    hipEvent_t es = ev.next(st);
    launch_schur(flev().view, ct, mixed_flush, st);
    check_launch("schur");
    hipEvent_t ee = ev.next(st);
    phase_ev.push_back({es, ee, ee, ee});
  }

  // The (kernel, entry) pairs of one stage of colour c for a shared launch; the
  // work space and the largest eliminated dimension travel in each entry.
  void stage_entries(int stage, int c, std::vector<std::pair<int, BatchEntry>>& out) {
    FactorLevel& F = flev();
    const bool fin = c >= plan().ncol;
    ColourTasks ct = fin ? fin_tasks() : colour_tasks(c);
    double2* buf = nullptr;
    int64_t aux = 0;
    switch (stage) {
      case BS_SCHUR:
      case BS_SCHUR_REDUCE:
        if (!fin) ct.colour = c - 1;
        break;
      case BS_GRAM:
      case BS_GRAM_REDUCE:
        buf = H->ws_gram.p;
        aux = gram_pstride;
        break;
      case BS_STEP0:
        buf = H->ws_eig.p;
        break;
      case BS_PROJ0:
      case BS_PROJ1:
        buf = H->ws_temp.p;
        break;
      case BS_LU:
        buf = H->ws_lu.p;
        break;
      default:
        break;
    }
    batch_stage_entries(stage, F.view, ct, mixed, mixed_flush, buf, aux, dmax, out);
  }

  // one synchronisation per level: ranks k~ and pivot status
  void readback() {
    FactorLevel& F = flev();
    const int nc = plan().nc;
    F.kt.assign(nc, 0);
    HIPCHK(hipMemcpyAsync(F.kt.data(), F.d_kt.p, nc * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(flags, F.d_flags.p, sizeof(flags), hipMemcpyDeviceToHost, st));
  }

  // after readback(): merge into the parent level (or the final dense block, with
  // the far blocks of the coarser levels when stopped early)
  void level_merge() {
    LevelPlan& P = plan();
    BuildLevel& Bd = H->build[j];
    FactorLevel& F = flev();
    const int nc = P.nc;
    if (flags[0]) fail(H2_ERR_SINGULAR, "zero pivot in the partial LU of a cluster at level " + std::to_string(l));
    for (int i = 0; i < nc; ++i)
      if (!P.nonempty[i]) F.kt[i] = 0;
    F.k = kk;
    DArr<double2>& parent_slots = H->slot_buf[(j + 1) & 1];
    LevelView& v = F.view;
    e_m0 = ev.next(st);
    const int npar = S.nclusters(l - 1);
    n_par.assign(npar, 0);
    off1.assign(npar, 0);
    for (int p = 0; p < npar; ++p) {
      off1[p] = P.nonempty[2 * p] ? F.kt[2 * p] : 0;
      n_par[p] = off1[p] + (P.nonempty[2 * p + 1] ? F.kt[2 * p + 1] : 0);
    }
    mt.assign(P.merge.size(), MergeTask{});
    int64_t dst_total = 0;
    std::vector<int64_t> pslot_off;
    if (l > ls) {
      const LevelPlan& Pp = H->plans[j + 1];
      pslot_off.assign(Pp.nslot + 1, 0);
      for (int s = 0; s < Pp.nslot; ++s)
        pslot_off[s + 1] = pslot_off[s] + (int64_t)n_par[Pp.slot_a[s]] * n_par[Pp.slot_b[s]];
      dst_total = pslot_off[Pp.nslot];
      for (size_t e = 0; e < P.merge.size(); ++e) {
        const MergeSrc& m = P.merge[e];
        if (m.pslot < 0 || m.pslot >= Pp.nslot) fail(H2_ERR_INTERNAL, "merge plan does not match the stop level");
        const int pa = Pp.slot_a[m.pslot], pb = Pp.slot_b[m.pslot];
        const int64_t ld = n_par[pa];
        const int64_t ro = m.ci ? off1[pa] : 0, co = m.dj ? off1[pb] : 0;
        MergeTask& t = mt[e];
        t.dst = pslot_off[m.pslot] + ro + co * ld;
        t.ldd = ld;
        t.kind = m.kind;
        t.slot = m.slot;
        t.ca = m.ca;
        t.cb = m.cb;
        t.soff = m.adm >= 0 ? Bd.soff[m.adm] : 0;
        t.ska = m.adm >= 0 ? Bd.k[m.ca] : 0;
        t.skb = m.adm >= 0 ? Bd.k[m.cb] : 0;
        t.tr = m.tr;
      }
    } else {
      H->final_off.assign(npar + 1, 0);
      for (int p = 0; p < npar; ++p) H->final_off[p + 1] = H->final_off[p] + n_par[p];
      H->nf = H->final_off[npar];
      H->stage.put(H->d_final_off, std::vector<int64_t>(H->final_off.begin(), H->final_off.end() - 1));
      dst_total = H->nf * H->nf;
      for (size_t e = 0; e < P.merge.size(); ++e) {
        const MergeSrc& m = P.merge[e];
        if (m.pslot < 0 || m.pslot >= npar * npar) fail(H2_ERR_INTERNAL, "merge plan does not match the stop level");
        const int pa = m.pslot / npar, pb = m.pslot % npar;
        const int64_t ro = H->final_off[pa] + (m.ci ? off1[pa] : 0);
        const int64_t co = H->final_off[pb] + (m.dj ? off1[pb] : 0);
        MergeTask& t = mt[e];
        t.dst = ro + co * H->nf;
        t.ldd = H->nf;
        t.kind = m.kind;
        t.slot = m.slot;
        t.ca = m.ca;
        t.cb = m.cb;
        t.soff = m.adm >= 0 ? Bd.soff[m.adm] : 0;
        t.ska = m.adm >= 0 ? Bd.k[m.ca] : 0;
        t.skb = m.adm >= 0 ? Bd.k[m.cb] : 0;
        t.tr = m.tr;
      }
    }
    DArr<MergeTask>& d_mt = H->ws_merge;
    H->stage.put(d_mt, mt);
    H->stage.flush(st);
    double2* dst;
    if (l > ls) {
      parent_slots.alloc(dst_total);
      dst = parent_slots.p;
    } else {
      H->Zf.alloc(dst_total);
      dst = H->Zf.p;
    }
    H->merge_elems += (double)dst_total;
    launch_zero(dst, dst_total, st);
    launch_merge(v, d_mt.p, (int)mt.size(), Bd.S.p, dst, st);
    check_launch("merge");
    if (l == ls && ls > l0) add_far_blocks(H, ls, n_par, off1, st);
    e_m1 = ev.next(st);
  }

  // after the merge's synchronisation: timings, the level's stats row, next level
  void level_close() {
    LevelPlan& P = plan();
    FactorLevel& F = flev();
    const int nc = P.nc;
    DArr<double2>& slots = H->slot_buf[j & 1];
    H->timing[4] += elapsed(e_m0, e_m1);
    H->level_ms.push_back(elapsed(e_level, e_m1));
    // stats row
    {
      int64_t sn = 0, mn = 0, sk = 0, mk = 0, skt = 0, mkt = 0, nkt = INT64_MAX, el = 0, ncl = 0;
      for (int i = 0; i < nc; ++i) {
        if (!P.nonempty[i]) continue;
        ++ncl;
        sn += F.n[i];
        mn = std::max<int64_t>(mn, F.n[i]);
        sk += kk[i];
        mk = std::max<int64_t>(mk, kk[i]);
        skt += F.kt[i];
        mkt = std::max<int64_t>(mkt, F.kt[i]);
        nkt = std::min<int64_t>(nkt, F.kt[i]);
        el += F.n[i] - F.kt[i];
      }
      H->stats_rows.push_back({l, ncl, sn, mn, sk, mk, skt, mkt, ncl ? nkt : 0, el});
    }
    n_cur = n_par;
    // keep this level's block arena for the next factorization unless memory is
    // short (the level two steps up reuses it; keeping it costs its full size)
    if (memory_short()) slots.release();
    --l;
  }

  // the final dense block (eq. 34 at the top of the tree or at the stop level), timings
  void finish() {
    hipEvent_t e_f0 = ev.next(st);
    dense_lu_factor(H, st);
    hipEvent_t t_end = ev.next(st);
    HIPCHK(hipStreamSynchronize(st));
    H->stats_rows.push_back({ls - 1, (int64_t)S.nclusters(ls - 1), H->nf, H->nf, 0, 0, 0, 0, 0, H->nf});
    H->timing[5] = elapsed(e_f0, t_end);
    H->level_ms.push_back(H->timing[5]);
    for (auto& pe : phase_ev) {
      H->timing[3] += elapsed(pe[0], pe[1]);
      H->timing[1] += elapsed(pe[1], pe[2]);
      H->timing[2] += elapsed(pe[2], pe[3]);
    }
    H->timing[0] = elapsed(t_begin, t_end);
    if (!phase_ev.empty()) {  // a fused batch's launches serve every problem: no per-kernel times
      if (ktime) {
        for (int f = 0; f < 5; ++f) H->kernel_ms[f] = 0.0;
        for (auto& ke : kern_ev) H->kernel_ms[std::get<2>(ke)] += elapsed(std::get<0>(ke), std::get<1>(ke));
      }
      H->kernel_ms[5] = H->timing[3];
      H->kernel_ms[6] = H->timing[4];
    }
    H->kernel_ms[7] = H->timing[5];
    H->ledger_valid = false;
    H->factored = true;
  }
};

static void factor_impl(h2_ctx* H, hipStream_t st) {
  FactorRun R(H, st);
  while (R.level_pending()) {
    R.level_begin();
    for (int c = 0; c < R.plan().ncol; ++c) R.run_colour(c);
    R.run_fin();
    R.readback();
    HIPCHK(hipStreamSynchronize(st));
    R.level_merge();
    HIPCHK(hipStreamSynchronize(st));
    R.level_close();
  }
  if (!R.done) R.finish();
}


// P Z_f = L U by blocked LU with partial pivoting (64-column panels, GEMM
// trailing updates), in place; the inverses of the 64 x 64 diagonal blocks of L
// and U are kept for the blocked triangular solves of the sweeps, and the row
// interchanges become one gather permutation.
static void dense_lu_factor(h2_ctx* H, hipStream_t st) {
  const int64_t n = H->nf;
  if (n == 0) return;
  double2* A = H->Zf.p;
  DArr<int32_t>& piv = H->dl_piv;
  DArr<int32_t>& flag = H->dl_flag;
  piv.alloc(n);
  flag.alloc(1);
  HIPCHK(hipMemsetAsync(flag.p, 0, sizeof(int32_t), st));
  const int64_t nb = (n + 63) / 64;
  DArr<double2>& linv = H->dl_linv;
  DArr<double2>& uinv = H->dl_uinv;
  linv.alloc(nb * 64 * 64);
  uinv.alloc(nb * 64 * 64);
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t j0 = b * 64, w = std::min<int64_t>(64, n - j0), rest = n - j0 - w;
    launch_dense_panel(A, n, j0, piv.p, linv.p + b * 4096, flag.p, st);
    check_launch("dense panel");
    if (rest > 0) {
      // U12 = L11^-1 A12 (in place: one tile row owns all 64 rows of its columns)
      launch_gemm_one({linv.p + b * 4096, A + j0 + (j0 + w) * n, A + j0 + (j0 + w) * n, 64, n, n, (int32_t)w,
                       (int32_t)rest, (int32_t)w, OP_N, OP_N, ST_SET},
                      st);
      // A22 -= L21 U12
      launch_gemm_one({A + (j0 + w) + j0 * n, A + j0 + (j0 + w) * n, A + (j0 + w) + (j0 + w) * n, n, n, n,
                       (int32_t)rest, (int32_t)rest, (int32_t)w, OP_N, OP_N, ST_SUB},
                      st);
      check_launch("dense trailing update");
    }
  }
  int32_t hf = 0;
  HIPCHK(hipMemcpyAsync(&hf, flag.p, sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (hf) fail(H2_ERR_SINGULAR, "zero pivot in the final dense LU");
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t j0 = b * 64, w = std::min<int64_t>(64, n - j0);
    launch_tri_inv_upper(A + j0 + j0 * n, n, (int)w, uinv.p + b * 4096, st);
  }
  check_launch("diagonal block inverses");
  // the row interchanges applied in order, as one gather: (P v)[i] = v[perm[i]]
  std::vector<int32_t> pv(n), perm(n);
  HIPCHK(hipMemcpyAsync(pv.data(), piv.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t j = 0; j < n; ++j) {
    if (pv[j] < j || pv[j] >= n) fail(H2_ERR_INTERNAL, "final LU pivot out of range");
    std::swap(perm[j], perm[pv[j]]);
  }
  H->dl_perm.upload(perm, st);
}

// y = Z_f^-1 x (adj = 0) or Z_f^-H x (adj = 1) with the final block's LU factors:
// gather, L forward, U backward (or U^H forward, L^H backward, scatter).  x is
// used as work space and overwritten; the result goes to y.  No host synchronisation.
static void dense_lu_apply(h2_ctx* H, double2* x, double2* y, int nrhs, int adj, hipStream_t st) {
  const int64_t n = H->nf;
  if (n == 0) return;
  const double2* A = H->Zf.p;
  const int64_t nb = (n + 63) / 64;
  const double2* linv = H->dl_linv.p;
  const double2* uinv = H->dl_uinv.p;
  if (nrhs > SMALL_RHS) {
    // many right-hand sides: each block step as two matrix-core GEMMs, y_b = D x_b
    // (D or D^H) and the coupling update of the unsolved rows (ST_SUB)
    double2* A0 = H->Zf.p;
    auto step = [&](int64_t j0, int mode, const double2* D, double2* xin, double2* yout) {
      const int w = (int)std::min<int64_t>(64, n - j0);
      const bool fwd = (mode == 0 || mode == 2), herm = (mode >= 2);
      launch_gemm_one({D, xin + j0, yout + j0, 64, n, n, w, nrhs, w, herm ? OP_C : OP_N, OP_N, ST_SET}, st);
      const int64_t r0 = fwd ? j0 + w : 0, rows = fwd ? n - j0 - w : j0;
      if (rows <= 0) return;
      // coupling of the block's columns (L or U below / above it) or, for the adjoint, of its rows
      const double2* Ac = herm ? A0 + j0 + r0 * n : A0 + r0 + j0 * n;
      launch_gemm_one({Ac, yout + j0, xin + r0, n, n, n, (int32_t)rows, nrhs, w, herm ? OP_C : OP_N, OP_N, ST_SUB},
                      st);
    };
    if (!adj) {
      launch_dense_perm(x, y, H->dl_perm.p, n, nrhs, n, 0, st);  // y = P x
      for (int64_t b = 0; b < nb; ++b) step(b * 64, 0, linv + b * 4096, y, x);        // x = L^-1 y
      for (int64_t b = nb - 1; b >= 0; --b) step(b * 64, 1, uinv + b * 4096, x, y);   // y = U^-1 x
    } else {
      for (int64_t b = 0; b < nb; ++b) step(b * 64, 2, uinv + b * 4096, x, y);        // y = U^-H x
      for (int64_t b = nb - 1; b >= 0; --b) step(b * 64, 3, linv + b * 4096, y, x);   // x = L^-H y
      launch_dense_perm(x, y, H->dl_perm.p, n, nrhs, n, 1, st);  // y = P^T x
    }
    check_launch("final block solve");
    return;
  }
  if (!adj) {
    launch_dense_perm(x, y, H->dl_perm.p, n, nrhs, n, 0, st);  // y = P x
    for (int64_t b = 0; b < nb; ++b)                            // x = L^-1 y
      launch_dense_trsv_step(A, n, b * 64, (int)std::min<int64_t>(64, n - b * 64), linv + b * 4096, y, x, n, nrhs,
                             0, st);
    for (int64_t b = nb - 1; b >= 0; --b)                       // y = U^-1 x
      launch_dense_trsv_step(A, n, b * 64, (int)std::min<int64_t>(64, n - b * 64), uinv + b * 4096, x, y, n, nrhs,
                             1, st);
  } else {
    for (int64_t b = 0; b < nb; ++b)                            // y = U^-H x
      launch_dense_trsv_step(A, n, b * 64, (int)std::min<int64_t>(64, n - b * 64), uinv + b * 4096, x, y, n, nrhs,
                             2, st);
    for (int64_t b = nb - 1; b >= 0; --b)                       // x = L^-H y
      launch_dense_trsv_step(A, n, b * 64, (int)std::min<int64_t>(64, n - b * 64), linv + b * 4096, y, x, n, nrhs,
                             3, st);
    launch_dense_perm(x, y, H->dl_perm.p, n, nrhs, n, 1, st);  // y = P^T x
  }
  check_launch("final block solve");
}

// ---------------------------------------------------------------------------
// sweeps
// ---------------------------------------------------------------------------
// Element counts of the sweep work buffers for nrhs right-hand sides: one
// vector per factored level, three N-vectors (final block in / out and the
// solve's own copy), the many-RHS panel scratch and the backward gather's
// partial sums.
struct SweepLayout {
  std::vector<int64_t> vbuf;
  int64_t vtmp = 0, vtmp3 = 0, scratch = 0, part = 0;
  int64_t total() const {
    int64_t t = 2 * vtmp + vtmp3 + scratch + part;
    for (int64_t v : vbuf) t += v;
    return t;
  }
};

static SweepLayout sweep_layout(const h2_ctx* H, int nrhs) {
  SweepLayout L;
  L.vbuf.resize(H->flev.size());
  for (size_t j = 0; j < H->flev.size(); ++j) L.vbuf[j] = std::max<int64_t>(1, H->flev[j].ntot) * nrhs;
  L.vtmp = std::max<int64_t>(1, std::max(H->nf, H->N)) * nrhs;
  L.vtmp3 = std::max<int64_t>(1, H->N) * nrhs;
  // per colour cluster: one (64 tiles) x 64 panel per block of 64 right-hand sides
  // (many RHS), SV_SPLIT partial vectors of SMALL_RHS columns (few RHS)
  int64_t blk = 1, blk_small = 1;
  for (size_t j = 0; j < H->flev.size(); ++j) {
    int maxcl = 1;
    for (const ColourPlan& C : H->plans[j].cols) maxcl = std::max<int>(maxcl, (int)C.cl.size());
    const int64_t ldp = (int64_t)H->flev[j].tiles * 64;
    blk = std::max<int64_t>(blk, (int64_t)maxcl * ldp * 64);
    blk_small = std::max<int64_t>(blk_small, (int64_t)maxcl * ldp * SMALL_RHS * SV_SPLIT);
  }
  if (nrhs <= SMALL_RHS) {
    L.scratch = 1;
    L.part = blk_small;
  } else {
    const int64_t zb = (nrhs + 63) / 64;
    L.scratch = blk * zb;
    L.part = blk * zb * BWD_SPLIT;
  }
  return L;
}

static void ensure_vbuf(h2_ctx* H, int nrhs) {
  if (H->vbuf_nrhs >= nrhs && !H->vbuf.empty()) return;
  H->drop_graphs();  // captured sweeps point at the old buffers
  const SweepLayout L = sweep_layout(H, nrhs);
  H->vbuf.resize(H->flev.size());  // existing buffers are kept when large enough
  for (size_t j = 0; j < H->flev.size(); ++j) H->vbuf[j].alloc(L.vbuf[j]);
  H->vtmp.alloc(L.vtmp);
  H->vtmp2.alloc(L.vtmp);
  H->vtmp3.alloc(L.vtmp3);
  H->sw_scratch.alloc(L.scratch);
  H->sw_part.alloc(L.part);
  H->vbuf_nrhs = nrhs;
}

static ColourTasks colour_tasks(const ColourPlan& C, int c, int tiles) {
  ColourTasks ct{};
  ct.cl = C.d_cl.p;
  ct.ncl = (int)C.cl.size();
  ct.sv_cl = C.d_sv_cl.p;
  ct.sv_cptr = C.d_sv_cptr.p;
  ct.sv_i = C.d_sv_i.p;
  ct.sv_ja = C.d_sv_ja.p;
  ct.nsv = (int)C.sv_cl.size();
  ct.colour = c;
  ct.tiles = tiles;
  return ct;
}

// Device work buffers of one sweep (laid out by sweep_layout).
struct SweepBufs {
  std::vector<double2*> vbuf;
  double2 *vtmp = nullptr, *vtmp2 = nullptr, *vtmp3 = nullptr, *scratch = nullptr, *part = nullptr;
};

static SweepBufs handle_bufs(h2_ctx* H, int nrhs) {
  ensure_vbuf(H, nrhs);
  SweepBufs B;
  for (auto& v : H->vbuf) B.vbuf.push_back(v.p);
  B.vtmp = H->vtmp.p;
  B.vtmp2 = H->vtmp2.p;
  B.vtmp3 = H->vtmp3.p;
  B.scratch = H->sw_scratch.p;
  B.part = H->sw_part.p;
  return B;
}

// in (tree order, ld N) -> out (tree order, ld N): out = M^-1 in (adj = 0) or M^-H in (adj = 1), on Z
static void sweep(h2_ctx* H, const SweepBufs& W, const double2* in, double2* out, int nrhs, int adj, hipStream_t st) {
  const Structure& S = H->S;
  const int64_t N = H->N;
  if (H->flev.empty()) {
    HIPCHK(hipMemcpyAsync(W.vtmp, in, N * nrhs * sizeof(double2), hipMemcpyDeviceToDevice, st));
    dense_lu_apply(H, W.vtmp, W.vtmp2, nrhs, adj, st);
    HIPCHK(hipMemcpyAsync(out, W.vtmp2, N * nrhs * sizeof(double2), hipMemcpyDeviceToDevice, st));
    check_launch("host.cpp:1314");
    return;
  }
  const int nlev = (int)H->flev.size();
  // level L vector = input
  HIPCHK(hipMemcpyAsync(W.vbuf[0], in, N * nrhs * sizeof(double2), hipMemcpyDeviceToDevice, st));
  for (int j = 0; j < nlev; ++j) {
    FactorLevel& F = H->flev[j];
    LevelPlan& P = H->plans[j];
    for (int c = 0; c < P.ncol; ++c) {
      ColourTasks ct = colour_tasks(P.cols[c], c, F.tiles);
      launch_sweep_fwd(F.view, ct, W.vbuf[j], F.d_voff.p, F.ntot, nrhs, adj, W.scratch, st);
    }
    const int npar = S.nclusters(P.l - 1);
    if (j + 1 < nlev) {
      FactorLevel& Fp = H->flev[j + 1];
      launch_vmerge(npar, F.d_kt.p, F.d_voff.p, Fp.d_voff.p, F.ntot, Fp.ntot, nrhs, W.vbuf[j], W.vbuf[j + 1], 1,
                    P.d_nonempty.p, st);
    } else {
      launch_vmerge(npar, F.d_kt.p, F.d_voff.p, H->d_final_off.p, F.ntot, H->nf, nrhs, W.vbuf[j], W.vtmp, 1,
                    P.d_nonempty.p, st);
      dense_lu_apply(H, W.vtmp, W.vtmp2, nrhs, adj, st);
      launch_vmerge(npar, F.d_kt.p, F.d_voff.p, H->d_final_off.p, F.ntot, H->nf, nrhs, W.vbuf[j], W.vtmp2, 0,
                    P.d_nonempty.p, st);
      check_launch("final block");
    }
    check_launch("host.cpp:1345");
  }
  for (int j = nlev - 1; j >= 0; --j) {
    FactorLevel& F = H->flev[j];
    LevelPlan& P = H->plans[j];
    if (j + 1 < nlev) {
      FactorLevel& Fp = H->flev[j + 1];
      launch_vmerge(S.nclusters(P.l - 1), F.d_kt.p, F.d_voff.p, Fp.d_voff.p, F.ntot, Fp.ntot, nrhs, W.vbuf[j],
                    W.vbuf[j + 1], 0, P.d_nonempty.p, st);
    }
    for (int c = P.ncol - 1; c >= 0; --c) {
      ColourTasks ct = colour_tasks(P.cols[c], c, F.tiles);
      launch_sweep_bwd(F.view, ct, W.vbuf[j], F.d_voff.p, F.ntot, nrhs, adj, W.part, BWD_SPLIT,
                       W.scratch, st);
    }
    check_launch("host.cpp:1359");
  }
  HIPCHK(hipMemcpyAsync(out, W.vbuf[0], N * nrhs * sizeof(double2), hipMemcpyDeviceToDevice, st));
}

// The sweep on H->vtmp3 in place, replayed from a captured graph when enabled.
static void sweep_vtmp3(h2_ctx* H, int nrhs, int adj, hipStream_t st) {
  const SweepBufs W = handle_bufs(H, nrhs);
  if (!H->use_graph || H->flev.empty()) {
    sweep(H, W, H->vtmp3.p, H->vtmp3.p, nrhs, adj, st);
    return;
  }
  const auto key = std::make_pair(nrhs, adj);
  auto it = H->sweep_graphs.find(key);
  if (it == H->sweep_graphs.end()) {
    if (!H->cap_stream) HIPCHK(hipStreamCreateWithFlags(&H->cap_stream, hipStreamNonBlocking));
    // the capture stream starts after everything queued on st so far
    hipEvent_t ev;
    HIPCHK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ev, st));
    HIPCHK(hipStreamWaitEvent(H->cap_stream, ev, 0));
    HIPCHK(hipStreamSynchronize(H->cap_stream));
    (void)hipEventDestroy(ev);
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(H->cap_stream, hipStreamCaptureModeThreadLocal));
    try {
      sweep(H, W, H->vtmp3.p, H->vtmp3.p, nrhs, adj, H->cap_stream);
    } catch (...) {
      (void)hipStreamEndCapture(H->cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    HIPCHK(hipStreamEndCapture(H->cap_stream, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(e);
    it = H->sweep_graphs.emplace(key, ex).first;
  }
  HIPCHK(hipGraphLaunch(it->second, st));
}

// y (tree order) = Z_H2 v (tree order)
static void matvec_tree(h2_ctx* H, const double2* v, double2* y, int nrhs, hipStream_t st) {
  const Structure& S = H->S;
  const int64_t N = H->N;
  const int L = S.L;
  launch_near_mv(S.nclusters(L), H->d_near_ptr.p, H->d_near_col.p, H->d_near_off.p, H->near_orig.p,
                 H->d_leaf_start.p, H->d_leaf_size.p, v, y, N, nrhs, st);
  check_launch("host.cpp:1371");
  if (S.l0 < 0) return;
  for (int l = S.l0; l <= L; ++l) {
    BuildLevel& B = H->build[L - l];
    const int nc = S.nclusters(l);
    if (B.ktot == 0) continue;
    DArr<double2>& xh = B.mv_x;
    DArr<double2>& yh = B.mv_y;
    xh.alloc(B.ktot * nrhs);
    yh.alloc(B.ktot * nrhs);
    launch_basis_mv(nc, B.d_rows.p, B.d_k.p, B.d_voff.p, B.V.p, B.d_cstart.p, v, B.d_xoff.p, xh.p, N, B.ktot, nrhs, 1,
                    0, st);
    launch_coupling_mv(nc, B.d_cptr.p, B.d_ccol.p, B.d_soff.p, B.d_k.p, B.d_k.p, B.S.p, B.d_xoff.p, xh.p, B.d_xoff.p,
                       yh.p, B.ktot, nrhs, st);
    launch_basis_mv(nc, B.d_rows.p, B.d_k.p, B.d_voff.p, B.V.p, B.d_xoff.p, yh.p, B.d_cstart.p, y, B.ktot, N, nrhs, 0,
                    1, st);
    check_launch("matvec level");
  }
}

}  // namespace h2

// ===========================================================================
// C ABI
// ===========================================================================
using namespace h2;

template <typename Fn>
static h2_status guarded(Fn&& fn) {
  try {
    g_err.clear();
    fn();
    return H2_OK;
  } catch (const Fail& f) {
    g_err = f.msg;
    return f.st;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return H2_ERR_OOM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return H2_ERR_INTERNAL;
  } catch (...) {
    g_err = "unknown failure";
    return H2_ERR_INTERNAL;
  }
}

static void check_device() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n < 1) fail(H2_ERR_DEVICE, "no HIP device available");
  hipDeviceProp_t prop;
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    fail(H2_ERR_DEVICE, std::string("device is ") + prop.gcnArchName + ", the library is built for gfx950");
  if (prop.sharedMemPerBlock < 140 * 1024)
    fail(H2_ERR_DEVICE, "device reports " + std::to_string(prop.sharedMemPerBlock) +
                            " bytes of LDS per workgroup; the eigensolver kernels need 137256");
}

static void validate_build(const double* points, int64_t n, double k, double h, const double* contrast, int32_t leaf,
                           double eta, double eps, const h2_options* opt, h2_handle* out) {
  if (!out) fail(H2_ERR_ARG, "out is NULL");
  if (!points || !contrast) fail(H2_ERR_ARG, "points or contrast is NULL");
  if (n < 1) fail(H2_ERR_ARG, "n < 1");
  if (!(k > 0) || !std::isfinite(k)) fail(H2_ERR_ARG, "k must be finite and > 0");
  if (!(h > 0) || !std::isfinite(h)) fail(H2_ERR_ARG, "h must be finite and > 0");
  if (leaf < 1) fail(H2_ERR_ARG, "leaf < 1");
  if (!(eta >= 0) || !std::isfinite(eta)) fail(H2_ERR_ARG, "eta must be finite and >= 0");
  if (!(eps > 0 && eps < 1)) fail(H2_ERR_ARG, "eps must lie in (0, 1)");
  for (int64_t i = 0; i < n; ++i) {
    if (!(contrast[i] > 0) || !std::isfinite(contrast[i])) fail(H2_ERR_ARG, "contrast must be finite and > 0");
    for (int d = 0; d < 3; ++d)
      if (!std::isfinite(points[3 * i + d])) fail(H2_ERR_ARG, "points must be finite");
  }
  if (opt) {
    if (opt->struct_size != sizeof(h2_options)) fail(H2_ERR_ARG, "h2_options.struct_size mismatch");
    if (opt->precision != H2_FP64 && opt->precision != H2_MIXED) fail(H2_ERR_ARG, "unknown precision");
    if (opt->order != H2_ORDER_COLOR) fail(H2_ERR_ARG, "unknown elimination order");
    if (!std::isfinite(opt->eps_fill) || opt->eps_fill >= 1) fail(H2_ERR_ARG, "eps_fill must be < 1");
    if (opt->forced_ranks && (opt->forced_ranks_len < 0 || opt->forced_ranks_len % 4))
      fail(H2_ERR_ARG, "forced_ranks_len must be a multiple of 4");
  }
}

extern "C" h2_status h2_structure(const double* points, int64_t n, double h, int32_t leaf, double eta, int64_t* counts,
                                  int64_t* perm, int32_t* colours) {
  return guarded([&] {
    if (!points || !counts) fail(H2_ERR_ARG, "points or counts is NULL");
    if (n < 1 || leaf < 1 || !(h > 0) || !(eta >= 0)) fail(H2_ERR_ARG, "invalid size or parameter");
    Structure S;
    std::vector<char> msg;
    if (!build_structure(points, n, h, leaf, eta, S, msg)) fail(H2_ERR_ARG, msg.data());
    const int L = S.L;
    int64_t mn = INT64_MAX, mx = 0;
    for (int64_t s : S.size[L]) {
      mn = std::min(mn, s);
      mx = std::max(mx, s);
    }
    counts[0] = n;
    counts[1] = L;
    counts[2] = S.l0;
    counts[3] = S.nclusters(L);
    counts[4] = mn;
    counts[5] = mx;
    counts[6] = (int64_t)S.adm[L].size();
    counts[7] = (int64_t)S.near[L].size();
    if (perm) std::memcpy(perm, S.perm.data(), n * sizeof(int64_t));
    if (colours) std::memcpy(colours, S.colour[L].data(), S.colour[L].size() * sizeof(int32_t));
  });
}

extern "C" h2_status h2_schur_schedule(const double* points, int64_t n, double h, int32_t leaf, double eta,
                                       int32_t level, int32_t* ncolours, int64_t* out, int64_t cap, int64_t* count) {
  return guarded([&] {
    if (!points || !ncolours || !count) fail(H2_ERR_ARG, "points, ncolours or count is NULL");
    if (n < 1 || leaf < 1 || !(h > 0) || !(eta >= 0)) fail(H2_ERR_ARG, "invalid size or parameter");
    std::unique_ptr<h2_ctx> H(new h2_ctx());
    std::vector<char> msg;
    if (!build_structure(points, n, h, leaf, eta, H->S, msg)) fail(H2_ERR_ARG, msg.data());
    const Structure& S = H->S;
    if (S.l0 < 0 || level < S.l0 || level > S.L) fail(H2_ERR_ARG, "level outside [l0, L]");
    LevelPlan P;
    build_plan_level(H.get(), level, P);
    int64_t terms = (int64_t)P.fin.sc_i.size();
    for (const ColourPlan& C : P.cols) terms += (int64_t)C.sc_i.size();
    *ncolours = P.ncol;
    *count = terms;
    if (!out) return;
    if (cap < 4 * terms) fail(H2_ERR_ARG, "cap < 4 * terms");
    int64_t w = 0;
    auto emit = [&](const ColourPlan& C, int ev) {
      for (size_t u = 0; u < C.sc_slot_u.size(); ++u) {
        const int s2 = C.sc_slot_u[u];
        for (int32_t q = C.sc_cptr_u[u]; q < C.sc_cptr_u[u + 1]; ++q) {
          out[w++] = ev;
          out[w++] = P.slot_a[s2];
          out[w++] = P.slot_b[s2];
          out[w++] = C.sc_i[q];
        }
      }
    };
    for (int c = 0; c < P.ncol; ++c) emit(P.cols[c], c);
    emit(P.fin, P.ncol);
  });
}

extern "C" h2_status h2_merge_schedule(const double* points, int64_t n, double h, int32_t leaf, double eta,
                                       int32_t level, int64_t* out, int64_t cap, int64_t* count) {
  return guarded([&] {
    if (!points || !count) fail(H2_ERR_ARG, "points or count is NULL");
    if (n < 1 || leaf < 1 || !(h > 0) || !(eta >= 0)) fail(H2_ERR_ARG, "invalid size or parameter");
    std::unique_ptr<h2_ctx> H(new h2_ctx());
    std::vector<char> msg;
    if (!build_structure(points, n, h, leaf, eta, H->S, msg)) fail(H2_ERR_ARG, msg.data());
    const Structure& S = H->S;
    if (S.l0 < 0 || level < S.l0 || level > S.L) fail(H2_ERR_ARG, "level outside [l0, L]");
    LevelPlan P, Pp;
    build_plan_level(H.get(), level, P);
    const bool to_final = level == S.l0;
    if (!to_final) build_plan_level(H.get(), level - 1, Pp);
    build_merge(H.get(), P, to_final ? nullptr : &Pp);
    const int npar = S.nclusters(level - 1);
    *count = (int64_t)P.merge.size();
    if (!out) return;
    if (cap < 7 * *count) fail(H2_ERR_ARG, "cap < 7 * records");
    int64_t w = 0;
    for (const MergeSrc& m : P.merge) {
      out[w++] = to_final ? m.pslot / npar : Pp.slot_a[m.pslot];
      out[w++] = to_final ? m.pslot % npar : Pp.slot_b[m.pslot];
      out[w++] = m.ci;
      out[w++] = m.dj;
      out[w++] = m.kind;
      out[w++] = m.ca;
      out[w++] = m.cb;
    }
  });
}

// Contrast-dependent device arrays: chi in tree and caller order and the
// scalings D = diag(k^2 h^3 chi) (matvec) and D^-1 (solve).
static void upload_contrast(h2_ctx* H, const double* contrast, hipStream_t st) {
  const int64_t n = H->N;
  const double k2h3 = H->k * H->k * std::pow(H->h, 3.0);
  std::vector<double> chi(n), ssolve(n), smat(n);
  for (int64_t t = 0; t < n; ++t) {
    const int64_t i = H->S.perm[t];
    chi[t] = contrast[i];
    smat[t] = k2h3 * contrast[i];
    ssolve[t] = 1.0 / smat[t];
  }
  H->chi_tree = chi;
  H->d_chi.upload(chi, st);
  H->d_chi_user.upload(std::vector<double>(contrast, contrast + n), st);
  H->d_scale_solve.upload(ssolve, st);
  H->d_scale_mat.upload(smat, st);
}

static void validate_contrast(const double* contrast, int64_t n) {
  if (!contrast) fail(H2_ERR_ARG, "contrast is NULL");
  for (int64_t i = 0; i < n; ++i)
    if (!(contrast[i] > 0.0) || !std::isfinite(contrast[i])) fail(H2_ERR_ARG, "contrast must be finite and > 0");
}

extern "C" h2_status h2_build(const double* points, int64_t n, double k, double h, const double* contrast, int32_t leaf,
                              double eta, double eps, const h2_options* opt, void* hip_stream, h2_handle* out) {
  return guarded([&] {
    validate_build(points, n, k, h, contrast, leaf, eta, eps, opt, out);
    *out = nullptr;
    std::unique_ptr<h2_ctx> H(new h2_ctx());
    if (opt && opt->struct_size >= offsetof(h2_options, alloc_ctx) + sizeof(void*)) {
      H->allocator.alloc = opt->alloc;
      H->allocator.free = opt->free;
      H->allocator.ctx = opt->alloc_ctx;
    }
    AllocScope scope(&H->allocator, (hipStream_t)hip_stream);
    std::vector<char> msg;
    if (!build_structure(points, n, h, leaf, eta, H->S, msg)) fail(H2_ERR_ARG, msg.data());
    check_device();
    hipStream_t st = (hipStream_t)hip_stream;
    H->N = n;
    H->k = k;
    H->h = h;
    H->eta = eta;
    H->eps = eps;
    H->leaf = leaf;
    H->eps_fill = (opt && opt->eps_fill > 0) ? opt->eps_fill : eps;
    H->precision = opt ? opt->precision : H2_FP64;
    const Structure& S = H->S;
    const int L = S.L;
    // forced ranks
    H->lvl_base.assign(L + 2, 0);
    for (int l = 0; l <= L; ++l) H->lvl_base[l + 1] = H->lvl_base[l] + S.nclusters(l);
    if (opt && opt->forced_ranks && opt->forced_ranks_len > 0) {
      H->has_forced = true;
      H->forced_k.assign(H->lvl_base[L + 1], -1);
      H->forced_kt.assign(H->lvl_base[L + 1], -1);
      for (int64_t e = 0; e + 3 < opt->forced_ranks_len; e += 4) {
        const int32_t l = opt->forced_ranks[e], t = opt->forced_ranks[e + 1];
        if (l < 0 || l > L || t < 0 || t >= S.nclusters(l)) fail(H2_ERR_ARG, "forced rank entry out of range");
        H->forced_k[H->lvl_base[l] + t] = opt->forced_ranks[e + 2];
        H->forced_kt[H->lvl_base[l] + t] = opt->forced_ranks[e + 3];
      }
    }
    // geometry in tree order
    std::vector<double> pts(3 * n);
    const double h3 = std::pow(h, 3.0);
    const double k2h3 = k * k * h3;
    for (int64_t t = 0; t < n; ++t) {
      const int64_t i = S.perm[t];
      for (int d = 0; d < 3; ++d) pts[3 * t + d] = points[3 * i + d];
    }
    std::vector<int32_t> leafid(n);
    for (int t = 0; t < S.nclusters(L); ++t)
      for (int64_t e = 0; e < S.size[L][t]; ++e) leafid[S.start[L][t] + e] = t;
    H->d_pts.upload(pts, st);
    upload_contrast(H.get(), contrast, st);
    H->d_leafid.upload(leafid, st);
    H->d_perm.upload(S.perm, st);
    const double a = std::cbrt(3.0 / (4.0 * M_PI)) * h;
    // c = (1 + jka) e^{-jka} - 1
    const double ka = k * a;
    const double cr = std::cos(ka), ci = -std::sin(ka);
    const double self_re = (1.0 * cr - ka * ci) - 1.0;
    const double self_im = (1.0 * ci + ka * cr);
    GeomView& g = H->geom;
    g.pts = H->d_pts.p;
    g.chi = H->d_chi.p;
    g.leafid = H->d_leafid.p;
    g.N = n;
    g.L = L;
    g.k = k;
    g.h = h;
    g.diag_re_c = self_re;
    g.diag_im_c = self_im;
    g.k2h3 = k2h3;
    if (S.l0 >= 0) {
      // plans
      H->plans.clear();
      H->plans.resize(L - S.l0 + 1);
      std::vector<int> levels;
      for (int l = L; l >= S.l0; --l) levels.push_back(l);
      build_plan_levels(H.get(), levels);
      int stop = S.l0;
      if (opt && opt->struct_size >= offsetof(h2_options, stop_level) + sizeof(int32_t) && opt->stop_level != 0) {
        if (opt->stop_level < S.l0 || opt->stop_level > L)
          fail(H2_ERR_ARG, "stop_level " + std::to_string(opt->stop_level) + " outside [l0, L] = [" +
                               std::to_string(S.l0) + ", " + std::to_string(L) + "]");
        stop = opt->stop_level;
      }
      H->stop = stop;
      for (int l = L; l >= S.l0; --l)
        build_merge(H.get(), H->plans[L - l], l > stop ? &H->plans[L - l + 1] : nullptr);
      for (auto& P : H->plans) upload_plan(P, st);
    }
    if (S.l0 >= 0) {
      construct(H.get(), st);
    } else {
      // no admissible block: only the inadmissible leaf blocks (the whole matrix)
      const auto& nl = S.near[L];
      H->near_off.assign(nl.size() + 1, 0);
      for (size_t e = 0; e < nl.size(); ++e)
        H->near_off[e + 1] = H->near_off[e] + S.size[L][nl[e].first] * S.size[L][nl[e].second];
      H->near_orig.alloc(H->near_off[nl.size()]);
      std::vector<int32_t> pr(nl.size()), pc(nl.size()), sz(S.nclusters(L));
      for (size_t e = 0; e < nl.size(); ++e) {
        pr[e] = nl[e].first;
        pc[e] = nl[e].second;
      }
      for (int t = 0; t < S.nclusters(L); ++t) sz[t] = (int32_t)S.size[L][t];
      std::vector<int64_t> cs(S.start[L].begin(), S.start[L].end());
      H->d_near_pr.upload(pr, st);
      H->d_near_pc.upload(pc, st);
      H->d_leaf_size.upload(sz, st);
      H->d_leaf_start.upload(cs, st);
      H->d_near_off.upload(H->near_off, st);
      launch_near_blocks(g, H->d_near_pr.p, H->d_near_pc.p, H->d_near_off.p, H->d_leaf_start.p, H->d_leaf_size.p, H->d_leaf_start.p,
                         H->d_leaf_size.p, (int)nl.size(), H->near_orig.p, st);
      check_launch("host.cpp:1590");
      std::vector<int32_t> nptr(S.nclusters(L) + 1, 0);
      for (const Pair& p : nl) nptr[p.first + 1]++;
      for (int t = 0; t < S.nclusters(L); ++t) nptr[t + 1] += nptr[t];
      H->d_near_ptr.upload(nptr, st);
      H->d_near_col.upload(pc, st);
    }
    H->d_norms.alloc(4096);
    HIPCHK(hipStreamSynchronize(st));
    *out = H.release();
  });
}

extern "C" h2_status h2_set_contrast(h2_handle H, const double* contrast, void* hip_stream) {
  return guarded([&] {
    if (!H) fail(H2_ERR_ARG, "handle is NULL");
    validate_contrast(contrast, H->N);
    hipStream_t st = (hipStream_t)hip_stream;
    AllocScope scope(&H->allocator, st);
    H->factored = false;
    upload_contrast(H, contrast, st);
    H->geom.chi = H->d_chi.p;
    // only the diagonal of Z depends on chi: recompute the inadmissible leaf blocks
    const Structure& S = H->S;
    launch_near_blocks(H->geom, H->d_near_pr.p, H->d_near_pc.p, H->d_near_off.p, H->d_leaf_start.p,
                       H->d_leaf_size.p, H->d_leaf_start.p, H->d_leaf_size.p, (int)S.near[S.L].size(),
                       H->near_orig.p, st);
    check_launch("set_contrast");
    HIPCHK(hipStreamSynchronize(st));
  });
}

extern "C" h2_status h2_set_sweep_graph(h2_handle H, int32_t enable) {
  return guarded([&] {
    if (!H) fail(H2_ERR_ARG, "handle is NULL");
    H->use_graph = enable != 0;
    if (!H->use_graph) H->drop_graphs();
  });
}

extern "C" h2_status h2_set_precision(h2_handle H, int32_t precision) {
  return guarded([&] {
    if (!H) fail(H2_ERR_ARG, "handle is NULL");
    if (precision != H2_FP64 && precision != H2_MIXED) fail(H2_ERR_ARG, "unknown precision");
    if (precision != H->precision) H->factored = false;
    H->precision = precision;
  });
}

static void set_stop(h2_ctx* H, int stop);

extern "C" h2_status h2_set_stop_level(h2_handle H, int32_t level) {
  return guarded([&] {
    if (!H) fail(H2_ERR_ARG, "handle is NULL");
    const Structure& S = H->S;
    if (S.l0 < 0) {
      if (level != 0) fail(H2_ERR_ARG, "no admissible block: the whole matrix is factored densely");
      return;
    }
    const int stop = level == 0 ? S.l0 : level;
    if (stop < S.l0 || stop > S.L)
      fail(H2_ERR_ARG, "stop level " + std::to_string(level) + " outside [l0, L] = [" + std::to_string(S.l0) +
                           ", " + std::to_string(S.L) + "]");
    set_stop(H, stop);
  });
}

// Measured choice of the stop level: factor with the stop at l0, l0 + 1, ... and
// keep the fastest.  A run that stops at ls knows the ranks of every level above
// it, hence the dense block a stop at ls + 1 would leave (the kept unknowns of
// level ls + 1); the search ends before that block would exceed max_final.
static void set_stop(h2_ctx* H, int stop) {
  const Structure& S = H->S;
  if (stop == H->stop) return;
  H->stop = stop;
  H->factored = false;
  // every level above the stop merges into its parent level's blocks, the stop level into
  // the final dense block (levels below it are not factored)
  for (int l = S.l0; l <= S.L; ++l)
    build_merge(H, H->plans[S.L - l], l > stop ? &H->plans[S.L - l + 1] : nullptr);
}

static void factor_checked(h2_ctx* H, hipStream_t st) {
  try {
    factor_impl(H, st);
  } catch (...) {
    H->factored = false;
    throw;
  }
}

// The stop level search (see h2_tune_stop_level); returns the chosen level.
static int tune_stop(h2_ctx* H, int64_t max_final, hipStream_t st, double* ms, int32_t n_ms, double* best_out) {
  const Structure& S = H->S;
  for (int32_t e = 0; ms && e < n_ms; ++e) ms[e] = -1.0;
  int best = S.l0;
  double best_ms = 0;
  for (int ls = S.l0; ls <= S.L; ++ls) {
    if (ls > S.l0) {
      // the dense block a stop at ls leaves: the kept unknowns of level ls (known from the last run)
      const FactorLevel& F = H->flev[S.L - ls];
      int64_t nf = 0;
      for (int t = 0; t < S.nclusters(ls); ++t)
        if (S.size[ls][t]) nf += F.kt[t];
      if (nf > max_final) break;
    }
    set_stop(H, ls);
    factor_checked(H, st);
    const double t = H->timing[0];
    if (ms && ls - S.l0 < n_ms) ms[ls - S.l0] = t;
    if (ls == S.l0 || t < best_ms) {
      best = ls;
      best_ms = t;
    }
  }
  set_stop(H, best);
  if (best_out) *best_out = best_ms;
  return best;
}

extern "C" h2_status h2_tune_stop_level(h2_handle H, int64_t max_final, void* hip_stream, int32_t* chosen,
                                        double* ms, int32_t n_ms) {
  return guarded([&] {
    if (!H || !chosen) fail(H2_ERR_ARG, "NULL argument");
    if (max_final < 1) fail(H2_ERR_ARG, "max_final < 1");
    hipStream_t st = (hipStream_t)hip_stream;
    AllocScope scope(&H->allocator, st);
    if (H->S.l0 < 0) {
      for (int32_t e = 0; ms && e < n_ms; ++e) ms[e] = -1.0;
      factor_impl(H, st);
      *chosen = 0;
      return;
    }
    *chosen = tune_stop(H, max_final, st, ms, n_ms, nullptr);
    if (!H->factored) factor_checked(H, st);
  });
}

extern "C" h2_status h2_set_schur_split(h2_handle H, int32_t level, int64_t below_wgs) {
  return guarded([&] {
    if (!H) fail(H2_ERR_ARG, "handle is NULL");
    const Structure& S = H->S;
    if (level < -1 || level > S.L) fail(H2_ERR_ARG, "level outside [0, L] (or -1 for every level)");
    if (below_wgs < -1) fail(H2_ERR_ARG, "below_wgs < -1");
    H->split_below.resize(S.L + 1, -1);
    if (level < 0)
      std::fill(H->split_below.begin(), H->split_below.end(), below_wgs);
    else
      H->split_below[level] = below_wgs;
    H->factored = false;
  });
}

extern "C" h2_status h2_set_mixed_flush(h2_handle H, int32_t level, int32_t mode) {
  return guarded([&] {
    if (!H) fail(H2_ERR_ARG, "handle is NULL");
    const Structure& S = H->S;
    if (level < -1 || level > S.L) fail(H2_ERR_ARG, "level outside [0, L] (or -1 for every level)");
    if (mode < -1 || mode > 1) fail(H2_ERR_ARG, "mode must be -1, 0 or 1");
    H->mixed_flush.resize(S.L + 1, -1);
    if (level < 0)
      std::fill(H->mixed_flush.begin(), H->mixed_flush.end(), mode);
    else
      H->mixed_flush[level] = mode;
    if (H->precision == H2_MIXED) H->factored = false;
  });
}

// New chunk sizes change the levels' Schur flush lists: rebuild those plans and
// every merge plan (which reads the plans of two levels), and upload them.
static void rebuild_plans(h2_ctx* H, const std::vector<int>& levels, hipStream_t st) {
  const Structure& S = H->S;
  if (S.l0 < 0 || levels.empty()) return;
  build_plan_levels(H, levels);
  for (int l = S.l0; l <= S.L; ++l)
    build_merge(H, H->plans[S.L - l], l > H->stop ? &H->plans[S.L - l + 1] : nullptr);
  for (int l : levels) upload_plan(H->plans[S.L - l], st);
  H->factored = false;
}

static void set_chunks(h2_ctx* H, const std::vector<int32_t>& chunk, hipStream_t st) {
  const Structure& S = H->S;
  std::vector<int32_t> old = H->schur_chunk;
  old.resize(S.L + 1, -1);
  std::vector<int32_t> nw = chunk;
  nw.resize(S.L + 1, -1);
  std::vector<int> changed;
  for (int l = std::max(S.l0, 0); l <= S.L; ++l) {
    const int a = old[l] > 0 ? old[l] : SCHUR_CHUNK_TERMS, b = nw[l] > 0 ? nw[l] : SCHUR_CHUNK_TERMS;
    if (a != b) changed.push_back(l);
  }
  H->schur_chunk = nw;
  rebuild_plans(H, changed, st);
}

extern "C" h2_status h2_set_schur_chunk(h2_handle H, int32_t level, int32_t terms) {
  return guarded([&] {
    if (!H) fail(H2_ERR_ARG, "handle is NULL");
    const Structure& S = H->S;
    if (level < -1 || level > S.L) fail(H2_ERR_ARG, "level outside [0, L] (or -1 for every level)");
    if (terms == 0 || terms < -1) fail(H2_ERR_ARG, "terms must be >= 1 (or -1 for the default)");
    std::vector<int32_t> ch = H->schur_chunk;
    ch.resize(S.L + 1, -1);
    if (level < 0)
      std::fill(ch.begin(), ch.end(), terms);
    else
      ch[level] = terms;
    AllocScope scope(&H->allocator, nullptr);
    set_chunks(H, ch, nullptr);
    HIPCHK(hipStreamSynchronize(nullptr));
  });
}

// Process-wide cache of measured tunings, keyed by everything the factorization's
// work depends on: the cluster tree and block structure (sizes of every cluster,
// eta), the accuracy, the form, forced ranks and the stop-level search bound.
struct TuneRecord {
  int32_t stop;
  std::vector<int64_t> split;
  std::vector<int32_t> mflush;
  std::vector<int32_t> chunk;
  double ms;
};
static std::mutex g_tune_mu;
static std::map<uint64_t, TuneRecord> g_tune_cache;

static uint64_t tuning_key(const h2_ctx* H, int64_t max_final) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) {
      h ^= c[i];
      h *= 1099511628211ull;
    }
  };
  const Structure& S = H->S;
  mix(&H->N, sizeof(H->N));
  mix(&H->k, sizeof(H->k));
  mix(&H->h, sizeof(H->h));
  mix(&H->leaf, sizeof(H->leaf));
  mix(&H->eta, sizeof(H->eta));
  mix(&H->eps, sizeof(H->eps));
  mix(&H->precision, sizeof(H->precision));
  mix(&max_final, sizeof(max_final));
  mix(&S.L, sizeof(S.L));
  mix(&S.l0, sizeof(S.l0));
  for (int l = 0; l <= S.L; ++l)
    if (!S.size[l].empty()) mix(S.size[l].data(), S.size[l].size() * sizeof(S.size[l][0]));
  // the construction ranks, which (with the sizes) set each level's work
  for (const BuildLevel& B : H->build)
    if (!B.k.empty()) mix(B.k.data(), B.k.size() * sizeof(B.k[0]));
  const int32_t hf = H->has_forced ? 1 : 0;
  mix(&hf, sizeof(hf));
  if (H->has_forced) {
    mix(H->forced_k.data(), H->forced_k.size() * sizeof(int32_t));
    mix(H->forced_kt.data(), H->forced_kt.size() * sizeof(int32_t));
  }
  return h;
}

extern "C" h2_status h2_tune(h2_handle H, int64_t max_final, void* hip_stream, h2_tuning* out) {
  return guarded([&] {
    if (!H || !out) fail(H2_ERR_ARG, "NULL argument");
    if (max_final < 1) fail(H2_ERR_ARG, "max_final < 1");
    hipStream_t st = (hipStream_t)hip_stream;
    AllocScope scope(&H->allocator, st);
    const Structure& S = H->S;
    std::memset(out, 0, sizeof(*out));
    for (int l = 0; l < H2_TUNING_MAX_LEVELS; ++l) {
      out->split_below[l] = -1;
      out->mixed_flush[l] = -1;
      out->schur_chunk[l] = -1;
    }
    if (S.L + 1 > H2_TUNING_MAX_LEVELS) fail(H2_ERR_ARG, "tree deeper than H2_TUNING_MAX_LEVELS");
    if (S.l0 < 0) {
      factor_checked(H, st);
      out->factor_ms = H->timing[0];
      return;
    }
    const uint64_t key = tuning_key(H, max_final);
    TuneRecord rec;
    bool cached = false;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      auto it = g_tune_cache.find(key);
      if (it != g_tune_cache.end()) {
        rec = it->second;
        cached = true;
      }
    }
    if (!cached) {
      // 1. the stop level, with the default split, flush and chunk rules
      H->split_below.assign(S.L + 1, -1);
      H->mixed_flush.assign(S.L + 1, -1);
      set_chunks(H, std::vector<int32_t>(S.L + 1, -1), st);
      rec.stop = tune_stop(H, max_final, st, nullptr, 0, nullptr);
      // 2. the split threshold of every factored level: one factorization per candidate
      //    (the same value on every level), each level keeps the candidate under which
      //    its own time (its colours and its merge) was lowest
      const int64_t cand[] = {0, 2048, SCHUR_SPLIT_BELOW, 32768, INT64_MAX};
      const int nlev = S.L - rec.stop + 1;
      std::vector<double> best(nlev, 0.0);
      rec.split.assign(S.L + 1, -1);
      for (int64_t c : cand) {
        std::fill(H->split_below.begin(), H->split_below.end(), c);
        factor_checked(H, st);
        for (int e = 0; e < nlev && e < (int)H->level_ms.size(); ++e) {
          const int l = S.L - e;
          if (rec.split[l] < 0 || H->level_ms[e] < best[e]) {
            rec.split[l] = c;
            best[e] = H->level_ms[e];
          }
        }
      }
      H->split_below = rec.split;
      // 3. mixed form: the flush kernel of every factored level (FP32 routing or plain
      //    FP64), chosen the same way
      rec.mflush.assign(S.L + 1, -1);
      if (H->precision == H2_MIXED) {
        std::vector<double> bm(nlev, 0.0);
        for (int32_t m = 0; m <= 1; ++m) {
          H->mixed_flush.assign(S.L + 1, m);
          factor_checked(H, st);
          for (int e = 0; e < nlev && e < (int)H->level_ms.size(); ++e) {
            const int l = S.L - e;
            if (rec.mflush[l] < 0 || H->level_ms[e] < bm[e]) {
              rec.mflush[l] = m;
              bm[e] = H->level_ms[e];
            }
          }
        }
      }
      H->mixed_flush = rec.mflush;
      // 4. the terms per chunk of split Schur tasks, chosen the same way (each candidate
      //    rebuilds the levels' flush lists)
      {
        const int32_t cand_chunk[] = {5, SCHUR_CHUNK_TERMS, 20};
        std::vector<double> bc(nlev, 0.0);
        rec.chunk.assign(S.L + 1, -1);
        for (int32_t cterms : cand_chunk) {
          set_chunks(H, std::vector<int32_t>(S.L + 1, cterms), st);
          factor_checked(H, st);
          for (int e = 0; e < nlev && e < (int)H->level_ms.size(); ++e) {
            const int l = S.L - e;
            if (rec.chunk[l] < 0 || H->level_ms[e] < bc[e]) {
              rec.chunk[l] = cterms;
              bc[e] = H->level_ms[e];
            }
          }
        }
        set_chunks(H, rec.chunk, st);
      }
      factor_checked(H, st);
      rec.ms = H->timing[0];
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune_cache[key] = rec;
    } else {
      set_stop(H, rec.stop);
      H->split_below = rec.split;
      H->mixed_flush = rec.mflush;
      set_chunks(H, rec.chunk, st);
      H->factored = false;
      factor_checked(H, st);
    }
    out->stop_level = rec.stop;
    out->from_cache = cached ? 1 : 0;
    for (int l = 0; l <= S.L; ++l) {
      out->split_below[l] = rec.split[l];
      out->mixed_flush[l] = rec.mflush[l];
      out->schur_chunk[l] = rec.chunk[l];
    }
    out->factor_ms = cached ? H->timing[0] : rec.ms;
  });
}

extern "C" h2_status h2_tune_cache_clear(void) {
  return guarded([&] {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache.clear();
  });
}

extern "C" h2_status h2_stop_level(h2_handle H, int32_t* level) {
  return guarded([&] {
    if (!H || !level) fail(H2_ERR_ARG, "NULL argument");
    *level = H->S.l0 < 0 ? 0 : H->stop;
  });
}

extern "C" h2_status h2_factor(h2_handle H, void* hip_stream) {
  return guarded([&] {
    if (!H) fail(H2_ERR_ARG, "handle is NULL");
    AllocScope scope(&H->allocator, (hipStream_t)hip_stream);
    try {
      factor_impl(H, (hipStream_t)hip_stream);
    } catch (...) {
      H->factored = false;
      throw;
    }
  });
}

static void validate_vec(h2_handle H, const void* a, const void* b, int32_t nrhs, int64_t ld) {
  if (!H) fail(H2_ERR_ARG, "handle is NULL");
  if (!a || !b) fail(H2_ERR_ARG, "vector pointer is NULL");
  if (nrhs < 1) fail(H2_ERR_ARG, "nrhs < 1");
  if (ld < H->N) fail(H2_ERR_ARG, "ld < n");
}

// x = M^-1 b (adj = 0) or x = M^-H b (adj = 1), M = L U D, optionally refined
// against A_H2 (adj = 0) or A_H2^H (adj = 1) until the column-max relative
// residual is <= tol.  b and x may alias.
static void solve_refined(h2_ctx* H, int adj, const void* b, void* x, int32_t nrhs, int64_t ld, double tol,
                          int32_t max_iter, hipStream_t st, h2_solve_info* info) {
  validate_vec(H, b, x, nrhs, ld);
  if (!(tol >= 0) || !std::isfinite(tol)) fail(H2_ERR_ARG, "tol must be finite and >= 0");
  if (tol > 0 && max_iter < 1) fail(H2_ERR_ARG, "max_iter < 1 with tol > 0");
  if (!H->factored) fail(H2_ERR_STATE, "solve before a successful h2_factor");
  const int64_t N = H->N;
  ensure_vbuf(H, nrhs);
  const double2* bb = (const double2*)b;
  double2* xx = (double2*)x;
  auto solve_once = [&](const double2* rhs, int64_t ldr, double2* outx, int64_t ldo, int accumulate) {
    if (!adj) {
      // M^-1 = D^-1 Z^-1
      launch_permute_in(rhs, ldr, H->d_perm.p, nullptr, 0, N, nrhs, H->vtmp3.p, N, st);
      sweep_vtmp3(H, nrhs, 0, st);
      launch_permute_out(H->vtmp3.p, N, H->d_perm.p, H->d_scale_solve.p, 0, N, nrhs, outx, ldo, accumulate, st);
    } else {
      // M^-H = Z^-H D^-1
      launch_permute_in(rhs, ldr, H->d_perm.p, H->d_scale_solve.p, 0, N, nrhs, H->vtmp3.p, N, st);
      sweep_vtmp3(H, nrhs, 1, st);
      launch_permute_out(H->vtmp3.p, N, H->d_perm.p, nullptr, 0, N, nrhs, outx, ldo, accumulate, st);
    }
    check_launch("solve");
  };
  if (info) {
    info->iterations = 0;
    info->rel_residual = -1.0;
    info->rel_residual_first = -1.0;
  }
  if (tol <= 0) {
    // b is read into the sweep's own buffer before x is written, so they may alias;
    // no host synchronisation and no allocation beyond first use
    solve_once(bb, ld, xx, ld, 0);
    return;
  }
  // copy of b (b and x may alias), kept for the residuals; work vectors live in the handle
  DArr<double2>& b0 = H->rf_b0;
  b0.alloc(N * nrhs);
  HIPCHK(hipMemcpy2DAsync(b0.p, N * sizeof(double2), bb, ld * sizeof(double2), N * sizeof(double2), nrhs,
                          hipMemcpyDeviceToDevice, st));
  solve_once(b0.p, N, xx, ld, 0);
  // iterative refinement against A_H2 = Z_H2 D (or its conjugate transpose D conj(Z_H2))
  DArr<double2>& r = H->rf_r;
  DArr<double2>& ax = H->rf_ax;
  DArr<double2>& vt = H->rf_vt;
  r.alloc(N * nrhs);
  ax.alloc(N * nrhs);
  vt.alloc(N * nrhs);
  std::vector<double> nb(nrhs), nr(nrhs);
  DArr<double>& d_nb = H->rf_nb;
  d_nb.alloc(nrhs);
  launch_col_norms(b0.p, N, N, nrhs, d_nb.p, st);
  HIPCHK(hipMemcpyAsync(nb.data(), d_nb.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  int it = 0;
  double rel = 0, first = -1;
  for (;;) {
    if (!adj) {
      launch_permute_in(xx, ld, H->d_perm.p, H->d_scale_mat.p, 0, N, nrhs, vt.p, N, st);
      matvec_tree(H, vt.p, H->vtmp3.p, nrhs, st);
      launch_permute_out(H->vtmp3.p, N, H->d_perm.p, nullptr, 0, N, nrhs, ax.p, N, 0, st);
    } else {
      launch_permute_in(xx, ld, H->d_perm.p, nullptr, 1, N, nrhs, vt.p, N, st);
      matvec_tree(H, vt.p, H->vtmp3.p, nrhs, st);
      launch_permute_out(H->vtmp3.p, N, H->d_perm.p, H->d_scale_mat.p, 1, N, nrhs, ax.p, N, 0, st);
    }
    launch_residual(b0.p, N, ax.p, N, r.p, N, N, nrhs, st);
    launch_col_norms(r.p, N, N, nrhs, d_nb.p, st);
    check_launch("refinement residual");
    HIPCHK(hipMemcpyAsync(nr.data(), d_nb.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    rel = 0;
    bool finite = true;
    for (int c = 0; c < nrhs; ++c) {
      const double rc = nb[c] > 0 ? nr[c] / nb[c] : nr[c];
      if (!std::isfinite(rc)) finite = false;
      rel = std::max(rel, rc);
    }
    if (!finite) rel = std::numeric_limits<double>::infinity();
    if (first < 0) first = rel;
    if (!finite) {
      if (info) {
        info->iterations = it;
        info->rel_residual = rel;
        info->rel_residual_first = first;
      }
      fail(H2_ERR_NOCONV, "refinement residual is not finite after " + std::to_string(it) + " iterations");
    }
    if (rel <= tol || it >= max_iter) break;
    solve_once(r.p, N, xx, ld, 1);
    ++it;
  }
  if (info) {
    info->iterations = it;
    info->rel_residual = rel;
    info->rel_residual_first = first;
  }
  if (rel > tol) {
    char msg[160];
    snprintf(msg, sizeof msg, "refinement did not reach tol within max_iter (relative residual %.3e after %d iterations, %.3e before)", rel, it, first);
    fail(H2_ERR_NOCONV, msg);
  }
}

// Run fn(k, stream_k) for every handle k concurrently: handle k works on its own
// stream from its own host thread (at most `workers` threads pull handles from a
// shared counter), after everything queued on the caller's stream, which in turn
// waits for all of them.  The first failure is reported.
static void check_batch(h2_handle* hs, int32_t count) {
  if (!hs || count < 1) fail(H2_ERR_ARG, "empty batch");
  for (int32_t k = 0; k < count; ++k) {
    if (!hs[k]) fail(H2_ERR_ARG, "handle is NULL");
    for (int32_t q = 0; q < k; ++q)
      if (hs[q] == hs[k]) fail(H2_ERR_ARG, "a handle appears twice in the batch");
  }
}

// Several problems factored in lockstep, level by level from each problem's finest
// level: every stage of colour index c (Schur flush, Step 0, projections, partial
// LU, panels) is one launch for all problems that have that colour, its work items
// listed per problem (entries sorted by their first workgroup).  Problems whose
// sizes select different kernel variants (Step 0 register tiles, register or LDS
// LU, fused one-tile projections, FP64 or mixed form) share a launch with those of
// the same variant.  Each problem's work items and kernels are the ones its own
// factorization launches, so the factors are bit-identical to one-by-one runs.
// ids: the problems' indices in the caller's batch (for messages); *bad_id: the
// index of the first failed problem, INT32_MAX when none failed in the problems'
// own steps.
static void factor_fused(h2_handle* hs, int32_t count, hipStream_t st, const int32_t* ids, int32_t* bad_id) {
  *bad_id = INT32_MAX;
  std::vector<std::unique_ptr<FactorRun>> runs(count);
  std::vector<char> failed(count, 0);
  h2_status first = H2_OK;
  std::string first_msg;
  auto step = [&](int32_t k, auto&& fn) {
    if (failed[k]) return;
    AllocScope scope(&hs[k]->allocator, st);
    const h2_status s = guarded(fn);
    if (s != H2_OK) {
      failed[k] = 1;
      hs[k]->factored = false;
      if (first == H2_OK) {
        first = s;
        first_msg = "batch item " + std::to_string(ids[k]) + ": " + g_err;
        *bad_id = ids[k];
      }
    }
  };
  for (int32_t k = 0; k < count; ++k) step(k, [&] { runs[k].reset(new FactorRun(hs[k], st)); });
  struct Group {
    int kernel;
    size_t off;
    int ne;
    int64_t blocks;
  };
  std::vector<std::pair<int, BatchEntry>> pairs;
  std::vector<BatchEntry> ent;
  std::vector<Group> groups;
  std::vector<int32_t> act;
  for (;;) {
    act.clear();
    for (int32_t k = 0; k < count; ++k)
      if (!failed[k] && runs[k]->level_pending()) act.push_back(k);
    if (act.empty()) break;
    for (int32_t k : act) step(k, [&] { runs[k]->level_begin(); });
    act.erase(std::remove_if(act.begin(), act.end(), [&](int32_t k) { return failed[k] != 0; }), act.end());
    int maxcol = 0;
    for (int32_t k : act) maxcol = std::max(maxcol, runs[k]->plan().ncol);
    ent.clear();
    groups.clear();
    // c < 0: the updates still pending at the end of each problem's level
    auto add_stage = [&](int stage, int c) {
      pairs.clear();
      for (int32_t k : act) {
        FactorRun& R = *runs[k];
        const int nc = R.plan().ncol;
        if (c < 0)
          R.stage_entries(stage, nc, pairs);
        else if (c < nc)
          R.stage_entries(stage, c, pairs);
      }
      std::stable_sort(pairs.begin(), pairs.end(),
                       [](const std::pair<int, BatchEntry>& a, const std::pair<int, BatchEntry>& b) {
                         return a.first < b.first;
                       });
      for (size_t i = 0; i < pairs.size();) {
        Group g{pairs[i].first, ent.size(), 0, 0};
        for (; i < pairs.size() && pairs[i].first == g.kernel; ++i) {
          BatchEntry e = pairs[i].second;
          e.first = (int32_t)g.blocks;
          g.blocks += (int64_t)e.gx * e.gy * e.gz;
          if (g.blocks > INT32_MAX) fail(H2_ERR_INTERNAL, "shared launch beyond 2^31 workgroups");
          ent.push_back(e);
          ++g.ne;
        }
        groups.push_back(g);
      }
    };
    for (int c = 0; c < maxcol; ++c)
      for (int s = 0; s < BS_COUNT; ++s) add_stage(s, c);
    add_stage(BS_SCHUR, -1);
    add_stage(BS_SCHUR_REDUCE, -1);
    {
      AllocScope scope(&hs[0]->allocator, st);
      hs[0]->batch_entries.upload(ent, st);
    }
    const BatchEntry* d_ent = hs[0]->batch_entries.p;
    for (const Group& g : groups) launch_batched(g.kernel, d_ent + g.off, g.ne, (int)g.blocks, st);
    check_launch("batched colour stages");
    for (int32_t k : act) step(k, [&] { runs[k]->readback(); });
    HIPCHK(hipStreamSynchronize(st));
    for (int32_t k : act) step(k, [&] { runs[k]->level_merge(); });
    HIPCHK(hipStreamSynchronize(st));
    for (int32_t k : act) step(k, [&] { runs[k]->level_close(); });
  }
  for (int32_t k = 0; k < count; ++k)
    if (!failed[k] && !runs[k]->done) step(k, [&] { runs[k]->finish(); });
  if (first != H2_OK) fail(first, first_msg);
}

template <typename Fn>
static void run_batch(h2_handle* hs, int32_t count, hipStream_t st, Fn&& fn) {
  check_batch(hs, count);
  hipEvent_t start;
  HIPCHK(hipEventCreateWithFlags(&start, hipEventDisableTiming));
  HIPCHK(hipEventRecord(start, st));
  for (int32_t k = 0; k < count; ++k) {
    if (!hs[k]->own_stream) HIPCHK(hipStreamCreateWithFlags(&hs[k]->own_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamWaitEvent(hs[k]->own_stream, start, 0));
  }
  std::atomic<int32_t> next{0};
  std::mutex mu;
  h2_status first = H2_OK;
  int32_t first_k = INT32_MAX;  // the lowest failing batch index is reported
  std::string first_msg;
  const int workers = std::max(1, std::min<int>(count, 8));
  auto work = [&]() {
    for (;;) {
      const int32_t k = next.fetch_add(1);
      if (k >= count) return;
      const h2_status stt = guarded([&] {
        AllocScope scope(&hs[k]->allocator, hs[k]->own_stream);
        fn(k, hs[k]->own_stream);
      });
      if (stt != H2_OK) {
        std::lock_guard<std::mutex> lk(mu);
        if (k < first_k) {
          first = stt;
          first_k = k;
          first_msg = "batch item " + std::to_string(k) + ": " + g_err;
        }
      }
    }
  };
  std::vector<std::thread> pool;
  for (int w = 1; w < workers; ++w) {
    try {
      pool.emplace_back(work);
    } catch (const std::system_error&) {
      break;  // fewer workers: the items are shared through `next`
    }
  }
  work();
  for (auto& t : pool) t.join();
  for (int32_t k = 0; k < count; ++k) {
    hipEvent_t done;
    HIPCHK(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    HIPCHK(hipEventRecord(done, hs[k]->own_stream));
    HIPCHK(hipStreamWaitEvent(st, done, 0));
    (void)hipEventDestroy(done);
  }
  (void)hipEventDestroy(start);
  if (first != H2_OK) fail(first, first_msg);
}

// The fused schedule over up to FUSED_GROUPS groups of problems, each group on a
// stream of its own driven by its own host thread: the latency-bound stages of one
// group (Step 0's eigen-solver, the partial LU, the final dense LU) and its host
// work between levels overlap with another group's launches.  Problems are dealt
// to the groups by size (largest first, in alternating order) so that the groups
// carry similar work.  Two groups measured best for fresh handles (16 boxes:
// 329 ms against 351, 354 and 367 ms with three, four and eight groups, 421 ms
// with one).
constexpr int FUSED_GROUPS = 2;

static void factor_fused_groups(h2_handle* hs, int32_t count, hipStream_t st) {
  const int ng = std::min<int>(FUSED_GROUPS, (count + 1) / 2);
  if (ng <= 1) {
    std::vector<int32_t> ids(count);
    for (int32_t k = 0; k < count; ++k) ids[k] = k;
    int32_t bad_id = 0;
    factor_fused(hs, count, st, ids.data(), &bad_id);
    return;
  }
  std::vector<int32_t> order(count);
  for (int32_t k = 0; k < count; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return hs[a]->N > hs[b]->N; });
  std::vector<std::vector<h2_handle>> grp(ng);
  std::vector<std::vector<int32_t>> gid(ng);
  for (int32_t i = 0; i < count; ++i) {
    const int r = i % ng, g = ((i / ng) & 1) ? ng - 1 - r : r;
    grp[g].push_back(hs[order[i]]);
    gid[g].push_back(order[i]);
  }
  hipEvent_t start;
  HIPCHK(hipEventCreateWithFlags(&start, hipEventDisableTiming));
  HIPCHK(hipEventRecord(start, st));
  std::vector<hipStream_t> gs(ng);
  for (int g = 0; g < ng; ++g) {
    h2_handle lead = grp[g][0];
    if (!lead->own_stream) HIPCHK(hipStreamCreateWithFlags(&lead->own_stream, hipStreamNonBlocking));
    gs[g] = lead->own_stream;
    HIPCHK(hipStreamWaitEvent(gs[g], start, 0));
  }
  std::vector<h2_status> stt(ng, H2_OK);
  std::vector<std::string> msg(ng);
  std::vector<int32_t> bad_id(ng, INT32_MAX);
  auto work = [&](int g) {
    stt[g] = guarded([&] { factor_fused(grp[g].data(), (int32_t)grp[g].size(), gs[g], gid[g].data(), &bad_id[g]); });
    if (stt[g] != H2_OK) msg[g] = g_err;
  };
  std::vector<std::thread> pool;
  for (int g = 1; g < ng; ++g) {
    try {
      pool.emplace_back(work, g);
    } catch (const std::system_error&) {
      work(g);  // no thread: this group runs on the calling thread
    }
  }
  work(0);
  for (auto& t : pool) t.join();
  for (int g = 0; g < ng; ++g) {
    hipEvent_t done;
    HIPCHK(hipEventCreateWithFlags(&done, hipEventDisableTiming));
    HIPCHK(hipEventRecord(done, gs[g]));
    HIPCHK(hipStreamWaitEvent(st, done, 0));
    (void)hipEventDestroy(done);
  }
  (void)hipEventDestroy(start);
  // report the failure of the lowest batch index
  int bad = -1;
  for (int g = 0; g < ng; ++g)
    if (stt[g] != H2_OK && (bad < 0 || bad_id[g] < bad_id[bad])) bad = g;
  if (bad >= 0) fail(stt[bad], msg[bad]);
}

// Sweeps of several factored problems in lockstep, each in place on its own
// vtmp3 (M^-1 or M^-H on Z, eq. 35): level step j is each problem's j-th finest
// level; every stage of colour c (forward: local products, then the gather into
// the partners; backward: the partial sums, then the local products) is one
// launch over all problems that have that colour, the merges between levels and
// the final block per problem in between.  Each problem's kernels and work
// items are those of its own sweep, so the results equal one-by-one sweeps bit
// for bit.  The work item table lives in `lead` (kept for later sweeps).
static void sweep_fused(h2_handle* hs, const std::vector<int32_t>& act, int nrhs, int adj, hipStream_t st,
                        h2_handle lead) {
  const int64_t nact = (int64_t)act.size();
  std::vector<SweepBufs> W(nact);
  std::vector<int32_t> fused;
  int maxlev = 0;
  for (int64_t a = 0; a < nact; ++a) {
    h2_ctx* H = hs[act[a]];
    AllocScope scope(&H->allocator, st);
    W[a] = handle_bufs(H, nrhs);
    if (H->flev.empty()) {
      sweep(H, W[a], H->vtmp3.p, H->vtmp3.p, nrhs, adj, st);  // the whole matrix is one dense block
      continue;
    }
    fused.push_back((int32_t)a);
    maxlev = std::max(maxlev, (int)H->flev.size());
    HIPCHK(hipMemcpyAsync(W[a].vbuf[0], H->vtmp3.p, H->N * nrhs * sizeof(double2), hipMemcpyDeviceToDevice, st));
  }
  if (fused.empty()) return;
  // ops in stream order: a shared launch (kind 0) or a per-problem merge (1: up,
  // 2: down) or final block (3)
  struct Op {
    int kind, kernel;
    size_t off;
    int ne;
    int64_t blocks;
    int32_t a, j;
  };
  std::vector<Op> ops;
  std::vector<SweepEntry> ent;
  std::vector<std::pair<int, SweepEntry>> pairs;
  auto add_stage = [&](int stage, int j, int c) {
    pairs.clear();
    for (int32_t a : fused) {
      h2_ctx* H = hs[act[a]];
      if (j >= (int)H->flev.size()) continue;
      FactorLevel& F = H->flev[j];
      LevelPlan& P = H->plans[j];
      if (c >= P.ncol) continue;
      const ColourTasks ct = colour_tasks(P.cols[c], c, F.tiles);
      sweep_stage_entries(stage, F.view, ct, W[a].vbuf[j], F.d_voff.p, F.ntot, nrhs, adj, W[a].part, BWD_SPLIT,
                          W[a].scratch, pairs);
    }
    std::stable_sort(pairs.begin(), pairs.end(),
                     [](const std::pair<int, SweepEntry>& x, const std::pair<int, SweepEntry>& y) {
                       return x.first < y.first;
                     });
    for (size_t i = 0; i < pairs.size();) {
      Op o{0, pairs[i].first, ent.size(), 0, 0, -1, j};
      for (; i < pairs.size() && pairs[i].first == o.kernel; ++i) {
        SweepEntry e = pairs[i].second;
        e.first = (int32_t)o.blocks;
        o.blocks += (int64_t)e.gx * e.gy * e.gz;
        if (o.blocks > INT32_MAX) fail(H2_ERR_INTERNAL, "shared sweep launch beyond 2^31 workgroups");
        ent.push_back(e);
        ++o.ne;
      }
      ops.push_back(o);
    }
  };
  auto maxcol = [&](int j) {
    int m = 0;
    for (int32_t a : fused) {
      h2_ctx* H = hs[act[a]];
      if (j < (int)H->flev.size()) m = std::max(m, H->plans[j].ncol);
    }
    return m;
  };
  for (int j = 0; j < maxlev; ++j) {
    const int mc = maxcol(j);
    for (int c = 0; c < mc; ++c) {
      add_stage(SS_FWD_LOCAL, j, c);
      add_stage(SS_FWD_GATHER, j, c);
    }
    for (int32_t a : fused) {
      const int nlev = (int)hs[act[a]]->flev.size();
      if (j < nlev) ops.push_back({j + 1 < nlev ? 1 : 3, 0, 0, 0, 0, a, j});
    }
  }
  for (int j = maxlev - 1; j >= 0; --j) {
    for (int32_t a : fused) {
      const int nlev = (int)hs[act[a]]->flev.size();
      if (j + 1 < nlev) ops.push_back({2, 0, 0, 0, 0, a, j});
    }
    for (int c = maxcol(j) - 1; c >= 0; --c) {
      add_stage(SS_BWD_PARTIAL, j, c);
      add_stage(SS_BWD_LOCAL, j, c);
    }
  }
  {
    AllocScope scope(&lead->allocator, st);
    lead->sweep_entries.upload(ent, st);
  }
  const SweepEntry* d_ent = lead->sweep_entries.p;
  for (const Op& o : ops) {
    if (o.kind == 0) {
      launch_sweep_batched(o.kernel, d_ent + o.off, o.ne, (int)o.blocks, st);
      continue;
    }
    h2_ctx* H = hs[act[o.a]];
    const SweepBufs& B = W[o.a];
    FactorLevel& F = H->flev[o.j];
    LevelPlan& P = H->plans[o.j];
    const int npar = H->S.nclusters(P.l - 1);
    if (o.kind == 1 || o.kind == 2) {
      FactorLevel& Fp = H->flev[o.j + 1];
      launch_vmerge(npar, F.d_kt.p, F.d_voff.p, Fp.d_voff.p, F.ntot, Fp.ntot, nrhs, B.vbuf[o.j], B.vbuf[o.j + 1],
                    o.kind == 1 ? 1 : 0, P.d_nonempty.p, st);
    } else {
      launch_vmerge(npar, F.d_kt.p, F.d_voff.p, H->d_final_off.p, F.ntot, H->nf, nrhs, B.vbuf[o.j], B.vtmp, 1,
                    P.d_nonempty.p, st);
      dense_lu_apply(H, B.vtmp, B.vtmp2, nrhs, adj, st);
      launch_vmerge(npar, F.d_kt.p, F.d_voff.p, H->d_final_off.p, F.ntot, H->nf, nrhs, B.vbuf[o.j], B.vtmp2, 0,
                    P.d_nonempty.p, st);
    }
  }
  check_launch("batched sweeps");
  for (int32_t a : fused) {
    h2_ctx* H = hs[act[a]];
    HIPCHK(hipMemcpyAsync(H->vtmp3.p, W[a].vbuf[0], H->N * nrhs * sizeof(double2), hipMemcpyDeviceToDevice, st));
  }
}

// h2_solve for every handle of a batch in lockstep on one stream (the refinement
// of eq. 35's solution against A_H2 as in solve_refined; the sweeps of all
// problems that still refine are fused).  A problem that fails (non-finite
// residual, tolerance not reached) is reported and the others go on.
static void solve_fused(h2_handle* hs, int32_t count, int adj, const void* const* b, void* const* x, int32_t nrhs,
                        const int64_t* ld, double tol, int32_t max_iter, hipStream_t st, h2_solve_info* infos) {
  check_batch(hs, count);
  if (!(tol >= 0) || !std::isfinite(tol)) fail(H2_ERR_ARG, "tol must be finite and >= 0");
  if (tol > 0 && max_iter < 1) fail(H2_ERR_ARG, "max_iter < 1 with tol > 0");
  for (int32_t k = 0; k < count; ++k) {
    validate_vec(hs[k], b[k], x[k], nrhs, ld[k]);
    if (!hs[k]->factored) fail(H2_ERR_STATE, "batch item " + std::to_string(k) + ": solve before a successful h2_factor");
  }
  h2_handle lead = hs[0];
  auto perm_in = [&](h2_ctx* H, const double2* rhs, int64_t ldr) {
    if (!adj)
      launch_permute_in(rhs, ldr, H->d_perm.p, nullptr, 0, H->N, nrhs, H->vtmp3.p, H->N, st);
    else
      launch_permute_in(rhs, ldr, H->d_perm.p, H->d_scale_solve.p, 0, H->N, nrhs, H->vtmp3.p, H->N, st);
  };
  auto perm_out = [&](h2_ctx* H, double2* outx, int64_t ldo, int accumulate) {
    if (!adj)
      launch_permute_out(H->vtmp3.p, H->N, H->d_perm.p, H->d_scale_solve.p, 0, H->N, nrhs, outx, ldo, accumulate, st);
    else
      launch_permute_out(H->vtmp3.p, H->N, H->d_perm.p, nullptr, 0, H->N, nrhs, outx, ldo, accumulate, st);
  };
  std::vector<int32_t> act(count);
  for (int32_t k = 0; k < count; ++k) {
    act[k] = k;
    AllocScope scope(&hs[k]->allocator, st);
    ensure_vbuf(hs[k], nrhs);
    if (infos) {
      infos[k].iterations = 0;
      infos[k].rel_residual = -1.0;
      infos[k].rel_residual_first = -1.0;
    }
  }
  if (tol <= 0) {
    for (int32_t k = 0; k < count; ++k) perm_in(hs[k], (const double2*)b[k], ld[k]);
    sweep_fused(hs, act, nrhs, adj, st, lead);
    for (int32_t k = 0; k < count; ++k) perm_out(hs[k], (double2*)x[k], ld[k], 0);
    check_launch("batched solve");
    return;
  }
  std::vector<std::vector<double>> nb(count, std::vector<double>(nrhs)), nr(count, std::vector<double>(nrhs));
  std::vector<int> it(count, 0);
  std::vector<double> first(count, -1.0), rel(count, 0.0);
  for (int32_t k = 0; k < count; ++k) {
    h2_ctx* H = hs[k];
    AllocScope scope(&H->allocator, st);
    const int64_t N = H->N;
    H->rf_b0.alloc(N * nrhs);
    HIPCHK(hipMemcpy2DAsync(H->rf_b0.p, N * sizeof(double2), b[k], ld[k] * sizeof(double2), N * sizeof(double2), nrhs,
                            hipMemcpyDeviceToDevice, st));
    H->rf_r.alloc(N * nrhs);
    H->rf_ax.alloc(N * nrhs);
    H->rf_vt.alloc(N * nrhs);
    H->rf_nb.alloc(nrhs);
    perm_in(H, H->rf_b0.p, N);
  }
  sweep_fused(hs, act, nrhs, adj, st, lead);
  for (int32_t k = 0; k < count; ++k) {
    h2_ctx* H = hs[k];
    perm_out(H, (double2*)x[k], ld[k], 0);
    launch_col_norms(H->rf_b0.p, H->N, H->N, nrhs, H->rf_nb.p, st);
    HIPCHK(hipMemcpyAsync(nb[k].data(), H->rf_nb.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  h2_status first_err = H2_OK;
  std::string first_msg;
  // the residuals run side by side, each problem's on a stream of its own after
  // everything queued on st; st waits for all of them
  for (int32_t k = 0; k < count; ++k)
    if (!hs[k]->own_stream) HIPCHK(hipStreamCreateWithFlags(&hs[k]->own_stream, hipStreamNonBlocking));
  EventPool rev;
  while (!act.empty()) {
    hipEvent_t ready = rev.next(st);
    for (int32_t k : act) {
      h2_ctx* H = hs[k];
      const int64_t N = H->N;
      double2* xx = (double2*)x[k];
      const hipStream_t st = H->own_stream;  // this problem's residual
      AllocScope scope(&H->allocator, st);
      HIPCHK(hipStreamWaitEvent(st, ready, 0));
      if (!adj) {
        launch_permute_in(xx, ld[k], H->d_perm.p, H->d_scale_mat.p, 0, N, nrhs, H->rf_vt.p, N, st);
        matvec_tree(H, H->rf_vt.p, H->vtmp3.p, nrhs, st);
        launch_permute_out(H->vtmp3.p, N, H->d_perm.p, nullptr, 0, N, nrhs, H->rf_ax.p, N, 0, st);
      } else {
        launch_permute_in(xx, ld[k], H->d_perm.p, nullptr, 1, N, nrhs, H->rf_vt.p, N, st);
        matvec_tree(H, H->rf_vt.p, H->vtmp3.p, nrhs, st);
        launch_permute_out(H->vtmp3.p, N, H->d_perm.p, H->d_scale_mat.p, 1, N, nrhs, H->rf_ax.p, N, 0, st);
      }
      launch_residual(H->rf_b0.p, N, H->rf_ax.p, N, H->rf_r.p, N, N, nrhs, st);
      launch_col_norms(H->rf_r.p, N, N, nrhs, H->rf_nb.p, st);
    }
    check_launch("batched refinement residuals");
    for (int32_t k : act) HIPCHK(hipStreamWaitEvent(st, rev.next(hs[k]->own_stream), 0));
    // the norms come back on st once every residual is done (one host wait)
    for (int32_t k : act)
      HIPCHK(hipMemcpyAsync(nr[k].data(), hs[k]->rf_nb.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<int32_t> next;
    for (int32_t k : act) {
      double r = 0;
      bool finite = true;
      for (int c = 0; c < nrhs; ++c) {
        const double rc = nb[k][c] > 0 ? nr[k][c] / nb[k][c] : nr[k][c];
        if (!std::isfinite(rc)) finite = false;
        r = std::max(r, rc);
      }
      if (!finite) r = std::numeric_limits<double>::infinity();
      rel[k] = r;
      if (first[k] < 0) first[k] = r;
      std::string msg;
      if (!finite) {
        msg = "refinement residual is not finite after " + std::to_string(it[k]) + " iterations";
      } else if (r > tol && it[k] >= max_iter) {
        char buf[160];
        snprintf(buf, sizeof buf,
                 "refinement did not reach tol within max_iter (relative residual %.3e after %d iterations, %.3e before)",
                 r, it[k], first[k]);
        msg = buf;
      }
      if (!msg.empty() && first_err == H2_OK) {
        first_err = H2_ERR_NOCONV;
        first_msg = "batch item " + std::to_string(k) + ": " + msg;
      }
      if (msg.empty() && r > tol) next.push_back(k);
    }
    act.swap(next);
    if (act.empty()) break;
    for (int32_t k : act) perm_in(hs[k], hs[k]->rf_r.p, hs[k]->N);
    sweep_fused(hs, act, nrhs, adj, st, lead);
    for (int32_t k : act) {
      perm_out(hs[k], (double2*)x[k], ld[k], 1);
      ++it[k];
    }
  }
  if (infos)
    for (int32_t k = 0; k < count; ++k) {
      infos[k].iterations = it[k];
      infos[k].rel_residual = rel[k];
      infos[k].rel_residual_first = first[k];
    }
  if (first_err != H2_OK) fail(first_err, first_msg);
}

extern "C" h2_status h2_solve(h2_handle H, const void* b, void* x, int32_t nrhs, int64_t ld, double tol,
                              int32_t max_iter, void* hip_stream, h2_solve_info* info) {
  return guarded([&] {
    AllocScope scope(H ? &H->allocator : nullptr, (hipStream_t)hip_stream);
    solve_refined(H, 0, b, x, nrhs, ld, tol, max_iter, (hipStream_t)hip_stream, info);
  });
}

extern "C" h2_status h2_solve_adjoint(h2_handle H, const void* g, void* lam, int32_t nrhs, int64_t ld, double tol,
                                      int32_t max_iter, void* hip_stream, h2_solve_info* info) {
  return guarded([&] {
    AllocScope scope(H ? &H->allocator : nullptr, (hipStream_t)hip_stream);
    solve_refined(H, 1, g, lam, nrhs, ld, tol, max_iter, (hipStream_t)hip_stream, info);
  });
}

extern "C" h2_status h2_solve_noalloc(h2_handle H, const void* b, void* x, int32_t nrhs, int64_t ld,
                                     void* hip_stream) {
  return guarded([&] {
    validate_vec(H, b, x, nrhs, ld);
    if (!H->factored) fail(H2_ERR_STATE, "solve before a successful h2_factor");
    hipStream_t st = (hipStream_t)hip_stream;
    const int64_t N = H->N;
    // the sweep's work buffers, each 256-byte aligned, carved from the fixed scratch
    const SweepLayout L = sweep_layout(H, nrhs);
    auto up = [](int64_t e) { return (e + 15) & ~int64_t(15); };
    int64_t need = up(L.vtmp) * 2 + up(L.vtmp3) + up(L.scratch) + up(L.part);
    for (int64_t v : L.vbuf) need += up(v);
    if (need > NOALLOC_SCRATCH_ELEMS)
      fail(H2_ERR_ARG, "h2_solve_noalloc: " + std::to_string(nrhs) + " right-hand sides of this problem need " +
                           std::to_string((need * 16) >> 20) + " MiB of work space, beyond its fixed " +
                           std::to_string((NOALLOC_SCRATCH_ELEMS * 16) >> 20) + " MiB");
    hipError_t e = hipSuccess;
    double2* base = noalloc_scratch(&e);
    if (!base) fail(H2_ERR_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    SweepBufs W;
    int64_t off = 0;
    auto take = [&](int64_t elems) {
      double2* p = base + off;
      off += up(elems);
      return p;
    };
    for (int64_t v : L.vbuf) W.vbuf.push_back(take(v));
    W.vtmp = take(L.vtmp);
    W.vtmp2 = take(L.vtmp);
    W.vtmp3 = take(L.vtmp3);
    W.scratch = take(L.scratch);
    W.part = take(L.part);
    // x = D^-1 Z^-1 b: b into tree order, the sweeps in place, scaled back to the caller's order
    launch_permute_in((const double2*)b, ld, H->d_perm.p, nullptr, 0, N, nrhs, W.vtmp3, N, st);
    sweep(H, W, W.vtmp3, W.vtmp3, nrhs, 0, st);
    launch_permute_out(W.vtmp3, N, H->d_perm.p, H->d_scale_solve.p, 0, N, nrhs, (double2*)x, ld, 0, st);
    check_launch("solve_noalloc");
  });
}

extern "C" h2_status h2_factor_batch_mode(h2_handle* hs, int32_t count, void* hip_stream, int32_t mode) {
  return guarded([&] {
    if (mode != H2_BATCH_FUSED && mode != H2_BATCH_STREAMS) fail(H2_ERR_ARG, "unknown batch mode");
    if (mode == H2_BATCH_FUSED) {
      check_batch(hs, count);
      factor_fused_groups(hs, count, (hipStream_t)hip_stream);
      return;
    }
    run_batch(hs, count, (hipStream_t)hip_stream, [&](int32_t k, hipStream_t s) {
      try {
        factor_impl(hs[k], s);
      } catch (...) {
        hs[k]->factored = false;
        throw;
      }
    });
  });
}

extern "C" h2_status h2_factor_batch(h2_handle* hs, int32_t count, void* hip_stream) {
  return h2_factor_batch_mode(hs, count, hip_stream, H2_BATCH_FUSED);
}

extern "C" h2_status h2_solve_batch_mode(h2_handle* hs, int32_t count, const void* const* b, void* const* x,
                                         int32_t nrhs, const int64_t* ld, double tol, int32_t max_iter,
                                         void* hip_stream, h2_solve_info* infos, int32_t mode) {
  return guarded([&] {
    if (!b || !x || !ld) fail(H2_ERR_ARG, "null pointer");
    if (mode != H2_BATCH_FUSED && mode != H2_BATCH_STREAMS) fail(H2_ERR_ARG, "unknown batch mode");
    if (mode == H2_BATCH_FUSED) {
      solve_fused(hs, count, 0, b, x, nrhs, ld, tol, max_iter, (hipStream_t)hip_stream, infos);
      return;
    }
    run_batch(hs, count, (hipStream_t)hip_stream, [&](int32_t k, hipStream_t s) {
      solve_refined(hs[k], 0, b[k], x[k], nrhs, ld[k], tol, max_iter, s, infos ? &infos[k] : nullptr);
      if (tol <= 0) HIPCHK(hipStreamSynchronize(s));
    });
  });
}

extern "C" h2_status h2_solve_batch(h2_handle* hs, int32_t count, const void* const* b, void* const* x, int32_t nrhs,
                                    const int64_t* ld, double tol, int32_t max_iter, void* hip_stream,
                                    h2_solve_info* infos) {
  return h2_solve_batch_mode(hs, count, b, x, nrhs, ld, tol, max_iter, hip_stream, infos, H2_BATCH_FUSED);
}

extern "C" h2_status h2_contrast_gradient(h2_handle H, const void* x, const void* g, const void* lam, int32_t nrhs,
                                          int64_t ld, double* grad_chi, void* hip_stream) {
  return guarded([&] {
    validate_vec(H, x, g, nrhs, ld);
    if (!lam || !grad_chi) fail(H2_ERR_ARG, "null pointer");
    hipStream_t st = (hipStream_t)hip_stream;
    launch_contrast_grad((const double2*)x, (const double2*)g, (const double2*)lam, ld, nrhs, H->d_chi_user.p,
                         H->N, grad_chi, st);
    check_launch("contrast gradient");
  });
}

extern "C" h2_status h2_matvec(h2_handle H, const void* x, void* y, int32_t nrhs, int64_t ld, int32_t conj_transpose,
                               void* hip_stream) {
  return guarded([&] {
    validate_vec(H, x, y, nrhs, ld);
    if (x == y) fail(H2_ERR_ARG, "x and y must not alias");
    hipStream_t st = (hipStream_t)hip_stream;
    AllocScope scope(&H->allocator, st);
    const int64_t N = H->N;
    // handle-owned, grown on demand: the product stays asynchronous
    DArr<double2>& v = H->mv_in;
    DArr<double2>& w = H->mv_out;
    v.alloc(N * nrhs);
    w.alloc(N * nrhs);
    if (!conj_transpose) {
      launch_permute_in((const double2*)x, ld, H->d_perm.p, H->d_scale_mat.p, 0, N, nrhs, v.p, N, st);
      matvec_tree(H, v.p, w.p, nrhs, st);
      launch_permute_out(w.p, N, H->d_perm.p, nullptr, 0, N, nrhs, (double2*)y, ld, 0, st);
    } else {
      launch_permute_in((const double2*)x, ld, H->d_perm.p, nullptr, 1, N, nrhs, v.p, N, st);
      matvec_tree(H, v.p, w.p, nrhs, st);
      launch_permute_out(w.p, N, H->d_perm.p, H->d_scale_mat.p, 1, N, nrhs, (double2*)y, ld, 0, st);
    }
    check_launch("matvec");
  });
}

extern "C" void h2_destroy(h2_handle H) {
  if (!H) return;
  try {
    // one wait for the device, then every buffer goes back without another
    (void)hipDeviceSynchronize();
    t_device_idle = true;
    delete H;
  } catch (...) {
  }
  t_device_idle = false;
}

extern "C" const char* h2_last_error(void) { return g_err.c_str(); }

extern "C" h2_status h2_stats(h2_handle H, int64_t* out, int32_t rows_cap, int32_t* rows) {
  return guarded([&] {
    if (!H || !out || !rows) fail(H2_ERR_ARG, "NULL argument");
    if (!H->factored) fail(H2_ERR_STATE, "h2_stats before h2_factor");
    const int nr = (int)H->stats_rows.size();
    *rows = nr;
    for (int r = 0; r < std::min(nr, (int)rows_cap); ++r)
      for (int c = 0; c < 10; ++c) out[10 * r + c] = H->stats_rows[r][c];
  });
}

extern "C" h2_status h2_level_timing(h2_handle H, double* ms, int32_t cap, int32_t* count) {
  return guarded([&] {
    if (!H || !count) fail(H2_ERR_ARG, "NULL argument");
    if (!H->factored) fail(H2_ERR_STATE, "h2_level_timing before h2_factor");
    const int nr = (int)H->level_ms.size();
    *count = nr;
    if (ms)
      for (int r = 0; r < std::min(nr, (int)cap); ++r) ms[r] = H->level_ms[r];
  });
}

extern "C" h2_status h2_forced_ranks_layout(h2_handle H, int32_t* out, int64_t cap, int64_t* count) {
  return guarded([&] {
    if (!H || !count) fail(H2_ERR_ARG, "NULL argument");
    const Structure& S = H->S;
    int64_t cnt = 0;
    if (S.l0 >= 0) {
      for (int l = S.L; l >= S.l0; --l) {
        const int j = S.L - l;
        for (int t = 0; t < S.nclusters(l); ++t) {
          if (S.size[l][t] == 0) continue;
          if (out && cnt < cap) {
            out[4 * cnt] = l;
            out[4 * cnt + 1] = t;
            out[4 * cnt + 2] = H->build[j].k[t];
            out[4 * cnt + 3] = (H->factored && j < (int)H->flev.size()) ? H->flev[j].kt[t] : -1;
          }
          ++cnt;
        }
      }
    }
    *count = cnt;
  });
}

// Algorithmic flop / byte ledger of the last factorization, from its actual
// ranks (complex multiply-add = 8 flops).  Schur: every eliminated cluster i
// adds 8 (sum_a m_a)^2 r_i flops over its partners' current row counts m_a;
// bytes count every flushed block read and written once per flush and every
// panel slice read once per term.
static void compute_ledger(h2_ctx* H) {
  const Structure& S = H->S;
  H->ledger.assign(10, 0.0);
  // per family: [3f + 1] flops, [3f + 2] bytes ([3f] holds the time, filled on request)
  std::vector<double>& K = H->kernel_led;
  K.assign(27, 0.0);
  double schur_fp32 = 0.0;  // mixed form: Schur flops of clusters whose terms may run in FP32
  auto add = [&](int f, double flops, double bytes) {
    K[3 * f + 1] += flops;
    K[3 * f + 2] += bytes;
  };
  for (size_t j = 0; j < H->flev.size(); ++j) {
    const LevelPlan& P = H->plans[j];
    const FactorLevel& F = H->flev[j];
    auto dim_after = [&](int a, int c) -> double { return P.colour[a] <= c ? F.kt[a] : F.n[a]; };
    // the panel maxima the mixed flush routes by (max|C|, max|R|, max|input block| per cluster)
    std::vector<unsigned long long> pmax;
    if (H->precision == H2_MIXED && F.mixed_flush && F.d_pmax.p) {
      pmax.resize(4 * (size_t)P.nc);
      HIPCHK(hipMemcpy(pmax.data(), F.d_pmax.p, pmax.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost));
    }
    auto flush_bytes = [&](const ColourPlan& C, int c) {
      if (!C.sc_slot.empty()) H->ledger[7] += 1.0;
      for (size_t x = 0; x < C.sc_slot.size(); ++x) {
        if (C.sc_sp[4 * x] > 0) continue;  // a later chunk of a split task: same block
        const int s = C.sc_slot[x];
        H->ledger[9] += 32.0 * dim_after(P.slot_a[s], c) * dim_after(P.slot_b[s], c);
      }
    };
    for (int c = 0; c < P.ncol; ++c) {
      flush_bytes(P.cols[c], c - 1);
      // Step 2: every stored block with an end in this colour, read and written once;
      // Q~^H from the left when its row cluster is in the colour, conj(Q~) from the right
      // when its column cluster is
      for (int sl : P.cols[c].pj_slot) {
        const int x = P.slot_a[sl], y = P.slot_b[sl];
        const bool cx = P.colour[x] == c, cy = P.colour[y] == c;
        const double rows = cx ? F.n[x] : dim_after(x, c - 1), cols = cy ? F.n[y] : dim_after(y, c - 1);
        add(2, (cx ? 8.0 * F.n[x] * F.n[x] * cols : 0.0) + (cy ? 8.0 * rows * F.n[y] * F.n[y] : 0.0),
            32.0 * rows * cols);
      }
      for (int i : P.cols[c].cl) {
        const double n = F.n[i], kt = F.kt[i], r = n - kt, k = F.k[i], d = n - k;
        double M = 0.0, M2 = 0.0, fillcols = 0.0, np = 0.0;
        for (int x = P.np_ptr[i]; x < P.np_ptr[i + 1]; ++x) {
          const int a = P.np_cl[x];
          const double ma = (a == i) ? kt : (P.colour[a] < c ? F.kt[a] : F.n[a]);
          M += ma;
          M2 += ma * ma;
          np += 1.0;
        }
        for (int x = P.fp_ptr[i]; x < P.fp_ptr[i + 1]; ++x) {
          const int b = P.fp_cl[x];
          fillcols += (P.colour[b] < c ? F.kt[b] : F.n[b]);
        }
        // targets (a, b) with a <= b only: the other half is their transpose
        const double schur = 8.0 * r * 0.5 * (M * M + M2);
        H->ledger[6] += schur;
        if (!pmax.empty() && r > 0) {
          double gc, gr, z;
          std::memcpy(&gc, &pmax[4 * i], 8);
          std::memcpy(&gr, &pmax[4 * i + 1], 8);
          std::memcpy(&z, &pmax[4 * i + 2], 8);
          if (gc * gr * std::sqrt(r) <= F32_KAPPA * z) schur_fp32 += schur;
        }
        H->ledger[9] += 16.0 * (np + 1.0) * M * r;  // C rows and R columns of every term
        // Gram, B_perp transforms, projections (one side of every stored block of row i), LU, panels
        const double gram = 8.0 * n * n * fillcols + 8.0 * (n * n * d + n * d * d + n * d * d);
        const double proj = 8.0 * n * n * (M - kt + n + fillcols);
        const double lu = 8.0 / 3.0 * r * r * r + 8.0 * r * r * (M + M);
        H->ledger[8] += schur + gram + proj + lu;
        // Gram G = W W^H of the n x fillcols fill-ins: W read, G written
        add(0, 8.0 * n * n * fillcols, 16.0 * n * fillcols + 16.0 * n * n);
        // G' = Bp^H G Bp (n^2 d + n d^2) and Q~ = [B, Bp U'] (n d^2): G, Bp read, Q~ written
        add(1, 8.0 * (n * n * d + 2.0 * n * d * d), 16.0 * (2.0 * n * n + n * d));
        // Q~ of the cluster read once by the projections
        add(2, 0.0, 16.0 * n * n);
        // LU of the r x r block and both triangular inverses: block read, L^-1 P and U^-1 written
        add(3, 16.0 / 3.0 * r * r * r, 48.0 * r * r);
        // C = Z_ai' U^-1 and R = L^-1 P Z_i'a over the M partner rows: inputs read for each panel,
        // panels written, L^-1 P and U^-1 read
        add(4, 16.0 * r * r * M, 64.0 * r * M + 32.0 * r * r);
        // one right-hand side: Q~ (forward and backward), L^-1 P, U^-1, C and R panels
        K[24] += 16.0 * (2.0 * n * n + 2.0 * r * r + 2.0 * r * M);
      }
    }
    flush_bytes(P.fin, P.ncol - 1);
  }
  const double nf = (double)H->nf;
  H->ledger[8] += 8.0 / 3.0 * nf * nf * nf;
  add(5, H->ledger[6], H->ledger[9]);
  add(6, 0.0, 32.0 * H->merge_elems);  // every parent element written once, its source read once
  add(7, 8.0 / 3.0 * nf * nf * nf, 32.0 * nf * nf);
  K[24] += 16.0 * nf * nf;  // the final block's L and U factors
  // matvec: near blocks, the expanded bases of every level and the couplings, once each
  double mv = (double)H->near_orig.n;
  for (const BuildLevel& B : H->build) mv += (double)B.V.n + (double)B.S.n;
  K[25] = 16.0 * mv;
  K[26] = H->ledger[6] > 0 ? schur_fp32 / H->ledger[6] : 0.0;
  (void)S;
  H->ledger_valid = true;
}

extern "C" h2_status h2_factor_timing(h2_handle H, double* out, int32_t n_out) {
  return guarded([&] {
    if (!H || !out || n_out < 6) fail(H2_ERR_ARG, "invalid argument");
    if (!H->factored) fail(H2_ERR_STATE, "h2_factor_timing before h2_factor");
    for (int i = 0; i < 6; ++i) out[i] = H->timing[i];
    if (n_out > 6 && !H->ledger_valid) compute_ledger(H);
    for (int i = 6; i < std::min<int32_t>(n_out, 10); ++i) out[i] = H->ledger.size() > (size_t)i ? H->ledger[i] : 0.0;
  });
}

extern "C" h2_status h2_set_kernel_timing(h2_handle H, int32_t enable) {
  return guarded([&] {
    if (!H) fail(H2_ERR_ARG, "handle is NULL");
    H->kernel_timing = enable != 0;
  });
}

extern "C" h2_status h2_kernel_ledger(h2_handle H, double* out, int32_t n_out) {
  return guarded([&] {
    if (!H || !out || n_out < 26) fail(H2_ERR_ARG, "invalid argument");
    if (!H->factored) fail(H2_ERR_STATE, "h2_kernel_ledger before h2_factor");
    if (!H->ledger_valid) compute_ledger(H);
    for (int i = 0; i < std::min<int32_t>(n_out, 27); ++i) out[i] = H->kernel_led[i];
    for (int f = 0; f < 8; ++f) out[3 * f] = H->kernel_ms[f];
  });
}
