// gfx950 kernels of the H^2 direct solver.
//
// Layout conventions: complex double ("double2") matrices are column-major;
// every cluster / block / panel lives in a packed arena at an element offset
// given per object.  Inside a cluster the coordinates after Steps 0-2 are
// "kept first": Q~ = [B  B_add  B~perp], so the k~ kept coordinates occupy
// rows [0, k~) and the r = n - k~ eliminated ones rows [k~, n).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

#include "h2_device.hpp"
#include "h2_kernels.hpp"

namespace h2 {

// The block index a kernel body works on: the hardware one for a problem's own
// launch, or, inside a launch shared by several problems (BatchEntry), the
// position within that problem's share.
struct VBlock {
  int x, y, z, gx, gy, gz;
};
__device__ __forceinline__ VBlock vblock() {
  return {(int)blockIdx.x, (int)blockIdx.y, (int)blockIdx.z, (int)gridDim.x, (int)gridDim.y, (int)gridDim.z};
}
// Entry of a shared launch that owns this workgroup (entries sorted by `first`).
// The table is read through the constant address space: the index is made
// wave-uniform, the fields are scalar loads, and the compiler may load a field
// again where it is used rather than hold every field in registers (as it does
// for kernel arguments).  The table is never written while a launch runs.
typedef const __attribute__((address_space(4))) BatchEntry ConstEntry;
struct EntryRef {
  const LevelView& v;
  const ColourTasks& c;
  double2* buf;
  int64_t aux;
  int i0;
};
__device__ __forceinline__ EntryRef locate(const BatchEntry* E, int ne, VBlock& VB) {
  ConstEntry* CE = (ConstEntry*)E;
  const int lin = blockIdx.x;
  int lo = 0, hi = ne - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (CE[mid].first <= lin)
      lo = mid;
    else
      hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  ConstEntry& e = CE[lo];
  int r = lin - e.first;
  VB.gx = e.gx;
  VB.gy = e.gy;
  VB.gz = e.gz;
  VB.x = r % e.gx;
  r /= e.gx;
  VB.y = r % e.gy;
  VB.z = r / e.gy;
  return {*(const LevelView*)&e.v, *(const ColourTasks*)&e.c, e.buf, e.aux, e.i0};
}

// The same for the entries of a shared sweep launch.
typedef const __attribute__((address_space(4))) SweepEntry ConstSweepEntry;
struct SweepRef {
  const LevelView& v;
  const ColourTasks& c;
  double2* vec;
  const int64_t* voff;
  int64_t ldv;
  int nrhs, adj;
  double2* part;
  int nsplit;
  double2* scratch;
};
__device__ __forceinline__ SweepRef locate_sweep(const SweepEntry* E, int ne, VBlock& VB) {
  ConstSweepEntry* CE = (ConstSweepEntry*)E;
  const int lin = blockIdx.x;
  int lo = 0, hi = ne - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (CE[mid].first <= lin)
      lo = mid;
    else
      hi = mid - 1;
  }
  lo = __builtin_amdgcn_readfirstlane(lo);
  ConstSweepEntry& e = CE[lo];
  int r = lin - e.first;
  VB.gx = e.gx;
  VB.gy = e.gy;
  VB.gz = e.gz;
  VB.x = r % e.gx;
  r /= e.gx;
  VB.y = r % e.gy;
  VB.z = r / e.gy;
  return {*(const LevelView*)&e.v, *(const ColourTasks*)&e.c, e.vec, e.voff, e.ldv, e.nrhs, e.adj, e.part, e.nsplit,
          e.scratch};
}

static inline __host__ __device__ int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }

// ===========================================================================
// VIE matrix entries Z = A D^-1 (generated on the fly)
// ===========================================================================
__device__ __forceinline__ double2 zentry(const GeomView& g, int64_t x, int64_t y) {
  if (x == y) {
    const double c = g.chi[x];
    const double den = g.k2h3 * c;  // k^2 h^3 chi
    return make_double2((1.0 + c * g.diag_re_c) / den, (c * g.diag_im_c) / den);
  }
  const double dx = g.pts[3 * x] - g.pts[3 * y];
  const double dy = g.pts[3 * x + 1] - g.pts[3 * y + 1];
  const double dz = g.pts[3 * x + 2] - g.pts[3 * y + 2];
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  double s, c;
  sincos(g.k * r, &s, &c);
  const double den = 4.0 * M_PI * r;
  return make_double2(c / den, -s / den);
}

__device__ __forceinline__ bool near_bit(const uint32_t* mask, int64_t nc, int64_t a, int64_t b) {
  const int64_t bit = a * nc + b;
  return (mask[bit >> 5] >> (bit & 31)) & 1u;
}

__global__ void __launch_bounds__(256) k_near_blocks(GeomView g, const int32_t* pr, const int32_t* pc,
                                                     const int64_t* off, const int64_t* rs,
                                                     const int32_t* rn, const int64_t* cs,
                                                     const int32_t* cn, double2* out) {
  const int p = blockIdx.x;
  const int a = pr[p], b = pc[p];
  const int m = rn[a], n = cn[b];
  const int64_t r0 = rs[a], c0 = cs[b];
  double2* o = out + off[p];
  for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
    const int i = e % m, j = e / m;
    o[e] = zentry(g, r0 + i, c0 + j);
  }
}

void launch_near_blocks(const GeomView& g, const int32_t* pr, const int32_t* pc, const int64_t* off,
                        const int64_t* rs, const int32_t* rn, const int64_t* cs, const int32_t* cn,
                        int npairs, double2* out, hipStream_t st) {
  if (npairs <= 0) return;
  hipLaunchKernelGGL(k_near_blocks, dim3(npairs), dim3(256), 0, st, g, pr, pc, off, rs, rn, cs, cn, out);
}

// e^{-jkr} / (4 pi r) from the table tab[m] = (cos, sin)(m pi/128): the phase
// kr = q pi/128 + f with q the nearest integer (two-part pi/128, so f carries
// no reduction error beyond one rounding), |f| <= pi/256, cos f and sin f by
// their Taylor series through f^6 and f^7 (truncation < 2e-21), combined by the
// angle-addition formulas: the classic table-driven scheme of elementary-function
// libraries.  The phase kr itself is only known to ~1e-16 kr, which dominates.
constexpr double PHASE_STEP_HI = 0.02454369260617026;    // pi / 128 rounded to double
constexpr double PHASE_STEP_LO = 9.567553118338697e-19;  // pi / 128 - PHASE_STEP_HI
constexpr double PHASE_INV_STEP = 40.74366543152521;     // 128 / pi

__device__ __forceinline__ double2 zfar(double xa, double xb, double xc, double ya, double yb, double yc, double k,
                                        const double2* tab) {
  const double dx = xa - ya;
  const double dy = xb - yb;
  const double dz = xc - yc;
  const double r = sqrt(dx * dx + dy * dy + dz * dz);
  const double ph = k * r;
  const double q = rint(ph * PHASE_INV_STEP);
  const double f = fma(-q, PHASE_STEP_LO, fma(-q, PHASE_STEP_HI, ph));
  const double f2 = f * f;
  const double sf = f * (1.0 + f2 * (-1.0 / 6.0 + f2 * (1.0 / 120.0 + f2 * (-1.0 / 5040.0))));
  const double cf = 1.0 + f2 * (-0.5 + f2 * (1.0 / 24.0 + f2 * (-1.0 / 720.0)));
  const double2 t = tab[(int)q & 255];
  const double c = t.x * cf - t.y * sf;
  const double s = t.y * cf + t.x * sf;
  const double inv = 1.0 / (4.0 * M_PI * r);
  return make_double2(c * inv, -s * inv);
}

// Fills tab[0..255] with (cos, sin)(m pi/128); 256 threads.
__device__ __forceinline__ void phase_table(double2* tab) {
  const int th = threadIdx.x;
  double sv, cv;
  sincos(fma((double)th, PHASE_STEP_HI, (double)th * PHASE_STEP_LO), &sv, &cv);
  tab[th] = make_double2(cv, sv);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Leaf far-field Gram G_t = sum_y Zm(t, y) Zm(t, y)^H (Zm: the entries of Z, zero
// where the leaf clusters of t and y form an inadmissible pair), split over column chunks.
// grid: (cluster, tile(2x2), chunk).  The tile's rows stay in registers; per slab
// each thread loads one column point and its mask bit, and the next slab's
// entries are generated while the current one is on the matrix cores.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_leaf_gram(GeomView g, const uint32_t* mask, int level,
                                                   const int64_t* cstart, const int32_t* csize,
                                                   int64_t kchunk, double2* part, int64_t stride,
                                                   const int64_t* goff, int ntr) {
  __shared__ TileSmem<double> s;
  __shared__ double2 tab[256];
  const int t = blockIdx.x, tile = blockIdx.y, ch = blockIdx.z;
  const int n = csize[t];
  const int tr = tile % ntr, tc = tile / ntr;
  if (tr * 64 >= n || tc * 64 >= n) return;
  phase_table(tab);
  const int m = min(64, n - tr * 64), nn = min(64, n - tc * 64);
  const int64_t k_begin = (int64_t)ch * kchunk;
  const int64_t k_end = min(g.N, k_begin + kchunk);
  const int64_t row_a = cstart[t] + tr * 64, row_b = cstart[t] + tc * 64;
  const int th = threadIdx.x;
  const int kk = th & 15;
  const bool diag = tr == tc;
  const int sh = g.L - level;
  const int64_t ncl = (int64_t)1 << level;
  const int64_t cx = (int64_t)(g.leafid[row_a] >> sh);
  double ra[4][3], rb[4][3];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int i = (th >> 4) + 16 * e;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      ra[e][d] = i < m ? g.pts[3 * (row_a + i) + d] : 0.0;
      rb[e][d] = (!diag && i < nn) ? g.pts[3 * (row_b + i) + d] : 0.0;
    }
  }
  double2 v[4], w[4];
  auto entries = [&](int64_t y, bool far, double ya, double yb, double yc) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = (th >> 4) + 16 * e;
      v[e] = (far && i < m) ? zfar(ra[e][0], ra[e][1], ra[e][2], ya, yb, yc, g.k, tab) : make_double2(0, 0);
      if (diag)
        w[e] = i < nn ? v[e] : make_double2(0, 0);
      else
        w[e] = (far && i < nn) ? zfar(rb[e][0], rb[e][1], rb[e][2], ya, yb, yc, g.k, tab) : make_double2(0, 0);
    }
  };
  auto column = [&](int64_t y, bool& far, double& ya, double& yb, double& yc) {
    far = false;
    ya = yb = yc = 0.0;
    if (y < k_end) {
      far = !near_bit(mask, ncl, cx, (int64_t)(g.leafid[y] >> sh));
      ya = g.pts[3 * y];
      yb = g.pts[3 * y + 1];
      yc = g.pts[3 * y + 2];
    }
  };
  TileAcc<double> acc;
  acc.zero();
  {
    bool far;
    double ya, yb, yc;
    column(k_begin + kk, far, ya, yb, yc);
    entries(k_begin + kk, far, ya, yb, yc);
  }
  for (int64_t k0 = k_begin; k0 < k_end; k0 += TK) {
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = (th >> 4) + 16 * e;
      s.are[kk][i] = v[e].x;
      s.aim[kk][i] = v[e].y;
      s.bre[kk][i] = w[e].x;
      s.bim[kk][i] = -w[e].y;
    }
    __syncthreads();
    const bool more = k0 + TK < k_end;
    bool far = false;
    double ya = 0.0, yb = 0.0, yc = 0.0;
    if (more) column(k0 + TK + kk, far, ya, yb, yc);
    mma_slab_bal<double>(s, acc, TK, (m + 15) >> 4, (nn + 15) >> 4);
    if (more) entries(k0 + TK + kk, far, ya, yb, yc);
  }
  double2* G = part + (int64_t)ch * stride + goff[t] + tr * 64 + (int64_t)tc * 64 * n;
  store_tile<double, double2>(acc, G, n, m, nn, ST_SET);
}

void launch_leaf_gram(const GeomView& g, const uint32_t* mask, int ncl, int level, const int64_t* cstart,
                      const int32_t* csize, int64_t kchunk, int nchunks, double2* part, int64_t stride,
                      const int64_t* goff, int ntr, hipStream_t st) {
  if (ncl <= 0) return;
  hipLaunchKernelGGL(k_leaf_gram, dim3(ncl, ntr * ntr, nchunks), dim3(256), 0, st, g, mask, level, cstart,
                     csize, kchunk, part, stride, goff, ntr);
}

__global__ void k_gram_reduce(const double2* part, double2* out, int64_t total, int nchunks,
                              int64_t stride) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    double2 a = part[e];
    for (int c = 1; c < nchunks; ++c) a = cadd(a, part[(int64_t)c * stride + e]);
    out[e] = a;
  }
}

void launch_gram_reduce(const double2* part, double2* out, const int64_t* off, const int32_t* sz, int ncl,
                        int nchunks, int64_t stride, hipStream_t st) {
  (void)off;
  (void)sz;
  (void)ncl;
  if (stride <= 0) return;
  int blocks = (int)imin64(4096, (stride + 255) / 256);
  hipLaunchKernelGGL(k_gram_reduce, dim3(blocks), dim3(256), 0, st, part, out, stride, nchunks, stride);
}

// ---------------------------------------------------------------------------
// Non-leaf construction rows: Y_c = V_c^H Zm(c, J) for children c (K = #c, Zm
// the entries of Z masked to the far field at `level`),
// written into the stacked row block of the parent.  grid: (child, tiles)
//
// Every point of c lies in the same level-`level` cluster, so the far-field
// mask of a column is fixed for the workgroup: each thread keeps its four
// columns' coordinates and mask bits in registers, and per slab loads one
// point's coordinates.  The next slab's V_c^H elements and point are fetched
// while the current slab is on the matrix cores, and its entries are generated
// after the MFMAs are issued, so the transcendental work overlaps them.  A
// column is masked (zero) where the level-`level` clusters of its point and of
// c form an inadmissible pair.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_proj_rows(GeomView g, const uint32_t* mask, int level,
                                                   const int64_t* cstart, const int32_t* csize,
                                                   const int32_t* ck, const int64_t* voff,
                                                   const double2* V, const int64_t* yoff,
                                                   const int32_t* yld, double2* Y, int64_t col0,
                                                   int ncols, int ntr) {
  __shared__ TileSmem<double> s;
  __shared__ double2 tab[256];
  const int c = blockIdx.x;
  const int kc = ck[c];
  const int tr = blockIdx.y % ntr, tc = blockIdx.y / ntr;
  if (tr * 64 >= kc || tc * 64 >= ncols) return;
  const int m = min(64, kc - tr * 64), nn = min(64, ncols - tc * 64);
  const int K = csize[c];
  const double2* A = V + voff[c] + (int64_t)tr * 64 * K;  // op C of V_c (#c x k_c, ld #c)
  const int64_t x0 = cstart[c];
  const int64_t y0 = col0 + tc * 64;
  const int th = threadIdx.x;
  phase_table(tab);
  const int kk = th & 15;
  const int mt = (m + 15) >> 4, nt = (nn + 15) >> 4;
  TileAcc<double> acc;
  acc.zero();
  if (K > 0) {
    const int sh = g.L - level;
    const int64_t ncl = (int64_t)1 << level;
    const int64_t cx = (int64_t)(g.leafid[x0] >> sh);
    double ya[4], yb[4], yc[4];
    bool far[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = (th >> 4) + 16 * e;
      far[e] = false;
      ya[e] = yb[e] = yc[e] = 0.0;
      if (j < nn) {
        const int64_t y = y0 + j;
        far[e] = !near_bit(mask, ncl, cx, (int64_t)(g.leafid[y] >> sh));
        ya[e] = g.pts[3 * y];
        yb[e] = g.pts[3 * y + 1];
        yc[e] = g.pts[3 * y + 2];
      }
    }
    // slab 0 operands
    double2 a[4], b[4];
    double xa = 0.0, xb = 0.0, xc = 0.0;
    bool xin = kk < K;
    if (xin) {
      xa = g.pts[3 * (x0 + kk)];
      xb = g.pts[3 * (x0 + kk) + 1];
      xc = g.pts[3 * (x0 + kk) + 2];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = (th >> 4) + 16 * e;
      a[e] = (i < m && kk < K) ? A[kk + (int64_t)i * K] : make_double2(0, 0);
      b[e] = (far[e] && xin) ? zfar(xa, xb, xc, ya[e], yb[e], yc[e], g.k, tab) : make_double2(0, 0);
    }
    for (int k0 = 0; k0 < K; k0 += TK) {
      __syncthreads();
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = (th >> 4) + 16 * e;
        s.are[kk][i] = a[e].x;
        s.aim[kk][i] = -a[e].y;
        s.bre[kk][i] = b[e].x;
        s.bim[kk][i] = b[e].y;
      }
      __syncthreads();
      const int k1 = k0 + TK;
      const bool more = k1 < K;
      if (more) {
        const int k = k1 + kk;
        xin = k < K;
        if (xin) {
          xa = g.pts[3 * (x0 + k)];
          xb = g.pts[3 * (x0 + k) + 1];
          xc = g.pts[3 * (x0 + k) + 2];
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = (th >> 4) + 16 * e;
          a[e] = (i < m && k < K) ? A[k + (int64_t)i * K] : make_double2(0, 0);
        }
      }
      mma_slab_bal<double>(s, acc, TK, mt, nt);
      if (more) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
          b[e] = (far[e] && xin) ? zfar(xa, xb, xc, ya[e], yb[e], yc[e], g.k, tab) : make_double2(0, 0);
      }
    }
  }
  double2* out = Y + yoff[c] + tr * 64 + (int64_t)tc * 64 * yld[c];
  store_tile<double, double2>(acc, out, yld[c], m, nn, ST_SET);
}

void launch_proj_rows(const GeomView& g, const uint32_t* mask, int level, int nch, const int64_t* cstart,
                      const int32_t* csize, const int32_t* ck, const int64_t* voff, const double2* V,
                      const int64_t* yoff, const int32_t* yld, double2* Y, int64_t col0, int ncols,
                      int ntr, hipStream_t st) {
  if (nch <= 0) return;
  const int tiles = ntr * ((ncols + 63) / 64);
  hipLaunchKernelGGL(k_proj_rows, dim3(nch, tiles), dim3(256), 0, st, g, mask, level, cstart, csize, ck,
                     voff, V, yoff, yld, Y, col0, ncols, ntr);
}

// G_t (d x d) += Y_t Y_t^H over ncols columns (Y_t ld = d).  grid: (cluster, 2x2 tiles)
__global__ void __launch_bounds__(256) k_gram_acc(const int32_t* dim, const int64_t* yoff, const double2* Y,
                                                  int ncols, const int64_t* goff, double2* G, int ntr) {
  __shared__ TileSmem<double> s;
  const int t = blockIdx.x;
  const int d = dim[t];
  const int tr = blockIdx.y % ntr, tc = blockIdx.y / ntr;
  if (tr * 64 >= d || tc * 64 >= d) return;
  const int m = min(64, d - tr * 64), nn = min(64, d - tc * 64);
  const double2* Yt = Y + yoff[t];
  TileAcc<double> acc;
  acc.zero();
  gemm_tile<double, double2>(s, acc, Yt + tr * 64, d, OP_N, Yt + tc * 64, d, OP_C, m, nn, ncols);
  store_tile<double, double2>(acc, G + goff[t] + tr * 64 + (int64_t)tc * 64 * d, d, m, nn, ST_ADD);
}

void launch_gram_acc(int ncl, const int32_t* dim, const int64_t* yoff, const double2* Y, int ncols,
                     const int64_t* goff, double2* G, int ntr, hipStream_t st) {
  if (ncl <= 0) return;
  hipLaunchKernelGGL(k_gram_acc, dim3(ncl, ntr * ntr), dim3(256), 0, st, dim, yoff, Y, ncols, goff, G, ntr);
}

// X_ts = V_t^H Z(t, s) (k_t x #s) for admissible pairs.  grid: (pair, tiles)
__global__ void __launch_bounds__(256) k_coupling_x(GeomView g, const int32_t* pt, const int32_t* ps,
                                                    const int64_t* tstart, const int32_t* tsz,
                                                    const int32_t* tk, const int64_t* voff,
                                                    const double2* V, const int64_t* xoff, double2* X,
                                                    int ntr) {
  __shared__ TileSmem<double> s;
  const int p = blockIdx.x;
  const int t = pt[p], u = ps[p];
  const int kt = tk[t], K = tsz[t], ns = tsz[u];
  const int tr = blockIdx.y % ntr, tc = blockIdx.y / ntr;
  if (tr * 64 >= kt || tc * 64 >= ns) return;
  const int m = min(64, kt - tr * 64), nn = min(64, ns - tc * 64);
  const double2* A = V + voff[t] + (int64_t)tr * 64 * K;
  const int64_t x0 = tstart[t], y0 = tstart[u] + tc * 64;
  TileAcc<double> acc;
  acc.zero();
  for (int k0 = 0; k0 < K; k0 += TK) {
    __syncthreads();
    load_a<double, double2>(s, A, K, OP_C, m, K, k0);
    {
      const int th = threadIdx.x;
      const int kk = th & 15;
      const int k = k0 + kk;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int j = (th >> 4) + 16 * e;
        double2 v = make_double2(0, 0);
        if (j < nn && k < K) v = zentry(g, x0 + k, y0 + j);
        s.bre[kk][j] = v.x;
        s.bim[kk][j] = v.y;
      }
    }
    __syncthreads();
    mma_slab_bal<double>(s, acc, TK, (m + 15) >> 4, (nn + 15) >> 4);
  }
  store_tile<double, double2>(acc, X + xoff[p] + tr * 64 + (int64_t)tc * 64 * kt, kt, m, nn, ST_SET);
}

void launch_coupling_x(const GeomView& g, int npairs, int ntr, int ntc, const int32_t* pt, const int32_t* ps,
                       const int64_t* tstart, const int32_t* tsz, const int32_t* tk, const int64_t* voff,
                       const double2* V, const int64_t* xoff, double2* X, hipStream_t st) {
  if (npairs <= 0) return;
  hipLaunchKernelGGL(k_coupling_x, dim3(npairs, ntr * ntc), dim3(256), 0, st, g, pt, ps, tstart, tsz, tk, voff,
                     V, xoff, X, ntr);
}

// ===========================================================================
// Generic host-resolved batched GEMM
// ===========================================================================
__global__ void __launch_bounds__(256) k_gemm_batched(const GemmTask* tasks, const int32_t* tile_task,
                                                      const int32_t* tile_rc) {
  __shared__ TileSmem<double> s;
  const GemmTask T = tasks[tile_task[blockIdx.x]];
  const int rc = tile_rc[blockIdx.x];
  const int tr = rc & 0xffff, tc = rc >> 16;
  const int m = min(64, T.m - tr * 64), n = min(64, T.n - tc * 64);
  if (m <= 0 || n <= 0) return;
  const double2* A = (T.opA == OP_N || T.opA == OP_R) ? T.A + tr * 64 : T.A + (int64_t)tr * 64 * T.lda;
  const double2* B = (T.opB == OP_N || T.opB == OP_R) ? T.B + (int64_t)tc * 64 * T.ldb : T.B + tc * 64;
  TileAcc<double> acc;
  acc.zero();
  gemm_tile<double, double2>(s, acc, A, T.lda, T.opA, B, T.ldb, T.opB, m, n, T.K);
  store_tile<double, double2>(acc, T.C + tr * 64 + (int64_t)tc * 64 * T.ldc, T.ldc, m, n, T.mode);
}

void launch_gemm_batched(const GemmTask* tasks, const int32_t* tile_task, const int32_t* tile_rc, int ntiles,
                         hipStream_t st) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(k_gemm_batched, dim3(ntiles), dim3(256), 0, st, tasks, tile_task, tile_rc);
}

// One GEMM passed by value (no task list in device memory): tile (blockIdx.x, blockIdx.y)
__global__ void __launch_bounds__(256) k_gemm_one(GemmTask T) {
  __shared__ TileSmem<double> s;
  const int tr = blockIdx.x, tc = blockIdx.y;
  const int m = min(64, T.m - tr * 64), n = min(64, T.n - tc * 64);
  if (m <= 0 || n <= 0) return;
  const double2* A = (T.opA == OP_N || T.opA == OP_R) ? T.A + tr * 64 : T.A + (int64_t)tr * 64 * T.lda;
  const double2* B = (T.opB == OP_N || T.opB == OP_R) ? T.B + (int64_t)tc * 64 * T.ldb : T.B + tc * 64;
  TileAcc<double> acc;
  acc.zero();
  gemm_tile<double, double2>(s, acc, A, T.lda, T.opA, B, T.ldb, T.opB, m, n, T.K);
  store_tile<double, double2>(acc, T.C + tr * 64 + (int64_t)tc * 64 * T.ldc, T.ldc, m, n, T.mode);
}

void launch_gemm_one(const GemmTask& T, hipStream_t st) {
  if (T.m <= 0 || T.n <= 0) return;
  hipLaunchKernelGGL(k_gemm_one, dim3((T.m + 63) / 64, (T.n + 63) / 64), dim3(256), 0, st, T);
}

// C = A^T for each task (A m x n, ld lda -> C n x m, ld ldc)
__global__ void k_transpose_copy(const GemmTask* tasks) {
  const GemmTask T = tasks[blockIdx.x];
  for (int e = threadIdx.x; e < T.m * T.n; e += blockDim.x) {
    const int i = e % T.m, j = e / T.m;
    T.C[j + (int64_t)i * T.ldc] = T.A[i + (int64_t)j * T.lda];
  }
}

void launch_transpose_copy(const GemmTask* tasks, int ntasks, hipStream_t st) {
  if (ntasks <= 0) return;
  hipLaunchKernelGGL(k_transpose_copy, dim3(ntasks), dim3(256), 0, st, tasks);
}

// ===========================================================================
// Cyclic Jacobi eigensolver for small Hermitian matrices
// ===========================================================================
struct Rot {
  double c, s;
  double2 e;  // unit phase of the off-diagonal entry
};

__device__ __forceinline__ void rr_pair(int k, int round, int m, int& p, int& q) {
  auto pl = [&](int pos) { return pos == 0 ? 0 : 1 + ((pos - 1 + round) % (m - 1)); };
  const int a = pl(k), b = pl(m - 1 - k);
  p = min(a, b);
  q = max(a, b);
}

// Diagonalise the m x m (m even, padded) Hermitian matrix A (ld m) in place,
// accumulating U (ld m, starts as identity).  256 threads.
__device__ void jacobi_core(double2* A, double2* U, int m, int rel, Rot* rot, int* flag, double fro) {
  const int tid = threadIdx.x;
  const int h = m / 2;
  // stopping rules reachable in double precision: |g_pq| <= 1e-15 ||G||_F (absolute)
  // or |g_pq| <= 4e-16 sqrt(|g_pp g_qq|) (relative accuracy for the small eigenvalues)
  const double tol_abs = 1e-15 * fro;
  for (int sweep = 0; sweep < 24; ++sweep) {
    if (tid == 0) *flag = 0;
    __syncthreads();
    for (int round = 0; round < m - 1; ++round) {
      if (tid < h) {
        int p, q;
        rr_pair(tid, round, m, p, q);
        const double a = A[p + p * m].x, d = A[q + q * m].x;
        const double2 b = A[p + q * m];
        const double bb = sqrt(cabs2(b));
        bool go = rel ? (bb > 4e-16 * sqrt(fabs(a * d)) && bb > 1e-300) : (bb > tol_abs);
        Rot R;
        if (go) {
          const double th = (d - a) / (2.0 * bb);
          const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
          R.c = 1.0 / sqrt(t * t + 1.0);
          R.s = t * R.c;
          R.e = make_double2(b.x / bb, b.y / bb);
          *flag = 1;
        } else {
          R.c = 1.0;
          R.s = 0.0;
          R.e = make_double2(1.0, 0.0);
        }
        rot[tid] = R;
      }
      __syncthreads();
      // two-sided update on 2x2 blocks (P <= Q); one block per work item
      for (int w = tid; w < h * h; w += blockDim.x) {
        const int P = w / h, Qi = w % h;
        if (P > Qi) continue;
        int p1, q1, p2, q2;
        rr_pair(P, round, m, p1, q1);
        rr_pair(Qi, round, m, p2, q2);
        const Rot a = rot[P], b = rot[Qi];
        const double2 x00 = A[p1 + p2 * m], x01 = A[p1 + q2 * m], x10 = A[q1 + p2 * m], x11 = A[q1 + q2 * m];
        // left: J_P^H X ; J^H = [[c, -s e], [s, c e]]
        const double2 se = make_double2(a.s * a.e.x, a.s * a.e.y), ce = make_double2(a.c * a.e.x, a.c * a.e.y);
        double2 y00 = make_double2(a.c * x00.x, a.c * x00.y), y01 = make_double2(a.c * x01.x, a.c * x01.y);
        y00 = csub(y00, cmul(se, x10));
        y01 = csub(y01, cmul(se, x11));
        double2 y10 = cadd(make_double2(a.s * x00.x, a.s * x00.y), cmul(ce, x10));
        double2 y11 = cadd(make_double2(a.s * x01.x, a.s * x01.y), cmul(ce, x11));
        // right: Y J_Q ; J = [[c, s], [-s conj(e), c conj(e)]]
        const double2 sec = make_double2(b.s * b.e.x, -b.s * b.e.y), cec = make_double2(b.c * b.e.x, -b.c * b.e.y);
        double2 z00 = csub(make_double2(b.c * y00.x, b.c * y00.y), cmul(sec, y01));
        double2 z01 = cadd(make_double2(b.s * y00.x, b.s * y00.y), cmul(cec, y01));
        double2 z10 = csub(make_double2(b.c * y10.x, b.c * y10.y), cmul(sec, y11));
        double2 z11 = cadd(make_double2(b.s * y10.x, b.s * y10.y), cmul(cec, y11));
        if (P == Qi) {
          z00.y = 0.0;
          z11.y = 0.0;
          if (a.s != 0.0) {
            z01 = make_double2(0.0, 0.0);
            z10 = make_double2(0.0, 0.0);
          } else {
            z10 = cconj(z01);
          }
          A[p1 + p1 * m] = z00;
          A[p1 + q1 * m] = z01;
          A[q1 + p1 * m] = z10;
          A[q1 + q1 * m] = z11;
        } else {
          A[p1 + p2 * m] = z00;
          A[p1 + q2 * m] = z01;
          A[q1 + p2 * m] = z10;
          A[q1 + q2 * m] = z11;
          A[p2 + p1 * m] = cconj(z00);
          A[q2 + p1 * m] = cconj(z01);
          A[p2 + q1 * m] = cconj(z10);
          A[q2 + q1 * m] = cconj(z11);
        }
      }
      // U <- U J for every row and pair
      for (int w = tid; w < m * h; w += blockDim.x) {
        const int row = w % m, Qi = w / m;
        int p, q;
        rr_pair(Qi, round, m, p, q);
        const Rot b = rot[Qi];
        if (b.s == 0.0) continue;
        const double2 up = U[row + p * m], uq = U[row + q * m];
        const double2 sec = make_double2(b.s * b.e.x, -b.s * b.e.y), cec = make_double2(b.c * b.e.x, -b.c * b.e.y);
        U[row + p * m] = csub(make_double2(b.c * up.x, b.c * up.y), cmul(sec, uq));
        U[row + q * m] = cadd(make_double2(b.s * up.x, b.s * up.y), cmul(cec, uq));
      }
      __syncthreads();
    }
    __syncthreads();
    if (*flag == 0) break;
    __syncthreads();
  }
}

// Shared driver: copy G (d x d, ld ldg) into the padded work matrix, run Jacobi,
// write sorted eigenvalues (descending) and eigenvectors (ld ldu).
__device__ void jacobi_solve(const double2* G, int ldg, int d, double2* A, double2* Uw, double* lam,
                             double2* Uout, int ldu, int rel, Rot* rot, int* flag, double* red) {
  const int m = d + (d & 1);
  const int tid = threadIdx.x;
  double part = 0.0;
  for (int e = tid; e < m * m; e += blockDim.x) {
    const int i = e % m, j = e / m;
    double2 v = make_double2(0, 0);
    if (i < d && j < d) v = G[i + (int64_t)j * ldg];
    if (i == j) v.y = 0.0;
    A[e] = v;
    Uw[e] = make_double2(i == j ? 1.0 : 0.0, 0.0);
    part += cabs2(v);
  }
  const double fro = sqrt(block_sum256(part, red));
  __syncthreads();
  if (m >= 2) jacobi_core(A, Uw, m, rel, rot, flag, fro);
  __syncthreads();
  // sort descending (stable by index)
  for (int j = tid; j < d; j += blockDim.x) {
    const double lj = A[j + j * m].x;
    int pos = 0;
    for (int i = 0; i < d; ++i) {
      const double li = A[i + i * m].x;
      pos += (li > lj) || (li == lj && i < j);
    }
    lam[pos] = lj;
    for (int r = 0; r < d; ++r) Uout[r + (int64_t)pos * ldu] = Uw[r + j * m];
  }
  __syncthreads();
}

constexpr int JLDS = 64;  // matrices up to 64 x 64 are diagonalised in LDS

__global__ void __launch_bounds__(256) k_jacobi(const int32_t* dims, const int64_t* goff, double2* G,
                                                const int64_t* uoff, double2* U, const int64_t* loff,
                                                double* lam, int rel, double2* scratch, const int64_t* soff) {
  __shared__ double2 sA[JLDS * JLDS];
  __shared__ double2 sU[JLDS * JLDS];
  __shared__ Rot rot[JLDS];
  __shared__ int flag;
  __shared__ double red[4];
  const int p = blockIdx.x;
  const int d = dims[p];
  if (d <= 0) return;
  double2 *A = sA, *Uw = sU;
  if (d > JLDS) {
    A = scratch + soff[p];
    Uw = A + (int64_t)(d + 1) * (d + 1);
  }
  Rot* rp = rot;
  // rotations for m/2 pairs: for m > 64 reuse the LDS slot budget (m/2 <= 128 needs 128 entries)
  __shared__ Rot rot_big[128];
  if (d > JLDS) rp = rot_big;
  jacobi_solve(G + goff[p], d, d, A, Uw, lam + loff[p], U + uoff[p], d, rel, rp, &flag, red);
}

void launch_jacobi(int nprob, const int32_t* dims, const int64_t* goff, double2* G, const int64_t* uoff,
                   double2* U, const int64_t* loff, double* lam, int rel, double2* scratch,
                   const int64_t* soff, hipStream_t st) {
  if (nprob <= 0) return;
  hipLaunchKernelGGL(k_jacobi, dim3(nprob), dim3(256), 0, st, dims, goff, G, uoff, U, loff, lam, rel, scratch,
                     soff);
}

// ===========================================================================
// Factorization level kernels
// ===========================================================================
__device__ __forceinline__ int dim_before(const LevelView& v, int a, int c) {
  return v.colour[a] < c ? v.kt[a] : v.n[a];
}
__device__ __forceinline__ int dim_after(const LevelView& v, int a, int c) {
  return v.colour[a] <= c ? v.kt[a] : v.n[a];
}

// B_perp: orthonormal complement of the basis B (n x k) through Householder QR.
__global__ void __launch_bounds__(256) k_householder_perp(LevelView v) {
  __shared__ double2 sA[64 * 64];
  __shared__ double2 tau[STEP0_DMAX];
  __shared__ double red[4];
  const int i = blockIdx.x;
  const int n = v.n[i], k = v.k[i], d = n - k;
  if (n == 0 || d == 0) return;
  double2* E = v.Bp + v.bp_off[i];  // n x d output
  double2* A = (n <= 64) ? sA : v.W + v.w_off[i];  // working copy of B (n x k)
  const double2* B = v.B + v.b_off[i];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  for (int e = tid; e < n * k; e += blockDim.x) A[e] = B[e];
  for (int e = tid; e < n * d; e += blockDim.x) {
    const int r = e % n, c = e / n;
    E[e] = make_double2(r == k + c ? 1.0 : 0.0, 0.0);
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    double part = 0.0;
    for (int r = j + 1 + tid; r < n; r += blockDim.x) part += cabs2(A[r + j * n]);
    const double sigma = block_sum256(part, red);
    const double2 alpha = A[j + j * n];
    double2 t = make_double2(0, 0);
    if (sigma > 0.0 || alpha.y != 0.0) {
      const double beta = -copysign(sqrt(cabs2(alpha) + sigma), alpha.x);
      t = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
      // scale = 1 / (alpha - beta)
      const double2 den = make_double2(alpha.x - beta, alpha.y);
      const double dd = cabs2(den);
      const double2 sc = make_double2(den.x / dd, -den.y / dd);
      __syncthreads();
      for (int r = j + 1 + tid; r < n; r += blockDim.x) A[r + j * n] = cmul(A[r + j * n], sc);
      if (tid == 0) A[j + j * n] = make_double2(beta, 0.0);
    }
    if (tid == 0) tau[j] = t;
    __syncthreads();
    // apply H^H = I - conj(tau) v v^H to the trailing columns
    if (t.x != 0.0 || t.y != 0.0) {
      for (int c = j + 1 + wv; c < k; c += 4) {
        double2 w = make_double2(0, 0);
        for (int r = j + lane; r < n; r += 64) {
          const double2 vr = (r == j) ? make_double2(1, 0) : A[r + j * n];
          w = cadd(w, cmulc(vr, A[r + c * n]));
        }
        w.x = wave_sum(w.x);
        w.y = wave_sum(w.y);
        const double2 f = cmul(cconj(t), w);
        for (int r = j + lane; r < n; r += 64) {
          const double2 vr = (r == j) ? make_double2(1, 0) : A[r + j * n];
          A[r + c * n] = csub(A[r + c * n], cmul(vr, f));
        }
      }
    }
    __syncthreads();
  }
  // E <- H_0 ... H_{k-1} [0; I]
  for (int j = k - 1; j >= 0; --j) {
    const double2 t = tau[j];
    if (t.x == 0.0 && t.y == 0.0) continue;
    for (int c = wv; c < d; c += 4) {
      double2 w = make_double2(0, 0);
      for (int r = j + lane; r < n; r += 64) {
        const double2 vr = (r == j) ? make_double2(1, 0) : A[r + j * n];
        w = cadd(w, cmulc(vr, E[r + c * n]));
      }
      w.x = wave_sum(w.x);
      w.y = wave_sum(w.y);
      const double2 f = cmul(t, w);
      for (int r = j + lane; r < n; r += 64) {
        const double2 vr = (r == j) ? make_double2(1, 0) : A[r + j * n];
        E[r + c * n] = csub(E[r + c * n], cmul(vr, f));
      }
    }
    __syncthreads();
  }
}

void launch_householder_perp(const LevelView& v, int nc, hipStream_t st) {
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_householder_perp, dim3(nc), dim3(256), 0, st, v);
}

// Step 0 Gram of the fill-ins in block row i: H_i = sum_b F_ib F_ib^H, split over
// GRAM_SPLIT partial sums (partner j goes to part j % GRAM_SPLIT) that
// k_gram_fill_reduce adds in a fixed order.  Partial j of colour cluster x sits at
// part + j * pstride + x * (64 tiles)^2.  grid: (cluster, tiles^2, part).  The
// partners of a part form one K stream with the next slab always in flight, and
// the tile's 16 x 16 output blocks are dealt evenly to the four wavefronts.  H_i
// is Hermitian, so only the blocks on or above the block diagonal are formed and
// the reduction writes their conjugate transposes below it.
constexpr int GRAM_RED_BLOCKS = 32;

struct GramTerm {
  const double2* A;
  const double2* B;
  int64_t lda, ldb;
  int opA, opB, K;
};

__device__ __forceinline__ bool gram_term(const LevelView& v, const ColourTasks& c, int i, int j, int tr, int tc,
                                          GramTerm& t) {
  const int b = v.fp_cl[j];
  const int code = v.fp_srow[j];
  t.K = dim_before(v, b, c.colour);
  if (t.K <= 0) return false;
  if (code >= 0) {  // F_ib stored as (i, b): n x m_b, ld n
    const int n = v.n[i];
    const double2* F = v.slots + v.slot_off[code];
    t.A = F + tr * 64;
    t.B = F + tc * 64;
    t.lda = t.ldb = n;
    t.opA = OP_N;
    t.opB = OP_C;
  } else {  // stored as (b, i): F_ib = S^T with S m_b x n, ld n_b
    const int nb = v.n[b];
    const double2* Sb = v.slots + v.slot_off[~code];
    t.A = Sb + (int64_t)tr * 64 * nb;
    t.B = Sb + (int64_t)tc * 64 * nb;
    t.lda = t.ldb = nb;
    t.opA = OP_T;
    t.opB = OP_R;
  }
  return true;
}

// The 16 x 16 output blocks of a partial Gram tile (tr, tc), tr <= tc, that
// wavefront w forms: all mt x nt blocks off the tile diagonal, only those on or
// above the block diagonal (rb <= cb, numbered column by column) on it; dealt to
// the four wavefronts in contiguous runs.  Block j of the run: (rb[j], cb[j]),
// rb[j] < 0 past its end.
__device__ __forceinline__ void gram_blocks(bool tri, int mt, int nt, int rb[4], int cb[4]) {
  const int w = threadIdx.x >> 6;
  const int cnt = tri ? mt * (mt + 1) / 2 : mt * nt, per = (cnt + 3) >> 2, k0 = w * per;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int kb = k0 + j;
    rb[j] = -1;
    cb[j] = 0;
    if (j >= per || kb >= cnt) continue;
    if (tri) {
      int c = 0;
      while ((c + 1) * (c + 2) / 2 <= kb) ++c;
      cb[j] = c;
      rb[j] = kb - c * (c + 1) / 2;
    } else {
      rb[j] = kb % mt;
      cb[j] = kb / mt;
    }
  }
}

// acc += op(A_tile) op(B_tile) on the given blocks for the first nk k-columns of one slab.
__device__ __forceinline__ void mma_slab_blocks(const TileSmem<double>& s, TileAcc<double>& acc, int nk,
                                                const int rb[4], const int cb[4]) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int q = 0; q < TK / 4; ++q) {
    if (q * 4 >= nk) break;
    const int kk = q * 4 + lk;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (rb[j] < 0) continue;
      const double ar = s.are[kk][rb[j] * 16 + li], ai = s.aim[kk][rb[j] * 16 + li];
      const double br = s.bre[kk][cb[j] * 16 + li], bi = s.bim[kk][cb[j] * 16 + li];
      auto& re = acc.re[j >> 1][j & 1];
      auto& im = acc.im[j >> 1][j & 1];
      re = mfma16(br, ar, re);
      re = mfma16(bi, -ai, re);
      im = mfma16(br, ai, im);
      im = mfma16(bi, ar, im);
    }
  }
}

__device__ __forceinline__ void gram_fill_body(const LevelView& v, const ColourTasks& c, double2* part, int64_t pstride,
                                               const VBlock& VB) {
  __shared__ TileSmem<double> s;
  const int i = c.cl[VB.x];
  const int n = v.n[i];
  const int tr = VB.y % c.tiles, tc = VB.y / c.tiles;
  const int sp = VB.z;
  // H_i is Hermitian: only tiles on or above the diagonal, and in diagonal tiles
  // only the blocks on or above the block diagonal; the reduction mirrors the rest
  if (tr * 64 >= n || tc * 64 >= n || tr > tc) return;
  const int m = min(64, n - tr * 64), nn = min(64, n - tc * 64);
  const int mt = (m + 15) >> 4, nt = (nn + 15) >> 4;
  int rbs[4], cbs[4];
  gram_blocks(tr == tc, mt, nt, rbs, cbs);
  TileAcc<double> acc;
  acc.zero();
  const int j_end = v.fp_ptr[i + 1];
  int j = v.fp_ptr[i] + sp;
  GramTerm cur;
  while (j < j_end && !gram_term(v, c, i, j, tr, tc, cur)) j += GRAM_SPLIT;
  if (j < j_end) {
    SlabRegs<double2> regs;
    int k0 = 0;
    slab_fetch<double2>(regs, cur.A, cur.lda, cur.opA, cur.B, cur.ldb, cur.opB, m, nn, cur.K, 0);
    while (true) {
      const int nk = min(TK, cur.K - k0);
      __syncthreads();
      slab_store<double, double2>(s, regs, cur.opA, cur.opB);
      __syncthreads();
      GramTerm nxt = cur;
      int nk0 = k0 + TK;
      bool more = true;
      if (nk0 >= cur.K) {
        nk0 = 0;
        j += GRAM_SPLIT;
        while (j < j_end && !gram_term(v, c, i, j, tr, tc, nxt)) j += GRAM_SPLIT;
        more = j < j_end;
      }
      if (more) slab_fetch<double2>(regs, nxt.A, nxt.lda, nxt.opA, nxt.B, nxt.ldb, nxt.opB, m, nn, nxt.K, nk0);
      mma_slab_blocks(s, acc, nk, rbs, cbs);
      if (!more) break;
      cur = nxt;
      k0 = nk0;
    }
  }
  const int64_t cstride = (int64_t)(c.tiles * 64) * (c.tiles * 64);
  double2* P = part + (int64_t)sp * pstride + (int64_t)VB.x * cstride + tr * 64 + (int64_t)tc * 64 * n;
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (rbs[j] < 0) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = rbs[j] * 16 + (lane & 15), col = cbs[j] * 16 + acc_col<double>(lane, q);
      if (r < m && col < nn) P[r + (int64_t)col * n] = make_double2(acc.re[j >> 1][j & 1][q], acc.im[j >> 1][j & 1][q]);
    }
  }
}
__global__ void __launch_bounds__(256) k_gram_fill(LevelView v, ColourTasks c, double2* part, int64_t pstride) {
  gram_fill_body(v, c, part, pstride, vblock());
}
__global__ void __launch_bounds__(256) k_gram_fill_b(const BatchEntry* E, int ne) {
  VBlock VB;
  const EntryRef e = locate(E, ne, VB);
  gram_fill_body(e.v, e.c, e.buf, e.aux, VB);
}

// H_i = sum of the partial Grams in a fixed order (deterministic); grid (cluster,
// GRAM_RED_BLOCKS), each workgroup taking the 16 x 16 blocks on or above the block
// diagonal in turn (thread (ti, tj): row ti, column tj of the block), writing the
// block and, off the diagonal, its conjugate transpose through LDS.
__device__ __forceinline__ void gram_fill_reduce_body(const LevelView& v, const ColourTasks& c, const double2* part,
                                                      int64_t pstride, const VBlock& VB) {
  __shared__ double2 blk[16][17];
  const int i = c.cl[VB.x];
  const int n = v.n[i];
  double2* H = v.W + v.w_off[i];
  const int64_t cstride = (int64_t)(c.tiles * 64) * (c.tiles * 64);
  const double2* P0 = part + (int64_t)VB.x * cstride;
  const int nb = (n + 15) >> 4, nblk = nb * (nb + 1) / 2;
  const int ti = threadIdx.x & 15, tj = threadIdx.x >> 4;
  for (int kb = VB.y; kb < nblk; kb += VB.gy) {
    int cb = 0;
    while ((cb + 1) * (cb + 2) / 2 <= kb) ++cb;
    const int rb = kb - cb * (cb + 1) / 2;
    const int r = rb * 16 + ti, q = cb * 16 + tj;
    double2 a = make_double2(0, 0);
    if (r < n && q < n) {
      const int64_t e = r + (int64_t)q * n;
      a = P0[e];
      for (int sp = 1; sp < GRAM_SPLIT; ++sp) a = cadd(a, P0[(int64_t)sp * pstride + e]);
      H[e] = a;
    }
    if (rb != cb) {
      __syncthreads();
      blk[tj][ti] = a;
      __syncthreads();
      // entry (cb*16 + ti, rb*16 + tj) is the conjugate of (rb*16 + tj, cb*16 + ti)
      const int r2 = cb * 16 + ti, q2 = rb * 16 + tj;
      const double2 b = blk[ti][tj];
      if (r2 < n && q2 < n) H[r2 + (int64_t)q2 * n] = make_double2(b.x, -b.y);
    }
  }
}
__global__ void k_gram_fill_reduce(LevelView v, ColourTasks c, const double2* part, int64_t pstride) {
  gram_fill_reduce_body(v, c, part, pstride, vblock());
}
__global__ void k_gram_fill_reduce_b(const BatchEntry* E, int ne) {
  VBlock VB;
  const EntryRef e = locate(E, ne, VB);
  gram_fill_reduce_body(e.v, e.c, e.buf, e.aux, VB);
}

void launch_gram_fill(const LevelView& v, const ColourTasks& c, double2* part, int64_t pstride, hipStream_t st) {
  if (c.ncl <= 0) return;
  hipLaunchKernelGGL(k_gram_fill, dim3(c.ncl, c.tiles * c.tiles, GRAM_SPLIT), dim3(256), 0, st, v, c, part, pstride);
  hipLaunchKernelGGL(k_gram_fill_reduce, dim3(c.ncl, GRAM_RED_BLOCKS), dim3(256), 0, st, v, c, part, pstride);
}

// phase 0: X = H B_perp ; phase 1: G' = B_perp^H X ; phase 2: Q~[:, k:n] = B_perp U'
__device__ __forceinline__ void xform_body(const LevelView& v, const ColourTasks& c, int phase, const VBlock& VB) {
  __shared__ TileSmem<double> s;
  const int i = c.cl[VB.x];
  const int n = v.n[i], k = v.k[i], d = n - k;
  if (d <= 0) return;
  const int tr = VB.y % c.tiles, tc = VB.y / c.tiles;
  double2* W = v.W + v.w_off[i];
  const double2* H = W;
  double2* X = W + (int64_t)n * n;
  double2* Gp = X + (int64_t)n * d;
  double2* Up = Gp + (int64_t)d * d;
  const double2* Bp = v.Bp + v.bp_off[i];
  TileAcc<double> acc;
  acc.zero();
  if (phase == 0) {
    if (tr * 64 >= n || tc * 64 >= d) return;
    const int m = min(64, n - tr * 64), nn = min(64, d - tc * 64);
    gemm_tile<double, double2>(s, acc, H + tr * 64, n, OP_N, Bp + (int64_t)tc * 64 * n, n, OP_N, m, nn, n);
    store_tile<double, double2>(acc, X + tr * 64 + (int64_t)tc * 64 * n, n, m, nn, ST_SET);
  } else if (phase == 1) {
    if (tr * 64 >= d || tc * 64 >= d) return;
    const int m = min(64, d - tr * 64), nn = min(64, d - tc * 64);
    gemm_tile<double, double2>(s, acc, Bp + (int64_t)tr * 64 * n, n, OP_C, X + (int64_t)tc * 64 * n, n, OP_N, m,
                               nn, n);
    store_tile<double, double2>(acc, Gp + tr * 64 + (int64_t)tc * 64 * d, d, m, nn, ST_SET);
  } else {
    if (tr * 64 >= n || tc * 64 >= d) return;
    const int m = min(64, n - tr * 64), nn = min(64, d - tc * 64);
    gemm_tile<double, double2>(s, acc, Bp + tr * 64, n, OP_N, Up + (int64_t)tc * 64 * d, d, OP_N, m, nn, d);
    double2* Qc = v.Q + v.q_off[i] + (int64_t)k * n;
    store_tile<double, double2>(acc, Qc + tr * 64 + (int64_t)tc * 64 * n, n, m, nn, ST_SET);
  }
}
__global__ void __launch_bounds__(256) k_xform(LevelView v, ColourTasks c, int phase) { xform_body(v, c, phase, vblock()); }
__global__ void __launch_bounds__(256) k_xform_b(const BatchEntry* E, int ne) {
  VBlock VB;
  const EntryRef e = locate(E, ne, VB);
  xform_body(e.v, e.c, e.i0, VB);
}

void launch_xform(const LevelView& v, const ColourTasks& c, int phase, hipStream_t st) {
  if (c.ncl <= 0) return;
  hipLaunchKernelGGL(k_xform, dim3(c.ncl, c.tiles * c.tiles), dim3(256), 0, st, v, c, phase);
}

// ---------------------------------------------------------------------------
// Step 0 eigen-solver for clusters that gain basis vectors (p > 0):
// Householder reduction of G' to a real symmetric tridiagonal T, all
// eigenvalues by bisection on Sturm counts, the p dominant eigenvectors by
// inverse iteration on T mapped back through the reflectors and
// re-orthonormalised, and an orthonormal complement by Householder QR.
// O(d) dependent steps instead of the O(d * sweeps) rounds of cyclic Jacobi.
// ---------------------------------------------------------------------------
// Scratch per cluster (dm = the level's largest d): G' copy (dm x dm), eigenvector
// block (dm x dm), tridiagonal work (4 dm doubles per vector): 4 dm^2 complex.


// ---------------------------------------------------------------------------
// Step 0 (Section 3.2, the basis extension by the fill-ins).  One workgroup of
// S0_NT threads per cluster; G' (d x d Hermitian) is held in packed lower
// storage, in LDS up to order STEP0_PACK_LDS, else in the cluster's scratch.
// ---------------------------------------------------------------------------
constexpr int S0_NT = 1024, S0_NW = S0_NT / 64;
constexpr int STEP0_PACK_LDS = 120;
constexpr int S0_PACK = STEP0_PACK_LDS * (STEP0_PACK_LDS + 1) / 2;  // double2 slots of the LDS matrix region
static_assert(STEP0_DMAX % 64 == 0 && STEP0_DMAX <= 512, "d-vectors are spread over at most eight elements per lane");

// Packed lower storage: element (r, c), r >= c, at c d - c (c - 1) / 2 + (r - c).
__device__ __forceinline__ int pidx(int r, int c, int d) { return c * d - (c * (c - 1)) / 2 + (r - c); }

// Sum / maximum over the workgroup's wavefronts in a fixed order (the same value in every thread).
__device__ __forceinline__ double s0_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < S0_NW; ++w) s += red[w];
  __syncthreads();
  return s;
}
__device__ __forceinline__ double s0_max(double v, double* red) {  // v >= 0
  v = wave_max_nonneg(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = red[0];
#pragma unroll
  for (int w = 1; w < S0_NW; ++w) s = fmax(s, red[w]);
  __syncthreads();
  return s;
}

// Lower Householder tridiagonalization A = Q T Q^H of the Hermitian matrix in
// packed lower storage P: Q = H_0 ... H_{d-2}, H_j = I - tau_j v_j v_j^H,
// v_j = [1; P(j+2:d, j)] on rows j+1..d-1, real off-diagonal beta_j.  Every
// wavefront forms v_j in registers (element r = lane + 64 q) from the same data
// in the same order, so the scalars agree bit for bit without a barrier; the
// product tau A22 v runs a row per wavefront (lanes on columns), the rank-2
// update a column per wavefront (lanes on rows).  ws and vs are d-vectors.
template <int NQ>
__device__ void hetrd_packed(double2* P, int d, double2* tau, double* dg, double* off, double2* ws, double2* vs) {
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  int cb[NQ];  // P[cb[q] + r] = A(r, c) for the lane's columns c = lane + 64 q and r >= c
#pragma unroll
  for (int q = 0; q < NQ; ++q) cb[q] = pidx(lane + 64 * q, lane + 64 * q, d) - (lane + 64 * q);
  for (int j = 0; j + 1 < d; ++j) {
    const int cj = pidx(j, j, d) - j;  // P[cj + r] = A(r, j) for r >= j
    double2 v[NQ];
    double xn2 = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int r = lane + 64 * q;
      v[q] = (r > j + 1 && r < d) ? P[cj + r] : make_double2(0, 0);
      xn2 += cabs2(v[q]);
    }
    xn2 = wave_sum(xn2);
    const double2 alpha = P[cj + j + 1];
    double2 t = make_double2(0, 0);
    double beta = alpha.x;
    if (xn2 > 0.0 || alpha.y != 0.0) {
      beta = -copysign(sqrt(cabs2(alpha) + xn2), alpha.x);
      const double rb = 1.0 / beta;
      t = make_double2((beta - alpha.x) * rb, -alpha.y * rb);
      const double2 den = make_double2(alpha.x - beta, alpha.y);
      const double rdd = 1.0 / cabs2(den);
      const double2 sc = make_double2(den.x * rdd, -den.y * rdd);
#pragma unroll
      for (int q = 0; q < NQ; ++q) v[q] = cmul(v[q], sc);
    }
    if (tid == 0) {
      tau[j] = t;
      off[j] = beta;
    }
    if (t.x == 0.0 && t.y == 0.0) continue;  // column j is already [beta; 0]: nothing written, no barrier needed
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if (lane + 64 * q == j + 1) v[q] = make_double2(1, 0);
    if (wv == 0)
      for (int q = 0; q < NQ; ++q) {
        const int r = lane + 64 * q;
        if (r > j && r < d) vs[r] = v[q];
      }
    // ws = tau A22 v, two rows per wavefront step
    for (int r = j + 1 + wv; r < d; r += 2 * S0_NW) {
      const int r2 = r + S0_NW;
      const int cr = pidx(r, r, d) - r, cr2 = pidx(r2 < d ? r2 : r, r2 < d ? r2 : r, d) - (r2 < d ? r2 : r);
      double2 a1 = make_double2(0, 0), a2 = make_double2(0, 0);
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int c = lane + 64 * q;
        if (c > j && c < d) {
          const double2 e1 = c <= r ? P[cb[q] + r] : cconj(P[cr + c]);
          a1 = cadd(a1, cmul(e1, v[q]));
          if (r2 < d) {
            const double2 e2 = c <= r2 ? P[cb[q] + r2] : cconj(P[cr2 + c]);
            a2 = cadd(a2, cmul(e2, v[q]));
          }
        }
      }
      a1.x = wave_sum(a1.x);
      a1.y = wave_sum(a1.y);
      a2.x = wave_sum(a2.x);
      a2.y = wave_sum(a2.y);
      if (lane == 0) {
        ws[r] = cmul(t, a1);
        if (r2 < d) ws[r2] = cmul(t, a2);
      }
    }
    __syncthreads();
    // w = ws - (Re(conj(tau) v^H ws) / 2) v, each wavefront for its own lanes
    double2 w[NQ];
    double pr = 0.0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int r = lane + 64 * q;
      w[q] = (r > j && r < d) ? ws[r] : make_double2(0, 0);
      const double2 z = cmulc(v[q], w[q]);
      pr += z.x * t.x + z.y * t.y;
    }
    const double hc = 0.5 * wave_sum(pr);
#pragma unroll
    for (int q = 0; q < NQ; ++q) w[q] = csub(w[q], make_double2(hc * v[q].x, hc * v[q].y));
    if (wv == 0) {
      for (int q = 0; q < NQ; ++q) {
        const int r = lane + 64 * q;
        if (r > j + 1 && r < d) P[cj + r] = v[q];
      }
      if (lane == 0) P[cj + j + 1] = make_double2(beta, 0.0);
    }
    // A22 -= w v^H + v w^H on the lower triangle, a column per wavefront
    for (int c = j + 1 + wv; c < d; c += S0_NW) {
      const double2 vc = vs[c], wsc = ws[c];
      const double2 wc = csub(wsc, make_double2(hc * vc.x, hc * vc.y));
      const int cc = pidx(c, c, d) - c;
#pragma unroll
      for (int q = 0; q < NQ; ++q) {
        const int r = lane + 64 * q;
        if (r >= c && r < d)
          P[cc + r] = csub(P[cc + r], cadd(cmul(w[q], cconj(vc)), cmul(v[q], cconj(wc))));
      }
    }
    __syncthreads();
  }
  for (int j = tid; j < d; j += blockDim.x) dg[j] = P[pidx(j, j, d)].x;
  __syncthreads();
}

// number of eigenvalues of T below sigma (Sturm count of the LDL^T pivots)
__device__ int sturm_count(const double* __restrict__ dg, const double* __restrict__ off, int d, double sigma,
                           double pivmin) {
  int cnt = 0;
  double q = dg[0] - sigma;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0) ++cnt;
#pragma unroll 4
  for (int i = 1; i < d; ++i) {
    q = (dg[i] - sigma) - off[i - 1] * off[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0) ++cnt;
  }
  return cnt;
}

// The same count without divisions, for a T scaled to norm <= 1 (diagonal dn,
// squared off-diagonal e2): sign changes of the leading principal minors
// p_i = (dn_i - x) p_{i-1} - e2_{i-1} p_{i-2}, kept in range by exact
// power-of-two rescaling.  A zero minor is replaced by -2^-200 times its
// predecessor (a tiny negative pivot, the limit the LDL^T count takes), so every
// minor is nonzero and a sign change is the xor of the two sign bits.  Branch-free.
__device__ int sturm_count_minors(const double* __restrict__ dn, const double* __restrict__ e2, int d, double x) {
  double p0 = 1.0, p1 = dn[0] - x;
  p1 = (p1 == 0.0) ? -0x1p-200 : p1;
  unsigned cnt = (unsigned)__double2hiint(p1) >> 31;
  auto step = [&](double dd, double ee) {
    double p2 = (dd - x) * p1 - ee * p0;
    p2 = (p2 == 0.0) ? -0x1p-200 * p1 : p2;
    cnt += (unsigned)(__double2hiint(p2) ^ __double2hiint(p1)) >> 31;
    p0 = p1;
    p1 = p2;
  };
  int i = 1;
  // four steps per round with their operands loaded up front; |p| grows at most
  // four-fold per step (|dn - x| <= 2, e2 <= 1), so one range check per round suffices
  for (; i + 3 < d; i += 4) {
    const double d0 = dn[i], d1 = dn[i + 1], d2 = dn[i + 2], d3 = dn[i + 3];
    const double f0 = e2[i - 1], f1 = e2[i], f2 = e2[i + 1], f3 = e2[i + 2];
    step(d0, f0);
    step(d1, f1);
    step(d2, f2);
    step(d3, f3);
    const double m = fmax(fabs(p0), fabs(p1));
    const double sc = m > 0x1p256 ? 0x1p-512 : (m < 0x1p-256 ? 0x1p512 : 1.0);
    p0 *= sc;
    p1 *= sc;
  }
  for (; i < d; ++i) step(dn[i], e2[i - 1]);
  return (int)cnt;
}

// Eigenvalues of the scaled tridiagonal (dn, e2, spectrum inside [glo, ghi])
// with ascending indices ks[0..cnt), out[t] for target t.  Multisection: a group
// of G probes brackets one eigenvalue, each probe one Sturm count per round, so a
// round narrows the bracket G + 1 fold; stops at a bracket of a few units in the
// last place of the eigenvalue or of the norm.  Up to S0_NW targets, a group is
// W whole wavefronts (W the largest power of two with W cnt <= S0_NW), combined
// through firstge[2 S0_NW] in LDS; beyond that, groups of G lanes of one wavefront.
// Every thread of the workgroup calls this.
__device__ void tri_eig_targets(const double* dn, const double* e2, int d, double glo, double ghi, const int* ks,
                                int cnt, double* out, int* firstge) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double lo0 = glo - 2.2e-16 * fabs(glo) - 0x1p-60, hi0 = ghi + 2.2e-16 * fabs(ghi) + 0x1p-60;
  if (cnt <= S0_NW) {
    int W = S0_NW;
    while (W * cnt > S0_NW) W >>= 1;
    const int G = 64 * W, t = wv / W, m = (wv % W) * 64 + lane;
    const int k = t < cnt ? ks[t] : 0;
    const double rg = 1.0 / (double)(G + 1), fm = (double)(m + 1) * rg;
    double lo = lo0, hi = hi0;
    bool done = t >= cnt;
    for (;;) {
      const bool ge = !done && sturm_count_minors(dn, e2, d, lo + (hi - lo) * fm) >= k + 1;
      const unsigned long long mask = __ballot(ge);
      if (lane == 0) firstge[wv] = mask ? (wv % W) * 64 + __ffsll((long long)mask) - 1 : G;
      __syncthreads();
      if (!done) {
        int f = G;
        for (int u = 0; u < W; ++u) f = min(f, firstge[t * W + u]);
        const double w = hi - lo;
        const double nlo = f > 0 ? lo + w * ((double)f * rg) : lo;   // probe f - 1, or lo
        const double nhi = f < G ? lo + w * ((double)(f + 1) * rg) : hi;
        if ((nlo == lo && nhi == hi) || !(nhi > nlo)) done = true;
        lo = nlo;
        hi = nhi;
        if (hi - lo <= 4.4e-16 * fmax(fabs(lo), fabs(hi)) + 0x1p-52) done = true;
      }
      if (lane == 0) firstge[S0_NW + wv] = done;
      __syncthreads();
      bool all = true;
      for (int u = 0; u < S0_NW; ++u) all = all && firstge[S0_NW + u];
      if (all) break;
    }
    if (t < cnt && m == 0) out[t] = 0.5 * (lo + hi);
    __syncthreads();
    return;
  }
  int G = 64;
  while (G > 1 && (int)(blockDim.x / G) < cnt) G >>= 1;
  const int ngroups = blockDim.x / G;
  const int gid = threadIdx.x / G, m = threadIdx.x % G;
  const int gbase = (lane / G) * G;
  const unsigned long long gmask = (G == 64) ? ~0ull : ((1ull << G) - 1ull);
  for (int t0 = 0; t0 < cnt; t0 += ngroups) {
    const int t = t0 + gid;
    const int k = t < cnt ? ks[t] : 0;
    double lo = lo0, hi = hi0;
    bool done = t >= cnt;
    while (__ballot(!done) != 0ull) {
      const double x = lo + (hi - lo) * (double)(m + 1) / (double)(G + 1);
      const bool ge = !done && sturm_count_minors(dn, e2, d, x) >= k + 1;
      const unsigned long long mask = (__ballot(ge) >> gbase) & gmask;
      if (!done) {
        double nlo, nhi;
        if (mask) {
          const int f = __ffsll((long long)mask) - 1;
          nhi = lo + (hi - lo) * (double)(f + 1) / (double)(G + 1);
          nlo = f > 0 ? lo + (hi - lo) * (double)f / (double)(G + 1) : lo;
        } else {
          nlo = lo + (hi - lo) * (double)G / (double)(G + 1);
          nhi = hi;
        }
        if ((nlo == lo && nhi == hi) || !(nhi > nlo)) done = true;
        lo = nlo;
        hi = nhi;
        if (hi - lo <= 4.4e-16 * fmax(fabs(lo), fabs(hi)) + 0x1p-52) done = true;
      }
    }
    if (t < cnt && m == 0) out[t] = 0.5 * (lo + hi);
  }
  __syncthreads();
}

// Inverse iteration for one eigenvector of T (dg, off) with shift lam: T - lam I
// = P L U with partial pivoting once, then three solves from a fixed start
// vector (each normalised; the scale is folded into the next forward pass), the
// result written to y (length d).  The factors live in six interleaved arrays of
// the caller's work area, element i of array a at W[(a d + i) nb], so that
// neighbouring threads (vectors) touch neighbouring words; the recurrences run in
// registers with the next operands loaded a step ahead.
__device__ void tri_inverse_iteration(const double* __restrict__ dg, const double* __restrict__ off, int d,
                                      double lam, double pivmin, int seed, double* __restrict__ W, int nb,
                                      double2* __restrict__ y) {
  double* rD = W;
  double* DU = W + (size_t)d * nb;
  double* DU2 = DU + (size_t)d * nb;
  double* F = DU2 + (size_t)d * nb;
  double* S = F + (size_t)d * nb;
  double* b = S + (size_t)d * nb;
  // factorization
  double cd = dg[0] - lam, cdu = d > 1 ? off[0] : 0.0;
#pragma unroll 4
  for (int i = 0; i + 1 < d; ++i) {
    const double sub = off[i], nd = dg[i + 1] - lam, ndu = (i + 2 < d) ? off[i + 1] : 0.0;
    const size_t o = (size_t)i * nb;
    if (fabs(cd) >= fabs(sub)) {
      if (fabs(cd) < pivmin) cd = cd >= 0 ? pivmin : -pivmin;
      const double f = sub / cd;
      rD[o] = 1.0 / cd;
      DU[o] = cdu;
      DU2[o] = 0.0;
      F[o] = f;
      S[o] = 0.0;
      cd = nd - f * cdu;
      cdu = ndu;
    } else {
      const double f = cd / sub;
      rD[o] = 1.0 / sub;
      DU[o] = nd;
      DU2[o] = ndu;
      F[o] = f;
      S[o] = 1.0;
      cd = cdu - f * nd;
      cdu = -f * ndu;
    }
  }
  if (fabs(cd) < pivmin) cd = cd >= 0 ? pivmin : -pivmin;
  rD[(size_t)(d - 1) * nb] = 1.0 / cd;
  double scale = 1.0;
  for (int it = 0; it < 3; ++it) {
    // forward: b <- L^-1 P^T (scale b)
    auto start = [&](int r) { return 1.0 + 0.37 * (double)((r * (seed + 3) + 7 * seed) % 11) / 11.0; };
    double cur = it == 0 ? start(0) : b[0] * scale;
    double nxt = d > 1 ? (it == 0 ? start(1) : b[nb] * scale) : 0.0;
#pragma unroll 4
    for (int i = 0; i + 1 < d; ++i) {
      const size_t o = (size_t)i * nb;
      const double f = F[o];
      const bool sw = S[o] != 0.0;
      const double after = (i + 2 < d) ? (it == 0 ? start(i + 2) : b[o + 2 * (size_t)nb] * scale) : 0.0;
      if (!sw) {
        b[o] = cur;
        cur = nxt - f * cur;
      } else {
        b[o] = nxt;
        cur = cur - f * nxt;
      }
      nxt = after;
    }
    // backward: U x = b
    double x1 = cur * rD[(size_t)(d - 1) * nb], x2 = 0.0;
    b[(size_t)(d - 1) * nb] = x1;
    double nrm = x1 * x1;
#pragma unroll 4
    for (int i = d - 2; i >= 0; --i) {
      const size_t o = (size_t)i * nb;
      const double xi = (b[o] - DU[o] * x1 - DU2[o] * x2) * rD[o];
      b[o] = xi;
      nrm += xi * xi;
      x2 = x1;
      x1 = xi;
    }
    scale = 1.0 / sqrt(nrm);
  }
  for (int i = 0; i < d; ++i) y[i] = make_double2(b[(size_t)i * nb] * scale, 0.0);
}

template <int NQ>
__device__ __forceinline__ void step0_eig_body(const LevelView& v, const ColourTasks& c, double2* scratch, int dm,
                                               const VBlock& VB) {
  __shared__ double2 sP[S0_PACK];
  __shared__ double2 ws[STEP0_DMAX], vs[STEP0_DMAX], tauv[STEP0_DMAX];
  __shared__ double dg[STEP0_DMAX], off[STEP0_DMAX], eig[STEP0_DMAX];
  __shared__ int ks[STEP0_DMAX];
  __shared__ int firstge[2 * S0_NW];
  __shared__ double red[S0_NW];
  __shared__ double bounds[4];
  __shared__ int s_p;
  const int64_t stride = 4 * (int64_t)dm * dm;
  const int i = c.cl[VB.x];
  const int n = v.n[i], k = v.k[i], d = n - k;
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  double2* Q = v.Q + v.q_off[i];
  const double2* B = v.B + v.b_off[i];
  for (int e = tid; e < n * k; e += blockDim.x) Q[e] = B[e];
  int p = 0;
  if (d > 0) {
    double2* W = v.W + v.w_off[i];
    double2* Gp = W + (int64_t)n * n + (int64_t)n * d;
    double2* Up = Gp + (int64_t)d * d;
    double2* scr = scratch + (int64_t)VB.x * stride;
    double2* A = (d <= STEP0_PACK_LDS) ? sP : scr;  // packed lower working matrix
    // p = 0 exactly when every eigenvalue of G' is below tau0^2 = (eps_fill nu)^2 (then
    // sigma_1(W) < eps_fill nu < nu and the threshold tau = eps_fill max(nu, sigma_1) = tau0).
    // G' is positive semidefinite, so a diagonal entry >= tau0^2 rules this out and
    // ||G'||_F < tau0^2 proves it; otherwise an LDL^H factorization of tau0^2 I - G'
    // decides (positive pivots iff positive definite).  Any orthonormal complement then
    // serves as B~perp: U' = I.
    const double tau0 = v.eps_fill * v.nu[i];
    const double t02 = tau0 * tau0;
    const bool forced = v.forced && v.forced[i] >= 0;
    bool skip;
    if (forced) {
      skip = v.forced[i] - k <= 0;
    } else {
      double fro = 0.0, gmax = 0.0;
      for (int e = tid; e < d * d; e += blockDim.x) {
        const double2 gv = Gp[e];
        fro += cabs2(gv);
        if (e % d == e / d) gmax = fmax(gmax, gv.x);
      }
      fro = s0_sum(fro, red);
      gmax = s0_max(gmax, red);
      if (!(tau0 > 0.0) || gmax >= t02) {
        skip = false;
      } else if (fro < t02 * t02) {
        skip = true;
      } else {
        for (int e = tid; e < d * d; e += blockDim.x) {
          const int r = e % d, q = e / d;
          if (r < q) continue;
          const double2 gv = Gp[e];
          A[pidx(r, q, d)] = (r == q) ? make_double2(t02 - gv.x, 0.0) : make_double2(-gv.x, -gv.y);
        }
        __syncthreads();
        skip = true;
        for (int j = 0; j < d; ++j) {
          const double piv = A[pidx(j, j, d)].x;
          if (!(piv > 0.0)) {
            skip = false;
            break;
          }
          const double rp = 1.0 / piv;
          const int cj = pidx(j, j, d) - j;
          for (int q = j + 1 + wv; q < d; q += S0_NW) {
            const double2 lq = cconj(A[cj + q]);
            const double2 mq = make_double2(lq.x * rp, lq.y * rp);
            const int cq = pidx(q, q, d) - q;
            for (int r = q + lane; r < d; r += 64) A[cq + r] = csub(A[cq + r], cmul(A[cj + r], mq));
          }
          __syncthreads();
        }
      }
      __syncthreads();
    }
    if (skip) {
      for (int e = tid; e < d * d; e += blockDim.x) Up[e] = make_double2((e % d) == (e / d) ? 1.0 : 0.0, 0.0);
      if (tid == 0 && v.margins) {
        v.margins[2 * i] = 1e300;
        v.margins[2 * i + 1] = -1.0;  // sigma_1 / tau < 1, not evaluated
      }
    } else {
      for (int e = tid; e < d * d; e += blockDim.x) {
        const int r = e % d, q = e / d;
        if (r >= q) A[pidx(r, q, d)] = Gp[e];
      }
      __syncthreads();
      hetrd_packed<NQ>(A, d, tauv, dg, off, ws, vs);
      // Gershgorin interval, pivot floor and the power-of-two scale of T
      if (tid == 0) {
        double lo = 1e300, hi = -1e300, emax = 0.0;
        for (int r = 0; r < d; ++r) {
          const double rad = (r > 0 ? fabs(off[r - 1]) : 0.0) + (r + 1 < d ? fabs(off[r]) : 0.0);
          lo = fmin(lo, dg[r] - rad);
          hi = fmax(hi, dg[r] + rad);
          if (r + 1 < d) emax = fmax(emax, off[r] * off[r]);
        }
        bounds[0] = lo;
        bounds[1] = hi;
        bounds[2] = fmax(emax, 1.0) * 2.2250738585072014e-308 / 2.2e-16;  // pivmin
        int ex;
        frexp(fmax(fmax(fabs(lo), fabs(hi)), 1e-300), &ex);
        bounds[3] = ldexp(1.0, -ex);  // 1 / 2^ex with 2^ex >= max(|lo|, |hi|)
      }
      __syncthreads();
      const double glo = bounds[0], ghi = bounds[1], pivmin = bounds[2], sinv = bounds[3];
      double* dn = (double*)ws;  // scaled diagonal and squared off-diagonal
      double* e2 = dn + STEP0_DMAX;
      for (int r = tid; r < d; r += blockDim.x) {
        dn[r] = dg[r] * sinv;
        const double o = (r + 1 < d) ? off[r] * sinv : 0.0;
        e2[r] = o * o;
      }
      if (tid == 0) ks[0] = d - 1;
      __syncthreads();
      // the largest eigenvalue matters only above nu^2 (tau = eps_fill max(nu, sigma_1)):
      // one Sturm count at nu^2 (or the Gershgorin bound) settles that first; then the
      // rank decision against tau^2 by one Sturm count
      const double nu2s = v.nu[i] * v.nu[i] * sinv;
      const bool below_nu = nu2s > ghi * sinv || sturm_count_minors(dn, e2, d, nu2s) == d;
      double s1 = 0.0;
      if (!below_nu) {
        tri_eig_targets(dn, e2, d, glo * sinv, ghi * sinv, ks, 1, eig, firstge);
        s1 = sqrt(fmax(eig[0] / sinv, 0.0));
      }
      const double tau = v.eps_fill * fmax(v.nu[i], s1);
      if (tid == 0) {
        int pp = (tau > 0.0) ? d - sturm_count(dg, off, d, tau * tau, pivmin) : 0;
        if (forced) pp = min(max(v.forced[i] - k, 0), d);
        s_p = pp;
      }
      __syncthreads();
      p = s_p;
      // the p largest eigenvalues (and the next one, for the margin), descending
      const int ne = min(p + 1, d);
      for (int j = tid; j < ne; j += blockDim.x) ks[j] = d - 1 - j;
      __syncthreads();
      tri_eig_targets(dn, e2, d, glo * sinv, ghi * sinv, ks, ne, eig, firstge);
      for (int j = tid; j < ne; j += blockDim.x) eig[j] /= sinv;
      __syncthreads();
      if (tid == 0 && v.margins) {
        v.margins[2 * i] = (tau > 0 && p > 0) ? sqrt(fmax(eig[p - 1], 0.0)) / tau : 1e300;
        v.margins[2 * i + 1] = (tau > 0 && p < d) ? sqrt(fmax(eig[p], 0.0)) / tau : 0.0;
      }
      // eigenvector block X (d x p, ld d) and the inverse-iteration work area: in LDS
      // behind the packed matrix when they fit, else in the cluster's scratch
      const int used = (d <= STEP0_PACK_LDS) ? d * (d + 1) / 2 : 0;
      const int tail = S0_PACK - used;
      double2* X;
      double* work;
      int nb;
      if (d * p + 3 * d * min(p, 4) <= tail) {
        X = sP + used;
        work = (double*)(X + d * p);
        nb = min(p, (tail - d * p) / (3 * d));
      } else {
        X = scr + (int64_t)dm * dm;
        work = (double*)(scr + 2 * (int64_t)dm * dm);
        nb = min(p, (int)((4 * (int64_t)dm * dm) / (6 * (int64_t)d)));
      }
      nb = max(1, min(nb, (int)blockDim.x));
      // inverse iteration for the p dominant eigenvectors of T (one thread per vector)
      const double tnorm = fmax(fabs(glo), fabs(ghi));
      for (int j0 = 0; j0 < p; j0 += nb) {
        const int j = j0 + tid;
        if (tid < nb && j < p)
          tri_inverse_iteration(dg, off, d, eig[j] + 4.4e-16 * tnorm * (1 + j % 3), fmax(pivmin, 2.2e-16 * tnorm), j,
                                work + tid, nb, X + (int64_t)j * d);
        __syncthreads();
      }
      // x = H_0 ... H_{d-2} y, one vector per wavefront, held in registers
      for (int cidx = wv; cidx < p; cidx += S0_NW) {
        double2* x = X + (int64_t)cidx * d;
        double2 xr[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int r = lane + 64 * q;
          xr[q] = (r < d) ? x[r] : make_double2(0, 0);
        }
        for (int j = d - 2; j >= 0; --j) {
          const double2 t = tauv[j];
          if (t.x == 0.0 && t.y == 0.0) continue;
          const int cj = pidx(j, j, d) - j;
          double2 vr[NQ];
          double2 s = make_double2(0, 0);
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const int r = lane + 64 * q;
            vr[q] = (r > j && r < d) ? (r == j + 1 ? make_double2(1, 0) : A[cj + r]) : make_double2(0, 0);
            s = cadd(s, cmulc(vr[q], xr[q]));
          }
          s.x = wave_sum(s.x);
          s.y = wave_sum(s.y);
          const double2 f = cmul(t, s);
#pragma unroll
          for (int q = 0; q < NQ; ++q) xr[q] = csub(xr[q], cmul(vr[q], f));
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int r = lane + 64 * q;
          if (r < d) x[r] = xr[q];
        }
      }
      __syncthreads();
      // U' = [orthonormal basis of span(X), its complement] = H'_0 ... H'_{p-1} from a
      // Householder QR of X.  QR: every wavefront forms the reflector in registers,
      // the owners update the later columns, one barrier per column.
      for (int j = 0; j < p; ++j) {
        double2* xj = X + (int64_t)j * d;
        double2 vr[NQ];
        double sg = 0.0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int r = lane + 64 * q;
          vr[q] = (r > j && r < d) ? xj[r] : make_double2(0, 0);
          sg += cabs2(vr[q]);
        }
        sg = wave_sum(sg);
        const double2 alpha = xj[j];
        double2 t = make_double2(0, 0);
        double beta = alpha.x;
        if (sg > 0.0 || alpha.y != 0.0) {
          beta = -copysign(sqrt(cabs2(alpha) + sg), alpha.x);
          t = make_double2((beta - alpha.x) / beta, -alpha.y / beta);
          const double2 den = make_double2(alpha.x - beta, alpha.y);
          const double dd = cabs2(den);
          const double2 sc = make_double2(den.x / dd, -den.y / dd);
#pragma unroll
          for (int q = 0; q < NQ; ++q) vr[q] = cmul(vr[q], sc);
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q)
          if (lane + 64 * q == j) vr[q] = make_double2(1, 0);
        if (t.x != 0.0 || t.y != 0.0) {
          for (int cc = j + 1 + wv; cc < p; cc += S0_NW) {
            double2* xc = X + (int64_t)cc * d;
            double2 s = make_double2(0, 0);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              const int r = lane + 64 * q;
              if (r >= j && r < d) s = cadd(s, cmulc(vr[q], xc[r]));
            }
            s.x = wave_sum(s.x);
            s.y = wave_sum(s.y);
            const double2 f = cmul(cconj(t), s);
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
              const int r = lane + 64 * q;
              if (r >= j && r < d) xc[r] = csub(xc[r], cmul(vr[q], f));
            }
          }
        }
        __syncthreads();
        if (wv == 0) {
          for (int q = 0; q < NQ; ++q) {
            const int r = lane + 64 * q;
            if (r > j && r < d) xj[r] = vr[q];
          }
          if (lane == 0) {
            xj[j] = make_double2(beta, 0.0);
            tauv[j] = t;
          }
        }
      }
      __syncthreads();
      // columns of E = H'_0 ... H'_{p-1}, one per wavefront in registers
      for (int cc = wv; cc < d; cc += S0_NW) {
        double2 er[NQ];
#pragma unroll
        for (int q = 0; q < NQ; ++q) er[q] = make_double2(lane + 64 * q == cc ? 1.0 : 0.0, 0.0);
        for (int j = min(cc, p - 1); j >= 0; --j) {
          const double2 t = tauv[j];
          if (t.x == 0.0 && t.y == 0.0) continue;
          const double2* xj = X + (int64_t)j * d;
          double2 vr[NQ];
          double2 s = make_double2(0, 0);
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            const int r = lane + 64 * q;
            vr[q] = (r >= j && r < d) ? (r == j ? make_double2(1, 0) : xj[r]) : make_double2(0, 0);
            s = cadd(s, cmulc(vr[q], er[q]));
          }
          s.x = wave_sum(s.x);
          s.y = wave_sum(s.y);
          const double2 f = cmul(t, s);
#pragma unroll
          for (int q = 0; q < NQ; ++q) er[q] = csub(er[q], cmul(vr[q], f));
        }
        double2* uc = Up + (int64_t)cc * d;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int r = lane + 64 * q;
          if (r < d) uc[r] = er[q];
        }
      }
    }
  }
  if (v.forced && v.forced[i] >= 0) p = min(max(v.forced[i] - k, 0), d);
  if (tid == 0) v.kt[i] = k + p;
}
template <int NQ>
__global__ void __launch_bounds__(S0_NT) k_step0_eig(LevelView v, ColourTasks c, double2* scratch, int dm) {
  step0_eig_body<NQ>(v, c, scratch, dm, vblock());
}
template <int NQ>
__global__ void __launch_bounds__(S0_NT) k_step0_eig_b(const BatchEntry* E, int ne) {
  VBlock VB;
  const EntryRef e = locate(E, ne, VB);
  step0_eig_body<NQ>(e.v, e.c, e.buf, e.i0, VB);
}

void launch_step0_eig(const LevelView& v, const ColourTasks& c, double2* scratch, int dm, hipStream_t st) {
  if (c.ncl <= 0) return;
  // lanes hold d-vectors in NQ registers each: the smallest of 1, 2, 4, 8 with 64 NQ >= dm
  if (dm <= 64)
    hipLaunchKernelGGL(k_step0_eig<1>, dim3(c.ncl), dim3(S0_NT), 0, st, v, c, scratch, dm);
  else if (dm <= 128)
    hipLaunchKernelGGL(k_step0_eig<2>, dim3(c.ncl), dim3(S0_NT), 0, st, v, c, scratch, dm);
  else if (dm <= 256)
    hipLaunchKernelGGL(k_step0_eig<4>, dim3(c.ncl), dim3(S0_NT), 0, st, v, c, scratch, dm);
  else
    hipLaunchKernelGGL(k_step0_eig<8>, dim3(c.ncl), dim3(S0_NT), 0, st, v, c, scratch, dm);
}

// Step 2 projections.  side 0: T = (x in colour ? Q~_x^H : I) Z ; side 1: Z = T (y in colour ? conj(Q~_y) : I)
template <typename R>
__device__ __forceinline__ void proj_body(const LevelView& v, const ColourTasks& c, double2* temp, int side,
                                          TileSmem<R>& s, const VBlock& VB) {
  const int task = VB.x;
  const int sl = c.pj_slot[task];
  const int x = v.slot_a[sl], y = v.slot_b[sl];
  const bool cx = v.colour[x] == c.colour, cy = v.colour[y] == c.colour;
  const int nx = v.n[x], ny = v.n[y];
  // rows of the output: for blocks whose row cluster is eliminated now and that
  // are fill-only (not inadmissible), the eliminated rows are dropped
  const int rows_in = cx ? nx : dim_before(v, x, c.colour);
  const int cols_in = cy ? ny : dim_before(v, y, c.colour);
  double2* Z = v.slots + v.slot_off[sl];
  double2* T = temp + c.pj_toff[task];
  const int tr = VB.y % c.tiles, tc = VB.y / c.tiles;
  if (side == 0) {
    if (tr * 64 >= rows_in || tc * 64 >= cols_in) return;
    const int m = min(64, rows_in - tr * 64), nn = min(64, cols_in - tc * 64);
    if (!cx) {
      for (int e = threadIdx.x; e < m * nn; e += blockDim.x) {
        const int i = e % m, j = e / m;
        T[tr * 64 + i + (int64_t)(tc * 64 + j) * nx] = Z[tr * 64 + i + (int64_t)(tc * 64 + j) * nx];
      }
      return;
    }
    TileAcc<R> acc;
    acc.zero();
    const double2* Q = v.Q + v.q_off[x];
    gemm_tile<R, double2>(s, acc, Q + (int64_t)tr * 64 * nx, nx, OP_C, Z + (int64_t)tc * 64 * nx, nx, OP_N, m,
                               nn, nx);
    store_tile<R, double2>(acc, T + tr * 64 + (int64_t)tc * 64 * nx, nx, m, nn, ST_SET);
  } else {
    const int rows = rows_in;
    if (tr * 64 >= rows || tc * 64 >= cols_in) return;
    const int m = min(64, rows - tr * 64), nn = min(64, cols_in - tc * 64);
    if (!cy) {
      for (int e = threadIdx.x; e < m * nn; e += blockDim.x) {
        const int i = e % m, j = e / m;
        Z[tr * 64 + i + (int64_t)(tc * 64 + j) * nx] = T[tr * 64 + i + (int64_t)(tc * 64 + j) * nx];
      }
      return;
    }
    TileAcc<R> acc;
    acc.zero();
    const double2* Q = v.Q + v.q_off[y];
    gemm_tile<R, double2>(s, acc, T + tr * 64, nx, OP_N, Q + (int64_t)tc * 64 * ny, ny, OP_R, m, nn, ny);
    store_tile<R, double2>(acc, Z + tr * 64 + (int64_t)tc * 64 * nx, nx, m, nn, ST_SET);
  }
}

template <typename R>
__device__ __forceinline__ void proj_kernel_body(const LevelView& v, const ColourTasks& c, double2* temp, int side,
                                                 int which, const VBlock& VB) {
  __shared__ TileSmem<R> s;
  const int sl = c.pj_slot[VB.x];
  const int x = v.slot_a[sl], y = v.slot_b[sl];
  if ((which == PJ_OFFDIAG && x == y) || (which == PJ_DIAG && x != y)) return;
  proj_body<R>(v, c, temp, side, s, VB);
}
template <typename R>
__global__ void __launch_bounds__(256) k_proj(LevelView v, ColourTasks c, double2* temp, int side, int which) {
  proj_kernel_body<R>(v, c, temp, side, which, vblock());
}
__global__ void __launch_bounds__(256) k_proj_b(const BatchEntry* E, int ne) {
  VBlock VB;
  const EntryRef e = locate(E, ne, VB);
  proj_kernel_body<double>(e.v, e.c, e.buf, e.i0, PJ_ALL, VB);
}

union ProjSmem {
  TileSmem<double> d;
  TileSmem<float> f;
};

// Mixed form in one launch: diagonal blocks (the large self terms of Z) in FP64,
// the others on FP32 matrix cores.
__device__ __forceinline__ void proj_mixed_body(const LevelView& v, const ColourTasks& c, double2* temp, int side,
                                                const VBlock& VB) {
  __shared__ ProjSmem s;
  const int sl = c.pj_slot[VB.x];
  if (v.slot_a[sl] == v.slot_b[sl])
    proj_body<double>(v, c, temp, side, s.d, VB);
  else
    proj_body<float>(v, c, temp, side, s.f, VB);
}
__global__ void __launch_bounds__(256) k_proj_mixed(LevelView v, ColourTasks c, double2* temp, int side) {
  proj_mixed_body(v, c, temp, side, vblock());
}
__global__ void __launch_bounds__(256) k_proj_mixed_b(const BatchEntry* E, int ne) {
  VBlock VB;
  const EntryRef e = locate(E, ne, VB);
  proj_mixed_body(e.v, e.c, e.buf, e.i0, VB);
}

// Fused Step 2 for levels whose blocks fit one 64x64 tile: the workgroup owns the
// whole block, so Z <- Q~_x^H Z and Z <- Z conj(Q~_y) are applied in place.  Fill
// blocks keep only the k~_x kept rows of a row cluster eliminated now.
template <typename R>
__device__ __forceinline__ void proj_fused_body(const LevelView& v, const ColourTasks& c, TileSmem<R>& s,
                                                const VBlock& VB) {
  const int sl = c.pj_slot[VB.x];
  const int x = v.slot_a[sl], y = v.slot_b[sl];
  const bool cx = v.colour[x] == c.colour, cy = v.colour[y] == c.colour;
  const int nx = v.n[x], ny = v.n[y];
  const bool fill = sl >= v.nnear;
  const int rows = cx ? (fill ? v.kt[x] : nx) : dim_before(v, x, c.colour);
  const int cols_in = cy ? ny : dim_before(v, y, c.colour);
  double2* Z = v.slots + v.slot_off[sl];
  if (cx && rows > 0 && cols_in > 0) {
    TileAcc<R> acc;
    acc.zero();
    gemm_tile<R, double2>(s, acc, v.Q + v.q_off[x], nx, OP_C, Z, nx, OP_N, rows, cols_in, nx);
    store_tile<R, double2>(acc, Z, nx, rows, cols_in, ST_SET);
    __syncthreads();
  }
  if (cy && rows > 0 && ny > 0) {
    TileAcc<R> acc;
    acc.zero();
    gemm_tile<R, double2>(s, acc, Z, nx, OP_N, v.Q + v.q_off[y], ny, OP_R, rows, ny, ny);
    store_tile<R, double2>(acc, Z, nx, rows, ny, ST_SET);
  }
}

template <typename R>
__device__ __forceinline__ void proj_fused_kernel_body(const LevelView& v, const ColourTasks& c, int which,
                                                       const VBlock& VB) {
  __shared__ TileSmem<R> s;
  const int sl = c.pj_slot[VB.x];
  const int x = v.slot_a[sl], y = v.slot_b[sl];
  if ((which == PJ_OFFDIAG && x == y) || (which == PJ_DIAG && x != y)) return;
  proj_fused_body<R>(v, c, s, VB);
}
template <typename R>
__global__ void __launch_bounds__(256) k_proj_fused(LevelView v, ColourTasks c, int which) {
  proj_fused_kernel_body<R>(v, c, which, vblock());
}
__global__ void __launch_bounds__(256) k_proj_fused_b(const BatchEntry* E, int ne) {
  VBlock VB;
  const EntryRef e = locate(E, ne, VB);
  proj_fused_kernel_body<double>(e.v, e.c, PJ_ALL, VB);
}

__device__ __forceinline__ void proj_fused_mixed_body(const LevelView& v, const ColourTasks& c, const VBlock& VB) {
  __shared__ ProjSmem s;
  const int sl = c.pj_slot[VB.x];
  if (v.slot_a[sl] == v.slot_b[sl])
    proj_fused_body<double>(v, c, s.d, VB);
  else
    proj_fused_body<float>(v, c, s.f, VB);
}
__global__ void __launch_bounds__(256) k_proj_fused_mixed(LevelView v, ColourTasks c) {
  proj_fused_mixed_body(v, c, vblock());
}
__global__ void __launch_bounds__(256) k_proj_fused_mixed_b(const BatchEntry* E, int ne) {
  VBlock VB;
  const EntryRef e = locate(E, ne, VB);
  proj_fused_mixed_body(e.v, e.c, VB);
}

// The mixed form projects the off-diagonal blocks in complex FP32 and keeps the
// diagonal blocks (which hold the large self terms of Z) in FP64.
void launch_proj_fused(const LevelView& v, const ColourTasks& c, bool mixed, hipStream_t st) {
  if (c.npj <= 0) return;
  if (mixed) {
    hipLaunchKernelGGL(k_proj_fused_mixed, dim3(c.npj), dim3(256), 0, st, v, c);
  } else {
    hipLaunchKernelGGL(k_proj_fused<double>, dim3(c.npj), dim3(256), 0, st, v, c, (int)PJ_ALL);
  }
}

void launch_proj(const LevelView& v, const ColourTasks& c, double2* temp, int side, bool mixed, hipStream_t st) {
  if (c.npj <= 0) return;
  const dim3 grid(c.npj, c.tiles * c.tiles);
  if (mixed) {
    hipLaunchKernelGGL(k_proj_mixed, grid, dim3(256), 0, st, v, c, temp, side);
  } else {
    hipLaunchKernelGGL(k_proj<double>, grid, dim3(256), 0, st, v, c, temp, side, (int)PJ_ALL);
  }
}

// Step 3a: partial LU with partial pivoting of F = Z_ii[k~:n, k~:n] (eqs. 9-11),
// then explicit L^-1 P and U^-1 (ld rmax = n - k).
//
// Up to LU_REG_MAX rows the elimination runs in registers: wavefront w owns the
// columns c = w + 16 s, lane l rows l and l + 64.  Pivoting is implicit (rows
// stay where they are; each row carries its position in the row-swapped order,
// and ties in max |re| + |im| go to the lowest position, as with explicit
// swaps), so a step costs one barrier: the owner of column j picks the pivot
// and posts the multipliers, every wavefront then updates its later columns.
// The factors are then written in the swapped order to F (LDS up to
// LU_LDS_MAX rows, else the cluster's scratch), and every column of U^-1 and of
// L^-1 is formed by one wavefront by substitution in registers and stored
// straight to the outputs.
constexpr int LU_NT = 1024, LU_NW = LU_NT / 64, LU_REG_MAX = 128, LU_CPW = LU_REG_MAX / LU_NW;

// value of lane l (wavefront-uniform) of a complex register
__device__ __forceinline__ double rl(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double2 lane_read(double2 v, int l) { return make_double2(rl(v.x, l), rl(v.y, l)); }
__device__ __forceinline__ double2 pick2(const double2 (&x)[2], int q) { return q == 0 ? x[0] : x[1]; }

__device__ __forceinline__ void lu_reg_body(const LevelView& v, const ColourTasks& c, double2* scratch, int rm,
                                            const VBlock& VB) {
  __shared__ double2 sF[LU_LDS_MAX * LU_LDS_MAX];
  __shared__ double2 lbuf[2][LU_REG_MAX];
  __shared__ double2 dinv[LU_REG_MAX];
  __shared__ int pivrow[LU_REG_MAX], pjpos[LU_REG_MAX];
  __shared__ int s_fail;
  const int i = c.cl[VB.x];
  const int n = v.n[i], kt = v.kt[i], r = n - kt, rmax = n - v.k[i];
  if (r <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const double2* Z = v.slots + v.slot_off[v.diag_slot[i]];
  double2* F = (r <= LU_LDS_MAX) ? sF : scratch + (int64_t)VB.x * ((int64_t)rm * rm + rm);
  double2 col[LU_CPW][2];
  int pos[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) pos[q] = lane + 64 * q;
#pragma unroll
  for (int s = 0; s < LU_CPW; ++s) {
    const int cc = wv + LU_NW * s;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int a = lane + 64 * q;
      col[s][q] = (cc < r && a < r) ? Z[kt + a + (int64_t)(kt + cc) * n] : make_double2(0, 0);
    }
  }
  if (tid == 0) s_fail = 0;
  __syncthreads();
  for (int j = 0; j < r; ++j) {
    const int so = j / LU_NW;
    if (wv == j % LU_NW) {
      double2 x[2];
#pragma unroll
      for (int s = 0; s < LU_CPW; ++s)
        if (s == so) {
          x[0] = col[s][0];
          x[1] = col[s][1];
        }
      // pivot: largest |re| + |im| among the rows not yet eliminated, lowest position on ties
      double best = -1.0;
      int bpos = 0x7fffffff, brow = 0;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int a = lane + 64 * q;
        if (a < r && pos[q] >= j) {
          const double val = fabs(x[q].x) + fabs(x[q].y);
          if (val > best || (val == best && pos[q] < bpos)) {
            best = val;
            bpos = pos[q];
            brow = a;
          }
        }
      }
      const double lbest = best;
      best = wave_max_nonneg(fmax(best, 0.0));  // 0: no nonzero candidate, the block is singular
      const int ppos = wave_min_int(lbest == best ? bpos : 0x7fffffff);
      const unsigned long long hit = __ballot(lbest == best && bpos == ppos);
      const int src = hit ? __ffsll((long long)hit) - 1 : 0;
      const int pr = min(max(__builtin_amdgcn_readlane(brow, src), 0), r - 1);
      bpos = ppos;
      const double2 piv = lane_read(pick2(x, pr >> 6), pr & 63);
      const double pd = cabs2(piv);
      const double2 pinv = make_double2(piv.x / pd, -piv.y / pd);
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int a = lane + 64 * q;
        const bool below = a < r && pos[q] >= j && a != pr;
        const double2 l = below ? cmul(x[q], pinv) : make_double2(0, 0);
        if (below) x[q] = l;
        if (a < LU_REG_MAX) lbuf[j & 1][a] = l;
      }
#pragma unroll
      for (int s = 0; s < LU_CPW; ++s)
        if (s == so) {
          col[s][0] = x[0];
          col[s][1] = x[1];
        }
      if (lane == 0) {
        if (!(best > 0.0) || !hit) s_fail = 1;
        pivrow[j] = pr;
        pjpos[j] = bpos;
        dinv[j] = pinv;
      }
    }
    __syncthreads();
    if (s_fail) {
      if (tid == 0) atomicMax(v.flags, i + 1);
      return;
    }
    const int pr = pivrow[j], pp = pjpos[j];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int a = lane + 64 * q;
      pos[q] = (a == pr) ? j : (pos[q] == j ? pp : pos[q]);
    }
    double2 l[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) l[q] = lbuf[j & 1][lane + 64 * q];
#pragma unroll
    for (int s = 0; s < LU_CPW; ++s) {
      if (wv + LU_NW * s > j && wv + LU_NW * s < r) {
        const double2 xp = lane_read(pick2(col[s], pr >> 6), pr & 63);
#pragma unroll
        for (int q = 0; q < 2; ++q) col[s][q] = csub(col[s][q], cmul(l[q], xp));
      }
    }
  }
  // the factors in the swapped row order
#pragma unroll
  for (int s = 0; s < LU_CPW; ++s) {
    const int cc = wv + LU_NW * s;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int a = lane + 64 * q;
      if (cc < r && a < r) F[pos[q] + (int64_t)cc * r] = col[s][q];
    }
  }
  __syncthreads();
  double2* Li = v.LU + v.lu_off[i];
  double2* Ui = Li + (int64_t)rmax * rmax;
  // column j of U^-1: back substitution U x = e_j
  for (int j = wv; j < r; j += LU_NW) {
    double2 x[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) x[q] = make_double2(lane + 64 * q == j ? 1.0 : 0.0, 0.0);
#pragma unroll 2
    for (int mm = j; mm >= 0; --mm) {
      const double2 xm = cmul(lane_read(pick2(x, mm >> 6), mm & 63), dinv[mm]);
      const double2* fc = F + (int64_t)mm * r;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int a = lane + 64 * q;
        if (a < mm) x[q] = csub(x[q], cmul(fc[a], xm));
        if (a == mm) x[q] = xm;
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int a = lane + 64 * q;
      if (a < r) Ui[a + (int64_t)j * rmax] = a <= j ? x[q] : make_double2(0, 0);
    }
  }
  // column j of L^-1 (unit lower): forward substitution L y = e_j, stored at column pivrow[j]
  for (int j = wv; j < r; j += LU_NW) {
    double2 y[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) y[q] = make_double2(lane + 64 * q == j ? 1.0 : 0.0, 0.0);
#pragma unroll 2
    for (int mm = j; mm + 1 < r; ++mm) {
      const double2 ym = lane_read(pick2(y, mm >> 6), mm & 63);
      const double2* fc = F + (int64_t)mm * r;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int a = lane + 64 * q;
        if (a > mm && a < r) y[q] = csub(y[q], cmul(fc[a], ym));
      }
    }
    double2* lc = Li + (int64_t)pivrow[j] * rmax;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int a = lane + 64 * q;
      if (a < r) lc[a] = a >= j ? y[q] : make_double2(0, 0);
    }
  }
}
__global__ void __launch_bounds__(LU_NT) k_lu_reg(LevelView v, ColourTasks c, double2* scratch, int rm) {
  lu_reg_body(v, c, scratch, rm, vblock());
}
__global__ void __launch_bounds__(LU_NT) k_lu_reg_b(const BatchEntry* E, int ne) {
  VBlock VB;
  const EntryRef e = locate(E, ne, VB);
  lu_reg_body(e.v, e.c, e.buf, e.i0, VB);
}

// Beyond LU_REG_MAX rows: the same factorization with explicit row swaps on F
// (LDS up to LU_LDS_MAX, else scratch) by a 256-thread workgroup.
__device__ __forceinline__ void lu_big_body(const LevelView& v, const ColourTasks& c, double2* scratch, int rm,
                                            const VBlock& VB) {
  __shared__ double2 sF[LU_LDS_MAX * LU_LDS_MAX];
  __shared__ double2 sT[LU_LDS_MAX];
  __shared__ int16_t perm[STEP0_DMAX];
  __shared__ int s_piv;
  __shared__ double s_pv;
  static_assert(STEP0_DMAX <= 32767, "pivot indices are 16-bit");
  const int i = c.cl[VB.x];
  const int n = v.n[i], kt = v.kt[i], r = n - kt, rmax = n - v.k[i];
  if (r <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const double2* Z = v.slots + v.slot_off[v.diag_slot[i]];
  const bool in_lds = r <= LU_LDS_MAX;
  double2* F = in_lds ? sF : scratch + (int64_t)VB.x * ((int64_t)rm * rm + rm);
  double2* tmp = in_lds ? sT : F + (int64_t)rm * rm;
  for (int e = tid; e < r * r; e += blockDim.x) {
    const int a = e % r, b = e / r;
    F[e] = Z[kt + a + (int64_t)(kt + b) * n];
  }
  for (int a = tid; a < r; a += blockDim.x) perm[a] = a;
  __syncthreads();
  for (int j = 0; j < r; ++j) {
    // pivot search by the first wavefront: max |re| + |im| in column j, first index on ties
    if (tid < 64) {
      double best = -1.0;
      int bi = r;
      for (int a = j + lane; a < r; a += 64) {
        const double val = fabs(F[a + j * r].x) + fabs(F[a + j * r].y);
        if (val > best) {
          best = val;
          bi = a;
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ov = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ov > best || (ov == best && oi < bi)) {
          best = ov;
          bi = oi;
        }
      }
      if (lane == 0) {
        s_piv = bi;
        s_pv = best;
      }
    }
    __syncthreads();
    const int pj = s_piv;
    if (!(s_pv > 0.0)) {
      if (tid == 0) atomicMax(v.flags, i + 1);
      return;
    }
    if (pj != j) {
      for (int b = tid; b < r; b += blockDim.x) {
        const double2 t = F[j + b * r];
        F[j + b * r] = F[pj + b * r];
        F[pj + b * r] = t;
      }
      if (tid == 0) {
        const int16_t t = perm[j];
        perm[j] = perm[pj];
        perm[pj] = t;
      }
      __syncthreads();
    }
    const double2 piv = F[j + j * r];
    const double pd = cabs2(piv);
    const double2 pinv = make_double2(piv.x / pd, -piv.y / pd);
    const int rem = r - j - 1;
    // multipliers go to tmp first so that the trailing update reads unscaled values only once
    for (int a = tid; a < rem; a += blockDim.x) tmp[a] = cmul(F[j + 1 + a + j * r], pinv);
    __syncthreads();
    for (int a = tid; a < rem; a += blockDim.x) F[j + 1 + a + j * r] = tmp[a];
    for (int e = tid; e < rem * rem; e += blockDim.x) {
      const int a = e % rem, b = j + 1 + e / rem;
      F[j + 1 + a + b * r] = csub(F[j + 1 + a + b * r], cmul(tmp[a], F[j + b * r]));
    }
    __syncthreads();
  }
  // U^-1 in place (upper triangle): column j from the inverted leading block,
  // U^-1[0:j, j] = -U^-1[0:j, 0:j] U[0:j, j] / U[j, j]
  for (int j = 0; j < r; ++j) {
    const double2 u = F[j + j * r];
    const double ud = cabs2(u);
    const double2 uinv = make_double2(u.x / ud, -u.y / ud);
    for (int a = tid; a < j; a += blockDim.x) {
      double2 acc = make_double2(0, 0);
      for (int mm = a; mm < j; ++mm) acc = cadd(acc, cmul(F[a + mm * r], F[mm + j * r]));
      tmp[a] = acc;
    }
    __syncthreads();
    for (int a = tid; a < j; a += blockDim.x) {
      const double2 t = cmul(tmp[a], uinv);
      F[a + j * r] = make_double2(-t.x, -t.y);
    }
    if (tid == 0) F[j + j * r] = uinv;
    __syncthreads();
  }
  // L^-1 in place (strict lower triangle, unit diagonal), columns right to left:
  // L^-1[j+1:, j] = -L^-1[j+1:, j+1:] L[j+1:, j]
  for (int j = r - 2; j >= 0; --j) {
    for (int a = j + 1 + tid; a < r; a += blockDim.x) {
      double2 acc = F[a + j * r];  // the unit diagonal of L^-1 times L[a, j]
      for (int mm = j + 1; mm < a; ++mm) acc = cadd(acc, cmul(F[a + mm * r], F[mm + j * r]));
      tmp[a] = acc;
    }
    __syncthreads();
    for (int a = j + 1 + tid; a < r; a += blockDim.x) F[a + j * r] = make_double2(-tmp[a].x, -tmp[a].y);
    __syncthreads();
  }
  // write out: U^-1 (upper) and L^-1 P (column j of L^-1 at column perm[j])
  double2* Li = v.LU + v.lu_off[i];
  double2* Ui = Li + (int64_t)rmax * rmax;
  for (int e = tid; e < r * r; e += blockDim.x) {
    const int a = e % r, b = e / r;
    const double2 f = F[a + b * r];
    Ui[a + (int64_t)b * rmax] = (a <= b) ? f : make_double2(0, 0);
    Li[a + (int64_t)perm[b] * rmax] = (a > b) ? f : make_double2(a == b ? 1.0 : 0.0, 0.0);
  }
}
__global__ void __launch_bounds__(256) k_lu_big(LevelView v, ColourTasks c, double2* scratch, int rm) {
  lu_big_body(v, c, scratch, rm, vblock());
}
__global__ void __launch_bounds__(256) k_lu_big_b(const BatchEntry* E, int ne) {
  VBlock VB;
  const EntryRef e = locate(E, ne, VB);
  lu_big_body(e.v, e.c, e.buf, e.i0, VB);
}

void launch_lu(const LevelView& v, const ColourTasks& c, double2* scratch, int rm, hipStream_t st) {
  if (c.ncl <= 0) return;
  if (rm <= LU_REG_MAX)
    hipLaunchKernelGGL(k_lu_reg, dim3(c.ncl), dim3(LU_NT), 0, st, v, c, scratch, rm);
  else
    hipLaunchKernelGGL(k_lu_big, dim3(c.ncl), dim3(256), 0, st, v, c, scratch, rm);
}

// Largest |re| + |im| over the workgroup, folded into *dst with an atomic max on
// the bit pattern (monotone for non-negative doubles).
__device__ void block_max_to(double mx, unsigned long long* dst) {
  __shared__ double red[4];
  mx = wave_max_nonneg(mx);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    atomicMax(dst, (unsigned long long)__double_as_longlong(m));
  }
}

__device__ void panel_max(const TileAcc<double>& acc, unsigned long long* dst) {
  double mx = 0.0;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int q = 0; q < 4; ++q) mx = fmax(mx, fabs(acc.re[t][u][q]) + fabs(acc.im[t][u][q]));
  block_max_to(mx, dst);
}

// Step 3a panels: R_i[:, a] = (L^-1 P) Z_ia[k~:n, 0:m_a]; C_i[a, :] = Z_ai[0:m_a, k~:n] U^-1.
// grid: (panel task, 2x2 tiles, which)
__device__ __forceinline__ void panels_body(const LevelView& v, const ColourTasks& c, const VBlock& VB) {
  __shared__ TileSmem<double> s;
  const int task = VB.x;
  const int i = c.pn_i[task], ja = c.pn_ja[task];
  const int a = v.np_cl[ja];
  const int n = v.n[i], kt = v.kt[i], r = n - kt, rmax = n - v.k[i];
  if (r <= 0) return;
  const int ma = (a == i) ? kt : dim_before(v, a, c.colour);
  const int na = v.n[a];
  const int tr = VB.y % c.tiles, tc = VB.y / c.tiles;
  const double2* Li = v.LU + v.lu_off[i];
  const double2* Ui = Li + (int64_t)rmax * rmax;
  const int off = v.np_off[ja];
  TileAcc<double> acc;
  acc.zero();
  if (VB.z == 0) {
    // R: r x ma
    if (tr * 64 >= r || tc * 64 >= ma) return;
    const int m = min(64, r - tr * 64), nn = min(64, ma - tc * 64);
    const int code = v.np_srow[ja];
    if (code >= 0) {  // rows k~.. of block (i, a), ld n
      const double2* Zia = v.slots + v.slot_off[code] + kt;
      gemm_tile<double, double2>(s, acc, Li + tr * 64, rmax, OP_N, Zia + (int64_t)tc * 64 * n, n, OP_N, m, nn, r);
    } else {  // block (i, a) = S^T, S = stored (a, i) with ld n_a: columns k~.. of S
      const double2* Sai = v.slots + v.slot_off[~code] + (int64_t)kt * na;
      gemm_tile<double, double2>(s, acc, Li + tr * 64, rmax, OP_N, Sai + tc * 64, na, OP_T, m, nn, r);
    }
    double2* R = v.RP + v.rp_off[i] + (int64_t)off * rmax;
    store_tile<double, double2>(acc, R + tr * 64 + (int64_t)tc * 64 * rmax, rmax, m, nn, ST_SET);
    if (v.pmax) {
      panel_max(acc, &v.pmax[4 * i + 1]);
      if (tr == 0 && tc == 0) {  // largest entry of the input block Z_ia[k~:n, 0:m_a]
        double mx = 0.0;
        for (int e = threadIdx.x; e < r * ma; e += blockDim.x) {
          const int q = e % r, j = e / r;
          const double2 z = code >= 0 ? v.slots[v.slot_off[code] + kt + q + (int64_t)j * n]
                                      : v.slots[v.slot_off[~code] + j + (int64_t)(kt + q) * na];
          mx = fmax(mx, fabs(z.x) + fabs(z.y));
        }
        block_max_to(mx, &v.pmax[4 * i + 2]);
      }
    }
  } else {
    // C: ma x r
    if (tr * 64 >= ma || tc * 64 >= r) return;
    const int m = min(64, ma - tr * 64), nn = min(64, r - tc * 64);
    const int code = v.np_scol[ja];
    if (code >= 0) {  // columns k~.. of block (a, i), ld n_a
      const double2* Zai = v.slots + v.slot_off[code] + (int64_t)kt * na;
      gemm_tile<double, double2>(s, acc, Zai + tr * 64, na, OP_N, Ui + (int64_t)tc * 64 * rmax, rmax, OP_N, m, nn,
                                 r);
    } else {  // block (a, i) = S^T, S = stored (i, a) with ld n: rows k~.. of S
      const double2* Sia = v.slots + v.slot_off[~code] + kt;
      gemm_tile<double, double2>(s, acc, Sia + (int64_t)tr * 64 * n, n, OP_T, Ui + (int64_t)tc * 64 * rmax, rmax,
                                 OP_N, m, nn, r);
    }
    const int pr = v.prow[i];
    double2* C = v.CP + v.cp_off[i] + off;
    store_tile<double, double2>(acc, C + tr * 64 + (int64_t)tc * 64 * pr, pr, m, nn, ST_SET);
    if (v.pmax) panel_max(acc, &v.pmax[4 * i]);
  }
}
__global__ void __launch_bounds__(256) k_panels(LevelView v, ColourTasks c) { panels_body(v, c, vblock()); }
__global__ void __launch_bounds__(256) k_panels_b(const BatchEntry* E, int ne) {
  VBlock VB;
  const EntryRef e = locate(E, ne, VB);
  panels_body(e.v, e.c, VB);
}

void launch_panels(const LevelView& v, const ColourTasks& c, hipStream_t st) {
  if (c.npn <= 0) return;
  hipLaunchKernelGGL(k_panels, dim3(c.npn, c.tiles * c.tiles, 2), dim3(256), 0, st, v, c);
}

// Step 3b: Z_ab[0:m_a, 0:m_b] -= sum_i C_i[a] R_i[b] (gather over the colour's clusters)
// One deferred Schur contribution of cluster i to a target block: the rows of
// its C panel that belong to partner ja and the columns of its R panel that
// belong to partner jb (eq. 12 with the panels of eqs. 10-11).
struct SchurTerm {
  const double2* C;
  const double2* R;
  int ldc, ldr, r;
};

// Cluster i's Schur terms may run in FP32 when their FP32 rounding, about
// u32 sqrt(r) max|C| max|R|, stays within F32_KAPPA u32 of the largest entry of the
// blocks its panels were formed from (maxima recorded by the panel kernel).
__device__ __forceinline__ bool f32_safe(const LevelView& v, int i, int r) {
  const double gc = __longlong_as_double((long long)v.pmax[4 * i]);
  const double gr = __longlong_as_double((long long)v.pmax[4 * i + 1]);
  const double z = __longlong_as_double((long long)v.pmax[4 * i + 2]);
  return gc * gr * sqrt((double)r) <= F32_KAPPA * z;
}

// sel: -1 every term, 1 only terms of clusters whose FP32 Schur terms are safe, 0 the others
__device__ __forceinline__ bool schur_term(const LevelView& v, const ColourTasks& c, int e, int tr, int tc, int sel,
                                           SchurTerm& t) {
  const int i = c.sc_i[e];
  const int n = v.n[i], kt = v.kt[i];
  t.r = n - kt;
  if (t.r <= 0) return false;
  if (sel >= 0 && f32_safe(v, i, t.r) != (sel != 0)) return false;
  const int rmax = n - v.k[i];
  t.ldc = v.prow[i];
  t.ldr = rmax;
  t.C = v.CP + v.cp_off[i] + v.np_off[c.sc_ja[e]] + tr * 64;
  t.R = v.RP + v.rp_off[i] + (int64_t)(v.np_off[c.sc_jb[e]] + tc * 64) * rmax;
  return true;
}

// Flush of the Schur updates (eq. 12) pending on a target block: every
// cluster eliminated since the block was last brought up to date adds
// -C_a R_b.  The contraction runs over the concatenated ranks of all pending
// terms as one stream of K slabs, with the next slab (possibly of the next
// term) in flight while the current one is multiplied.  Block dimensions are
// those after colour c.colour (kept rows for processed clusters).  The mixed
// form (MIX) multiplies the slabs of terms whose clusters' panels show no
// growth on FP32 matrix cores into a second set of accumulators, folded into
// the FP64 ones at the end; the other terms (where the update nearly cancels
// the block and FP32 rounding would dominate) stay in FP64.
constexpr int MIX_MIN_K = 64;

union SchurSmem {
  TileSmem<double> d;
  TileSmem<float> f;
};
static_assert(sizeof(SchurSmem) >= 2 * 64 * 64 * sizeof(float), "slab LDS holds one 64 x 64 complex FP32 tile");

// acc += sum over the task's terms selected by sel of C_a R_b (one K stream)
template <typename R>
__device__ __forceinline__ void schur_stream(const LevelView& v, const ColourTasks& c, int e, int e_end, int tr,
                                             int tc, int m, int nn, int mt, int nt, int sel, TileSmem<R>& s,
                                             TileAcc<R>& acc) {
  SchurTerm cur;
  while (e < e_end && !schur_term(v, c, e, tr, tc, sel, cur)) ++e;
  if (e >= e_end) return;
  SlabRegs<double2> regs;
  int k0 = 0;
  slab_fetch<double2>(regs, cur.C, cur.ldc, OP_N, cur.R, cur.ldr, OP_N, m, nn, cur.r, 0);
  while (true) {
    const int nk = min(TK, cur.r - k0);
    __syncthreads();
    slab_store<R, double2>(s, regs, OP_N, OP_N);
    __syncthreads();
    SchurTerm nxt = cur;
    int nk0 = k0 + TK;
    bool more = true;
    if (nk0 >= cur.r) {
      nk0 = 0;
      ++e;
      while (e < e_end && !schur_term(v, c, e, tr, tc, sel, nxt)) ++e;
      more = e < e_end;
    }
    if (more) slab_fetch<double2>(regs, nxt.C, nxt.ldc, OP_N, nxt.R, nxt.ldr, OP_N, m, nn, nxt.r, nk0);
    mma_slab_bal<R>(s, acc, nk, mt, nt);
    if (!more) break;
    cur = nxt;
    k0 = nk0;
  }
}

template <bool MIX>
__device__ __forceinline__ void schur_flush(const LevelView& v, const ColourTasks& c, SchurSmem& s, const VBlock& VB) {
  const int task = VB.x;
  const int sl = c.sc_slot[task];
  const int a = v.slot_a[sl], b = v.slot_b[sl];
  const int ma = dim_after(v, a, c.colour), mb = dim_after(v, b, c.colour);
  const int tr = VB.y % c.tiles, tc = VB.y / c.tiles;
  if (tr * 64 >= ma || tc * 64 >= mb) return;
  const int m = min(64, ma - tr * 64), nn = min(64, mb - tc * 64);
  const int mt = (m + 15) >> 4, nt = (nn + 15) >> 4;
  const int part = c.sc_sp[4 * task], nparts = c.sc_sp[4 * task + 1];
  const int e0 = c.sc_cptr[task], e_end = c.sc_cptr[task + 1];
  {
    int e = e0;
    SchurTerm t;
    while (e < e_end && !schur_term(v, c, e, tr, tc, -1, t)) ++e;
    if (e >= e_end && nparts == 1) return;  // nothing eliminated against this block
  }
  const int na = v.n[a];
  double2* Z = v.slots + v.slot_off[sl] + tr * 64 + (int64_t)tc * 64 * na;
  TileAcc<double> acc;
  acc.zero();
  // mixed form: the FP32 pass pays only when the FP32-safe terms carry enough of
  // the contraction (MIX_MIN_K columns); otherwise every term runs in FP64
  bool split_prec = false;
  if (MIX) {
    // the FP32-safe contraction columns of the task, its terms spread over the lanes
    // (one round of loads rather than a chain of them per term)
    int kf = 0;
    for (int e = e0 + (int)(threadIdx.x & 63); e < e_end; e += 64) {
      SchurTerm t;
      if (schur_term(v, c, e, tr, tc, 1, t)) kf += t.r;
    }
    split_prec = wave_sum_int(kf) >= MIX_MIN_K;
  }
  if (split_prec) {
    // FP32 terms first; their sums then seed the FP64 accumulators (through LDS:
    // the two MFMA shapes place a block's elements on different lanes), so the
    // two accumulator sets are never live together
    TileAcc<float> accf;
    accf.zero();
    schur_stream<float>(v, c, e0, e_end, tr, tc, m, nn, mt, nt, 1, s.f, accf);
    float* fre = reinterpret_cast<float*>(&s);
    float* fim = fre + 64 * 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int cnt = mt * nt, per = (cnt + 3) >> 2;
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kb = w * per + j;
      if (j >= per || kb >= cnt) continue;
      const int rb = kb % mt, cb = kb / mt;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int o = rb * 16 + (lane & 15) + 64 * (cb * 16 + acc_col<float>(lane, q));
        fre[o] = accf.re[j >> 1][j & 1][q];
        fim[o] = accf.im[j >> 1][j & 1][q];
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kb = w * per + j;
      if (j >= per || kb >= cnt) continue;
      const int rb = kb % mt, cb = kb / mt;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int o = rb * 16 + (lane & 15) + 64 * (cb * 16 + acc_col<double>(lane, q));
        acc.re[j >> 1][j & 1][q] = (double)fre[o];
        acc.im[j >> 1][j & 1][q] = (double)fim[o];
      }
    }
    schur_stream<double>(v, c, e0, e_end, tr, tc, m, nn, mt, nt, 0, s.d, acc);
  } else {
    schur_stream<double>(v, c, e0, e_end, tr, tc, m, nn, mt, nt, -1, s.d, acc);
  }
  if (nparts == 1) {
    store_tile_bal_sub<double, double2>(acc, Z, na, m, nn, mt, nt);
    return;
  }
  // a chunk of a split task: its partial tile goes to scratch (k_schur_reduce adds the
  // chunks); the group keeps ta tb tiles per chunk, ta = ceil(n_a / 64), tb = ceil(n_b / 64)
  const int ta = (na + 63) >> 6, tb = (v.n[b] + 63) >> 6;
  double2* Pc = c.sc_part + ((int64_t)c.sc_gbase[c.sc_sp[4 * task + 3]] + (int64_t)part * ta * tb + tr + ta * tc) * 4096;
  store_tile_bal_set<double, double2>(acc, Pc, 64, m, nn, mt, nt);
}

// FP64 form at four waves per SIMD (128 registers); the mixed form needs both
// accumulator shapes and runs at three.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_schur_fp64(LevelView v,
                                                                                        ColourTasks c) {
  __shared__ SchurSmem s;
  schur_flush<false>(v, c, s, vblock());
}
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_schur_fp64_b(const BatchEntry* E,
                                                                                          int ne) {
  __shared__ SchurSmem s;
  VBlock VB;
  const EntryRef e = locate(E, ne, VB);
  schur_flush<false>(e.v, e.c, s, VB);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_schur_mixed(LevelView v,
                                                                                         ColourTasks c) {
  __shared__ SchurSmem s;
  schur_flush<true>(v, c, s, vblock());
}
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_schur_mixed_b(const BatchEntry* E,
                                                                                           int ne) {
  __shared__ SchurSmem s;
  VBlock VB;
  const EntryRef e = locate(E, ne, VB);
  schur_flush<true>(e.v, e.c, s, VB);
}

// Split tasks: Z -= the sum of the chunks' partial tiles, added in chunk order.
// grid: (group, tiles^2, 4); each workgroup takes a quarter of the tile's
// elements, four per thread, with the block values and all four elements'
// partials of a chunk in flight together.
__device__ __forceinline__ void schur_reduce_body(const LevelView& v, const ColourTasks& c, const VBlock& VB) {
  const int task = c.sc_gtask[VB.x];
  const int sl = c.sc_slot[task];
  const int a = v.slot_a[sl], b = v.slot_b[sl];
  const int ma = dim_after(v, a, c.colour), mb = dim_after(v, b, c.colour);
  const int tr = VB.y % c.tiles, tc = VB.y / c.tiles;
  if (tr * 64 >= ma || tc * 64 >= mb) return;
  const int m = min(64, ma - tr * 64), nn = min(64, mb - tc * 64);
  const int nparts = c.sc_sp[4 * task + 1];
  const int na = v.n[a];
  const int ta = (na + 63) >> 6, tb = (v.n[b] + 63) >> 6;
  const int64_t tt = (int64_t)ta * tb;
  const double2* P0 = c.sc_part + ((int64_t)c.sc_gbase[VB.x] + tr + ta * tc) * 4096;
  double2* Z = v.slots + v.slot_off[sl] + tr * 64 + (int64_t)tc * 64 * na;
  int off[4];
  bool ok[4];
  double2 zv[4], sum[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int q = VB.z * 1024 + u * 256 + threadIdx.x;  // element (q % 64, q / 64) of the tile
    const int i = q & 63, j = q >> 6;
    ok[u] = i < m && j < nn;
    off[u] = i + 64 * j;
    zv[u] = ok[u] ? Z[i + (int64_t)j * na] : make_double2(0, 0);
    sum[u] = make_double2(0, 0);
  }
#pragma unroll 2
  for (int ch = 0; ch < nparts; ++ch) {
    const double2* Pc = P0 + (int64_t)ch * tt * 4096;
    double2 pv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) pv[u] = ok[u] ? Pc[off[u]] : make_double2(0, 0);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      sum[u].x += pv[u].x;
      sum[u].y += pv[u].y;
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (ok[u]) Z[(off[u] & 63) + (int64_t)(off[u] >> 6) * na] = make_double2(zv[u].x - sum[u].x, zv[u].y - sum[u].y);
}
__global__ void __launch_bounds__(256) k_schur_reduce(LevelView v, ColourTasks c) { schur_reduce_body(v, c, vblock()); }
__global__ void __launch_bounds__(256) k_schur_reduce_b(const BatchEntry* E, int ne) {
  VBlock VB;
  const EntryRef e = locate(E, ne, VB);
  schur_reduce_body(e.v, e.c, VB);
}

void launch_schur(const LevelView& v, const ColourTasks& c, bool mixed, hipStream_t st) {
  if (c.nsc <= 0) return;
  const dim3 grid(c.nsc, c.tiles * c.tiles), rgrid(c.ngrp > 0 ? c.ngrp : 1, c.tiles * c.tiles, 4);
  if (mixed)
    hipLaunchKernelGGL(k_schur_mixed, grid, dim3(256), 0, st, v, c);
  else
    hipLaunchKernelGGL(k_schur_fp64, grid, dim3(256), 0, st, v, c);
  if (c.ngrp > 0) hipLaunchKernelGGL(k_schur_reduce, rgrid, dim3(256), 0, st, v, c);
}

// ===========================================================================
// Level end
// ===========================================================================
__global__ void k_zero(double2* p, int64_t n) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    p[e] = make_double2(0, 0);
}

// dst + dst_off[b] <- src + src_off[b], len[b] elements, one workgroup per block
__global__ void k_copy_blocks(const double2* src, const int64_t* src_off, double2* dst, const int64_t* dst_off,
                              const int64_t* len) {
  const int b = blockIdx.x;
  const double2* a = src + src_off[b];
  double2* d = dst + dst_off[b];
  for (int64_t e = threadIdx.x; e < len[b]; e += blockDim.x) d[e] = a[e];
}

void launch_copy_blocks(const double2* src, const int64_t* src_off, double2* dst, const int64_t* dst_off,
                        const int64_t* len, int nb, hipStream_t st) {
  if (nb <= 0) return;
  hipLaunchKernelGGL(k_copy_blocks, dim3(nb), dim3(256), 0, st, src, src_off, dst, dst_off, len);
}

// Host arrays staged in one buffer, spread to their device arrays: one workgroup
// per piece of at most STAGE_PIECE bytes, 16-byte words (pieces start 16-byte
// aligned on both sides), the last 4-byte words of a piece one per thread.
__global__ void __launch_bounds__(256) k_scatter_segments(const char* base, const CopySeg* segs) {
  const CopySeg sg = segs[blockIdx.x];
  const char* a = base + sg.src;
  char* d = static_cast<char*>(sg.dst);
  const int64_t q = sg.bytes >> 4;
  for (int64_t e = threadIdx.x; e < q; e += blockDim.x)
    reinterpret_cast<uint4*>(d)[e] = reinterpret_cast<const uint4*>(a)[e];
  const int64_t w0 = q << 2, words = sg.bytes >> 2;
  if (w0 + threadIdx.x < words)
    reinterpret_cast<uint32_t*>(d)[w0 + threadIdx.x] = reinterpret_cast<const uint32_t*>(a)[w0 + threadIdx.x];
}

void launch_scatter_segments(const char* base, const CopySeg* segs, int nseg, hipStream_t st) {
  if (nseg <= 0) return;
  hipLaunchKernelGGL(k_scatter_segments, dim3(nseg), dim3(256), 0, st, base, segs);
}

void launch_zero(double2* p, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int blocks = (int)imin64(8192, (n + 255) / 256);
  hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, st, p, n);
}

__global__ void k_merge(LevelView v, const MergeTask* tasks, const double2* S, double2* dst) {
  const MergeTask t = tasks[blockIdx.x];
  const int ka = v.kt[t.ca], kb = v.kt[t.cb];
  double2* D = dst + t.dst;
  // source element (i, j) of the ordered pair (ca, cb); a transposed source
  // stores (cb, ca) with leading dimension n_cb
  const int64_t si = t.tr ? (int64_t)v.n[t.cb] : 1, sj = t.tr ? 1 : (int64_t)v.n[t.ca];
  if (t.kind == 0 || t.kind == 2) {
    const double2* Z = v.slots + v.slot_off[t.slot];
    for (int e = threadIdx.x; e < ka * kb; e += blockDim.x) {
      const int i = e % ka, j = e / ka;
      D[i + j * t.ldd] = Z[i * si + j * sj];
    }
  } else {
    const double2* F = t.slot >= 0 ? v.slots + v.slot_off[t.slot] : nullptr;
    for (int e = threadIdx.x; e < ka * kb; e += blockDim.x) {
      const int i = e % ka, j = e / ka;
      double2 val = make_double2(0, 0);
      if (i < t.ska && j < t.skb) val = S[t.soff + i + (int64_t)j * t.ska];
      if (F) val = cadd(val, F[i * si + j * sj]);
      D[i + j * t.ldd] = val;
    }
  }
}

void launch_merge(const LevelView& v, const MergeTask* t, int nt, const double2* S, double2* dst,
                  hipStream_t st) {
  if (nt <= 0) return;
  hipLaunchKernelGGL(k_merge, dim3(nt), dim3(256), 0, st, v, t, S, dst);
}

// B_p (n_p x k_p) = transfer matrix T_p with zero rows for the children's added columns (eq. 23)
__global__ void k_parent_basis(const int32_t* pn, const int32_t* pk, const int32_t* k1, const int32_t* k2,
                               const int32_t* off1, const int64_t* toff, const double2* T,
                               const int64_t* boff, double2* B) {
  const int p = blockIdx.x;
  const int n = pn[p], k = pk[p];
  const double2* Tp = T + toff[p];
  const int ld = k1[p] + k2[p];
  double2* Bp = B + boff[p];
  for (int e = threadIdx.x; e < n * k; e += blockDim.x) {
    const int r = e % n, col = e / n;
    double2 val = make_double2(0, 0);
    if (r < k1[p])
      val = Tp[r + (int64_t)col * ld];
    else if (r >= off1[p] && r < off1[p] + k2[p])
      val = Tp[k1[p] + (r - off1[p]) + (int64_t)col * ld];
    Bp[e] = val;
  }
}

void launch_parent_basis(int np, const int32_t* pn, const int32_t* pk, const int32_t* k1, const int32_t* k2,
                         const int32_t* off1, const int64_t* toff, const double2* T, const int64_t* boff,
                         double2* B, hipStream_t st) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_parent_basis, dim3(np), dim3(256), 0, st, pn, pk, k1, k2, off1, toff, T, boff, B);
}

// ===========================================================================
// Dense final LU (blocked right-looking, panel width 64)
// ===========================================================================
// Panel of the final dense LU: columns [j0, j0 + w) over rows [j0, n), partial
// pivoting (largest |re| + |im|, lowest row on ties, as zgetrf).  Row interchanges
// are applied to the panel's own columns only (k_dense_laswp applies them to the
// others).  The columns are taken in groups of DP_GROUP.  One workgroup factors a
// group: per column the pivot, the interchange, the L column and the rank-1
// update of the group's later columns in a single pass over the rows (each thread
// keeps DP_RU rows' loads in flight, and the pass also yields the next column's
// pivot candidates), then the group's rows of the later panel columns become U
// rows (L_gg^-1 times them).  The rows below the group of the later panel
// columns are then updated by a matrix-core GEMM over many workgroups, so the
// single workgroup never streams the whole panel.
constexpr int DP_GROUP = 4;
constexpr int DP_RU = 4;

// the workgroup's pivot from per-thread candidates (value, row): largest value,
// lowest row among equal values
__device__ __forceinline__ void dense_pivot(double best, int bi, double* rv, int* ri, double& pv, int& pj) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double wm = wave_max_nonneg(fmax(best, 0.0));
  const int wi = wave_min_int(best == wm ? bi : 0x7fffffff);
  if (lane == 0) {
    rv[wv] = wm;
    ri[wv] = wi;
  }
  __syncthreads();
  pv = rv[0];
  pj = ri[0];
  for (int u = 1; u < 16; ++u)
    if (rv[u] > pv || (rv[u] == pv && ri[u] < pj)) {
      pv = rv[u];
      pj = ri[u];
    }
  __syncthreads();
}

__global__ void __launch_bounds__(1024) k_dense_group(double2* A, int64_t n, int64_t j0, int g0, int32_t* piv,
                                                      double2* linv, int32_t* flag) {
  __shared__ double rv[16];
  __shared__ int ri[16];
  __shared__ double2 srow[DP_GROUP];
  __shared__ double2 sD[64 * 64];
  if (*flag) return;  // an earlier group met a zero pivot: the factorization has failed
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int w = (int)imin64(64, n - j0), ge = min(w, g0 + DP_GROUP);
  // pivot candidates of the group's first column
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int64_t a = j0 + g0 + tid; a < n; a += blockDim.x) {
    const double2 x = A[a + (j0 + g0) * n];
    const double val = fabs(x.x) + fabs(x.y);
    if (val > best) {
      best = val;
      bi = (int)a;
    }
  }
  for (int jj = g0; jj < ge; ++jj) {
    const int64_t j = j0 + jj;
    double pv;
    int pj;
    dense_pivot(best, bi, rv, ri, pv, pj);
    if (!(pv > 0.0) || pj >= n) {
      if (tid == 0) *flag = 1;
      return;
    }
    if (tid == 0) piv[j] = pj;
    // interchange rows j and pj within the panel's columns
    if (pj != j && tid < w) {
      const int64_t cb = (j0 + tid) * n;
      const double2 t = A[j + cb];
      A[j + cb] = A[pj + cb];
      A[pj + cb] = t;
    }
    __syncthreads();
    const double2 p = A[j + j * n];
    const double pd = cabs2(p);
    const double2 pinv = make_double2(p.x / pd, -p.y / pd);
    const int nb = ge - jj - 1;  // later columns of the group
    if (tid < nb) srow[tid] = A[j + (j + 1 + tid) * n];
    __syncthreads();
    best = -1.0;
    bi = 0x7fffffff;
    for (int64_t a0 = j + 1 + tid; a0 < n; a0 += (int64_t)DP_RU * blockDim.x) {
      double2 l[DP_RU], x[DP_RU][DP_GROUP - 1];
#pragma unroll
      for (int u = 0; u < DP_RU; ++u) {
        const int64_t a = a0 + (int64_t)u * blockDim.x;
        if (a < n) {
          l[u] = A[a + j * n];
#pragma unroll
          for (int q = 0; q < DP_GROUP - 1; ++q)
            if (q < nb) x[u][q] = A[a + (j + 1 + q) * n];
        }
      }
#pragma unroll
      for (int u = 0; u < DP_RU; ++u) {
        const int64_t a = a0 + (int64_t)u * blockDim.x;
        if (a < n) {
          const double2 lv = cmul(l[u], pinv);
          A[a + j * n] = lv;
#pragma unroll
          for (int q = 0; q < DP_GROUP - 1; ++q)
            if (q < nb) {
              const double2 y = csub(x[u][q], cmul(lv, srow[q]));
              A[a + (j + 1 + q) * n] = y;
              if (q == 0) {  // candidate for the next column's pivot (rows visited in increasing order)
                const double val = fabs(y.x) + fabs(y.y);
                if (val > best) {
                  best = val;
                  bi = (int)a;
                }
              }
            }
        }
      }
    }
    __syncthreads();
  }
  // the group's rows of the later panel columns: U_g = L_gg^-1 A[group rows, later columns]
  const int ng = ge - g0, nl = w - ge;
  for (int b = tid; b < nl; b += blockDim.x) {
    const int64_t cb = (j0 + ge + b) * n;
    double2 u[DP_GROUP];
#pragma unroll
    for (int k = 0; k < DP_GROUP; ++k) {
      if (k >= ng) break;
      double2 v = A[j0 + g0 + k + cb];
      for (int q = 0; q < k; ++q) v = csub(v, cmul(A[j0 + g0 + k + (j0 + g0 + q) * n], u[q]));
      u[k] = v;
      A[j0 + g0 + k + cb] = v;
    }
  }
  if (ge < w) return;
  __syncthreads();
  // last group: explicit inverse of the panel's unit-lower diagonal block, a column
  // per wavefront by forward substitution, rows on lanes, the block in LDS
  for (int e = tid; e < w * w; e += blockDim.x) sD[(e % w) + 64 * (e / w)] = A[j0 + (e % w) + (j0 + e / w) * n];
  __syncthreads();
  for (int col = wv; col < 64; col += 16) {
    double2 y = make_double2(lane == col ? 1.0 : 0.0, 0.0);
    if (col < w)
      for (int mm = col; mm + 1 < w; ++mm) {
        const double2 ym = lane_read(y, mm);
        if (lane > mm && lane < w) y = csub(y, cmul(sD[lane + 64 * mm], ym));
      }
    linv[lane + col * 64] = (col < w && lane >= col && lane < w) ? y : make_double2(0, 0);
  }
}

// The panel's row interchanges (rows j <-> piv[j], j = j0 .. j0 + w - 1, in order)
// applied to every column outside the panel: a thread per column.
__global__ void k_dense_laswp(double2* A, int64_t n, int64_t j0, int w, const int32_t* piv) {
  int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= n - w) return;
  if (c >= j0) c += w;  // skip the panel's columns
  double2* col = A + c * n;
  for (int jj = 0; jj < w; ++jj) {
    const int64_t j = j0 + jj, pj = piv[j];
    // a panel that met a zero pivot stops early and leaves later entries unset
    // (the factorization then fails): only in-range interchanges are applied
    if (pj > j && pj < n) {
      const double2 t = col[j];
      col[j] = col[pj];
      col[pj] = t;
    }
  }
}

void launch_dense_panel(double2* A, int64_t n, int64_t j0, int32_t* piv, double2* linv, int32_t* flag,
                        hipStream_t st) {
  const int w = (int)std::min<int64_t>(64, n - j0);
  for (int g0 = 0; g0 < w; g0 += DP_GROUP) {
    hipLaunchKernelGGL(k_dense_group, dim3(1), dim3(1024), 0, st, A, n, j0, g0, piv, linv, flag);
    const int ge = std::min(w, g0 + DP_GROUP);
    const int64_t rows = n - j0 - ge;
    // rows below the group of the later panel columns -= L[rows, group] U[group, later columns]
    if (ge < w && rows > 0)
      launch_gemm_one({A + (j0 + ge) + (j0 + g0) * n, A + (j0 + g0) + (j0 + ge) * n, A + (j0 + ge) + (j0 + ge) * n,
                       n, n, n, (int32_t)rows, w - ge, ge - g0, OP_N, OP_N, ST_SUB},
                      st);
  }
  if (n - w > 0)
    hipLaunchKernelGGL(k_dense_laswp, dim3((unsigned)((n - w + 255) / 256)), dim3(256), 0, st, A, n, j0, w, piv);
}

// inverse of the upper-triangular 64 x 64 (or smaller) diagonal block at A (ld n) -> Uinv
// (ld 64): a column per wavefront by back substitution, rows on lanes, the block in LDS
__global__ void __launch_bounds__(1024) k_tri_inv_upper(const double2* A, int64_t n, int w, double2* Uinv) {
  __shared__ double2 sU[64 * 64];
  __shared__ double2 dinv[64];
  const int tid = threadIdx.x, lane = tid & 63, wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  for (int e = tid; e < w * w; e += blockDim.x) sU[(e % w) + 64 * (e / w)] = A[(e % w) + (int64_t)(e / w) * n];
  __syncthreads();
  if (tid < w) {
    const double2 u = sU[tid + 64 * tid];
    const double ud = cabs2(u);
    dinv[tid] = make_double2(u.x / ud, -u.y / ud);
  }
  __syncthreads();
  for (int col = wv; col < 64; col += 16) {
    double2 x = make_double2(lane == col ? 1.0 : 0.0, 0.0);
    if (col < w)
      for (int mm = col; mm >= 0; --mm) {
        const double2 xm = cmul(lane_read(x, mm), dinv[mm]);
        if (lane == mm) x = xm;
        if (lane < mm) x = csub(x, cmul(sU[lane + 64 * mm], xm));
      }
    Uinv[lane + col * 64] = (col < w && lane <= col) ? x : make_double2(0, 0);
  }
}

void launch_tri_inv_upper(const double2* A, int64_t n, int w, double2* Uinv, hipStream_t st) {
  hipLaunchKernelGGL(k_tri_inv_upper, dim3(1), dim3(1024), 0, st, A, n, w, Uinv);
}

// X (n x n) = P: the permutation produced by the recorded row interchanges
__global__ void k_perm_matrix(double2* X, int64_t n, const int32_t* piv) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n; c += (int64_t)gridDim.x * blockDim.x) {
    int64_t pos = c;
    for (int64_t j = 0; j < n; ++j) {
      const int64_t pj = piv[j];
      if (pos == j)
        pos = pj;
      else if (pos == pj)
        pos = j;
    }
    X[pos + c * n] = make_double2(1, 0);
  }
}

void launch_apply_perm_cols(double2* X, int64_t n, const int32_t* piv, hipStream_t st) {
  int blocks = (int)imin64(1024, (n + 255) / 256);
  hipLaunchKernelGGL(k_perm_matrix, dim3(blocks), dim3(256), 0, st, X, n, piv);
}

// ---------------------------------------------------------------------------
// Solves with the final block's LU factors (P Z_f = L U, L unit lower and U upper
// stored in place, 64 x 64 inverses of their diagonal blocks kept).
// ---------------------------------------------------------------------------
// out[i] = in[perm[i]] (scatter = 0) or out[perm[i]] = in[i] (scatter = 1), nrhs columns
__global__ void k_dense_perm(const double2* in, double2* out, const int32_t* perm, int64_t n, int nrhs, int64_t ld,
                             int scatter) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t q = perm[i];
  for (int c = 0; c < nrhs; ++c) {
    if (scatter)
      out[q + c * ld] = in[i + c * ld];
    else
      out[i + c * ld] = in[q + c * ld];
  }
}

constexpr int TRSV_RHS = 16;  // right-hand sides per LDS pass

// One block step of a right-looking triangular solve on the 64-row block at j0
// (w rows).  Every workgroup forms t = D x_b for the block (D = its diagonal
// block's inverse, or that inverse's conjugate transpose), workgroup 0 stores t
// in y_b, and each workgroup subtracts the block's coupling times t from its
// share of the rows still to be solved (in x, in place; x_b itself is only read):
//   mode 0  L y = x, forward:  x[r] -= L[r, b] t for r >= j0 + w
//   mode 1  U y = x, backward: x[r] -= U[r, b] t for r < j0
//   mode 2  U^H y = x, forward:  x[r] -= U[b, r]^H t for r >= j0 + w
//   mode 3  L^H y = x, backward: x[r] -= L[b, r]^H t for r < j0
// Modes 0/1 read columns of the factor (a thread per row, coalesced); modes 2/3
// read rows of it (a wavefront per row, 64 consecutive entries, DPP sums).
__global__ void __launch_bounds__(256) k_dense_trsv_step(const double2* A, int64_t n, int64_t j0, int w,
                                                         const double2* D, double2* x, double2* y, int64_t ld,
                                                         int nrhs, int mode) {
  __shared__ double2 t[64 * TRSV_RHS];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const bool fwd = (mode == 0 || mode == 2);
  const int64_t r0 = fwd ? j0 + w : 0, r1 = fwd ? n : j0;
  const bool rowwise = (mode >= 2);
  const int64_t rows_per_wg = rowwise ? 16 : 256;
  const int64_t rbeg = r0 + blockIdx.x * rows_per_wg;
  for (int c0 = 0; c0 < nrhs; c0 += TRSV_RHS) {
    const int nc = min(TRSV_RHS, nrhs - c0);
    __syncthreads();
    // t = D x_b (mode 0/1) or D^H x_b (mode 2/3) for nc columns: thread (row i, column),
    // sixteen loads in flight (D is zero outside the block's w x w corner)
    for (int e = tid; e < 64 * nc; e += blockDim.x) {
      const int i = e & 63, c = e >> 6;
      double2 acc = make_double2(0, 0);
      const double2* xb = x + j0 + (c0 + c) * ld;
      for (int k0 = 0; k0 < w; k0 += 16) {
        double2 dv[16], xv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int k = k0 + u;
          dv[u] = k < w ? (rowwise ? D[k + 64 * i] : D[i + 64 * k]) : make_double2(0, 0);
          xv[u] = k < w ? xb[k] : make_double2(0, 0);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) acc = cadd(acc, rowwise ? cmulc(dv[u], xv[u]) : cmul(dv[u], xv[u]));
      }
      t[i + 64 * c] = i < w ? acc : make_double2(0, 0);
    }
    __syncthreads();
    if (blockIdx.x == 0)
      for (int e = tid; e < 64 * nc; e += blockDim.x)
        if ((e & 63) < w) y[j0 + (e & 63) + (c0 + (e >> 6)) * ld] = t[e];
    if (!rowwise) {
      const int64_t r = rbeg + tid;
      if (r < r1 && r < rbeg + rows_per_wg) {
        double2 acc[TRSV_RHS];
#pragma unroll
        for (int c = 0; c < TRSV_RHS; ++c) acc[c] = make_double2(0, 0);
        for (int k0 = 0; k0 < w; k0 += 16) {
          double2 av[16];
#pragma unroll
          for (int u = 0; u < 16; ++u) av[u] = (k0 + u < w) ? A[r + (j0 + k0 + u) * n] : make_double2(0, 0);
#pragma unroll
          for (int u = 0; u < 16; ++u)
#pragma unroll
            for (int c = 0; c < TRSV_RHS; ++c)
              if (c < nc) acc[c] = cadd(acc[c], cmul(av[u], t[k0 + u + 64 * c]));
        }
        for (int c = 0; c < nc; ++c) {
          double2* p = x + r + (c0 + c) * ld;
          *p = csub(*p, acc[c]);
        }
      }
    } else {
      // four wavefronts, four rows each; lane k holds conj(A[j0 + k, r])
      for (int q = 0; q < 4; ++q) {
        const int64_t r = rbeg + wv * 4 + q;
        if (r >= r1) break;  // uniform per wavefront
        const double2 a = lane < w ? cconj(A[j0 + lane + r * n]) : make_double2(0, 0);
        for (int c = 0; c < nc; ++c) {
          const double2 pr = cmul(a, t[lane + 64 * c]);
          const double sr = wave_sum(pr.x), si = wave_sum(pr.y);
          if (lane == 0) {
            double2* p = x + r + (c0 + c) * ld;
            *p = make_double2(p->x - sr, p->y - si);
          }
        }
      }
    }
  }
}

void launch_dense_perm(const double2* in, double2* out, const int32_t* perm, int64_t n, int nrhs, int64_t ld,
                       int scatter, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_dense_perm, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, out, perm, n, nrhs, ld,
                     scatter);
}

void launch_dense_trsv_step(const double2* A, int64_t n, int64_t j0, int w, const double2* D, double2* x,
                            double2* y, int64_t ld, int nrhs, int mode, hipStream_t st) {
  const bool fwd = (mode == 0 || mode == 2);
  const int64_t rows = fwd ? n - j0 - w : j0;
  const int64_t per = (mode >= 2) ? 16 : 256;
  const int64_t nwg = std::max<int64_t>(1, (rows + per - 1) / per);
  hipLaunchKernelGGL(k_dense_trsv_step, dim3((unsigned)nwg), dim3(256), 0, st, A, n, j0, w, D, x, y, ld, nrhs, mode);
}

// ===========================================================================
// Substitution sweeps (nrhs columns, right-hand sides are the N dimension of
// the MFMA tiles; blockIdx.z selects a block of 64 right-hand sides)
// ===========================================================================
// C (m x n) (op)= op(A) op(B) over every 64x64 tile, by one workgroup.
__device__ void wg_gemm(TileSmem<double>& s, const double2* A, int64_t lda, int opA, const double2* B, int64_t ldb,
                        int opB, double2* C, int64_t ldc, int m, int n, int K, int mode) {
  for (int tr = 0; tr * 64 < m; ++tr)
    for (int tc = 0; tc * 64 < n; ++tc) {
      const int mm = min(64, m - tr * 64), nn = min(64, n - tc * 64);
      const double2* At = (opA == OP_N || opA == OP_R) ? A + tr * 64 : A + (int64_t)tr * 64 * lda;
      const double2* Bt = (opB == OP_N || opB == OP_R) ? B + (int64_t)tc * 64 * ldb : B + tc * 64;
      TileAcc<double> acc;
      acc.zero();
      gemm_tile<double, double2>(s, acc, At, lda, opA, Bt, ldb, opB, mm, nn, K);
      store_tile<double, double2>(acc, C + tr * 64 + (int64_t)tc * 64 * ldc, ldc, mm, nn, mode);
    }
}

// Forward (adj 0): b_i <- Q~^H b_i, b_i' <- (L^-1 P) b_i'.
// Adjoint phase A (adj 1): g_i <- Q~^T g_i, g_i' <- U^-H g_i'.
// scratch: (ncl * gridDim.z) blocks of (64 tiles) x 64.
__device__ __forceinline__ void k_sw_fwd_local_body(LevelView v, ColourTasks c, double2* vec, const int64_t* voff,
                                                      int64_t ldv, int nrhs, int adj, double2* scratch, const VBlock& VB) {
  __shared__ TileSmem<double> s;
  const int i = c.cl[VB.x];
  const int n = v.n[i], kt = v.kt[i], r = n - kt, rmax = n - v.k[i];
  if (n == 0) return;
  const int c0 = VB.z * 64, nr = min(64, nrhs - c0);
  const int ldy = c.tiles * 64;
  double2* Y = scratch + ((int64_t)VB.z * VB.gx + VB.x) * ldy * 64;
  double2* b = vec + voff[i] + (int64_t)c0 * ldv;
  const double2* Q = v.Q + v.q_off[i];
  wg_gemm(s, Q, n, adj ? OP_T : OP_C, b, ldv, OP_N, Y, ldy, n, nr, n, ST_SET);
  __syncthreads();
  for (int e = threadIdx.x; e < kt * nr; e += blockDim.x) {
    const int row = e % kt, col = e / kt;
    b[row + (int64_t)col * ldv] = Y[row + (int64_t)col * ldy];
  }
  if (r > 0) {
    const double2* Li = v.LU + v.lu_off[i];
    const double2* Ui = Li + (int64_t)rmax * rmax;
    if (!adj)
      wg_gemm(s, Li, rmax, OP_N, Y + kt, ldy, OP_N, b + kt, ldv, r, nr, r, ST_SET);
    else
      wg_gemm(s, Ui, rmax, OP_C, Y + kt, ldy, OP_N, b + kt, ldv, r, nr, r, ST_SET);
  }
}
__global__ void __launch_bounds__(256) k_sw_fwd_local(LevelView v, ColourTasks c, double2* vec, const int64_t* voff,
                                                      int64_t ldv, int nrhs, int adj, double2* scratch) {
  k_sw_fwd_local_body(v, c, vec, voff, ldv, nrhs, adj, scratch, vblock());
}
__global__ void __launch_bounds__(256) k_sw_fwd_local_b(const SweepEntry* E, int ne) {
  VBlock VB;
  const SweepRef e = locate_sweep(E, ne, VB);
  k_sw_fwd_local_body(e.v, e.c, e.vec, e.voff, e.ldv, e.nrhs, e.adj, e.scratch, VB);
}

// b_a[0:m_a] -= sum_i C_i[a] b_i'  (adj: g_a -= R_i[:, a]^H g_i').  grid: (target, row tiles, rhs blocks)
__device__ __forceinline__ void k_sw_fwd_gather_body(LevelView v, ColourTasks c, double2* vec, const int64_t* voff,
                                                       int64_t ldv, int nrhs, int adj, const VBlock& VB) {
  __shared__ TileSmem<double> s;
  const int task = VB.x;
  const int a = c.sv_cl[task];
  const int ma = dim_after(v, a, c.colour);
  const int tr = VB.y;
  if (tr * 64 >= ma) return;
  const int m = min(64, ma - tr * 64);
  const int c0 = VB.z * 64, nr = min(64, nrhs - c0);
  TileAcc<double> acc;
  acc.zero();
  for (int e = c.sv_cptr[task]; e < c.sv_cptr[task + 1]; ++e) {
    const int i = c.sv_i[e];
    const int n = v.n[i], kt = v.kt[i], r = n - kt, rmax = n - v.k[i];
    if (r <= 0) continue;
    const int off = v.np_off[c.sv_ja[e]];
    const double2* bi = vec + voff[i] + kt + (int64_t)c0 * ldv;
    if (!adj) {
      const int pr = v.prow[i];
      gemm_tile<double, double2>(s, acc, v.CP + v.cp_off[i] + off + tr * 64, pr, OP_N, bi, ldv, OP_N, m, nr, r);
    } else {
      gemm_tile<double, double2>(s, acc, v.RP + v.rp_off[i] + (int64_t)(off + tr * 64) * rmax, rmax, OP_C, bi, ldv,
                                 OP_N, m, nr, r);
    }
  }
  store_tile<double, double2>(acc, vec + voff[a] + tr * 64 + (int64_t)c0 * ldv, ldv, m, nr, ST_SUB);
}
__global__ void __launch_bounds__(256) k_sw_fwd_gather(LevelView v, ColourTasks c, double2* vec, const int64_t* voff,
                                                       int64_t ldv, int nrhs, int adj) {
  k_sw_fwd_gather_body(v, c, vec, voff, ldv, nrhs, adj, vblock());
}
__global__ void __launch_bounds__(256) k_sw_fwd_gather_b(const SweepEntry* E, int ne) {
  VBlock VB;
  const SweepRef e = locate_sweep(E, ne, VB);
  k_sw_fwd_gather_body(e.v, e.c, e.vec, e.voff, e.ldv, e.nrhs, e.adj, VB);
}

// Partial sums of the backward gather: part_j = sum over partners of chunk j of
// R_i[:, a] y_a (adj: C_i[a, :]^H g_a).  grid: (cluster, chunk, rhs blocks)
__device__ __forceinline__ void k_sw_bwd_partial_body(LevelView v, ColourTasks c, const double2* vec,
                                                        const int64_t* voff, int64_t ldv, int nrhs, int adj,
                                                        double2* part, int nsplit, const VBlock& VB) {
  __shared__ TileSmem<double> s;
  const int i = c.cl[VB.x];
  const int n = v.n[i], kt = v.kt[i], r = n - kt, rmax = n - v.k[i];
  const int chunk = VB.y;
  const int c0 = VB.z * 64, nr = min(64, nrhs - c0);
  const int ldp = c.tiles * 64;
  double2* P = part + (((int64_t)VB.z * VB.gx + VB.x) * nsplit + chunk) * ldp * 64;
  if (r <= 0) return;
  const int pr = v.prow[i];
  for (int tr = 0; tr * 64 < r; ++tr) {
    const int m = min(64, r - tr * 64);
    TileAcc<double> acc;
    acc.zero();
    for (int j = v.np_ptr[i] + chunk; j < v.np_ptr[i + 1]; j += nsplit) {
      const int a = v.np_cl[j];
      const int ma = (a == i) ? kt : dim_before(v, a, c.colour);
      const double2* ya = vec + voff[a] + (int64_t)c0 * ldv;
      const int off = v.np_off[j];
      if (!adj)
        gemm_tile<double, double2>(s, acc, v.RP + v.rp_off[i] + tr * 64 + (int64_t)off * rmax, rmax, OP_N, ya, ldv,
                                   OP_N, m, nr, ma);
      else
        gemm_tile<double, double2>(s, acc, v.CP + v.cp_off[i] + off + (int64_t)tr * 64 * pr, pr, OP_C, ya, ldv, OP_N,
                                   m, nr, ma);
    }
    store_tile<double, double2>(acc, P + tr * 64, ldp, m, nr, ST_SET);
  }
}
__global__ void __launch_bounds__(256) k_sw_bwd_partial(LevelView v, ColourTasks c, const double2* vec,
                                                        const int64_t* voff, int64_t ldv, int nrhs, int adj,
                                                        double2* part, int nsplit) {
  k_sw_bwd_partial_body(v, c, vec, voff, ldv, nrhs, adj, part, nsplit, vblock());
}
__global__ void __launch_bounds__(256) k_sw_bwd_partial_b(const SweepEntry* E, int ne) {
  VBlock VB;
  const SweepRef e = locate_sweep(E, ne, VB);
  k_sw_bwd_partial_body(e.v, e.c, e.vec, e.voff, e.ldv, e.nrhs, e.adj, e.part, e.nsplit, VB);
}

// Backward (adj 0): y_i' <- U^-1 (y_i' - sum parts), y_i <- conj(Q~) y_i.
// Adjoint phase B (adj 1): g_i' <- (L^-1 P)^H (g_i' - sum parts), g_i <- Q~ g_i.
__device__ __forceinline__ void k_sw_bwd_local_body(LevelView v, ColourTasks c, double2* vec, const int64_t* voff,
                                                      int64_t ldv, int nrhs, int adj, const double2* part, int nsplit,
                                                      double2* scratch, const VBlock& VB) {
  __shared__ TileSmem<double> s;
  const int i = c.cl[VB.x];
  const int n = v.n[i], kt = v.kt[i], r = n - kt, rmax = n - v.k[i];
  if (n == 0) return;
  const int c0 = VB.z * 64, nr = min(64, nrhs - c0);
  const int ldp = c.tiles * 64;
  double2* Y = scratch + ((int64_t)VB.z * VB.gx + VB.x) * ldp * 64;
  double2* y = vec + voff[i] + (int64_t)c0 * ldv;
  const double2* P = part + ((int64_t)VB.z * VB.gx + VB.x) * nsplit * ldp * 64;
  // Y = [y[0:kt]; acc] with acc = y' - sum of the partial sums
  for (int e = threadIdx.x; e < n * nr; e += blockDim.x) {
    const int row = e % n, col = e / n;
    double2 val = y[row + (int64_t)col * ldv];
    if (row >= kt)
      for (int j = 0; j < nsplit; ++j) val = csub(val, P[(int64_t)j * ldp * 64 + (row - kt) + (int64_t)col * ldp]);
    Y[row + (int64_t)col * ldp] = val;
  }
  __syncthreads();
  if (r > 0) {
    const double2* Li = v.LU + v.lu_off[i];
    const double2* Ui = Li + (int64_t)rmax * rmax;
    // y' into the vector, then copied back into Y for the basis change
    if (!adj)
      wg_gemm(s, Ui, rmax, OP_N, Y + kt, ldp, OP_N, y + kt, ldv, r, nr, r, ST_SET);
    else
      wg_gemm(s, Li, rmax, OP_C, Y + kt, ldp, OP_N, y + kt, ldv, r, nr, r, ST_SET);
    __syncthreads();
    for (int e = threadIdx.x; e < r * nr; e += blockDim.x) {
      const int row = e % r, col = e / r;
      Y[kt + row + (int64_t)col * ldp] = y[kt + row + (int64_t)col * ldv];
    }
    __syncthreads();
  }
  const double2* Q = v.Q + v.q_off[i];
  wg_gemm(s, Q, n, adj ? OP_N : OP_R, Y, ldp, OP_N, y, ldv, n, nr, n, ST_SET);
}
__global__ void __launch_bounds__(256) k_sw_bwd_local(LevelView v, ColourTasks c, double2* vec, const int64_t* voff,
                                                      int64_t ldv, int nrhs, int adj, const double2* part, int nsplit,
                                                      double2* scratch) {
  k_sw_bwd_local_body(v, c, vec, voff, ldv, nrhs, adj, part, nsplit, scratch, vblock());
}
__global__ void __launch_bounds__(256) k_sw_bwd_local_b(const SweepEntry* E, int ne) {
  VBlock VB;
  const SweepRef e = locate_sweep(E, ne, VB);
  k_sw_bwd_local_body(e.v, e.c, e.vec, e.voff, e.ldv, e.nrhs, e.adj, e.part, e.nsplit, e.scratch, VB);
}

// ---------------------------------------------------------------------------
// Small right-hand-side counts (nrhs <= SMALL_RHS): matrix-vector products,
// coalesced along the column-major storage.
// ---------------------------------------------------------------------------
// y[0:m] = op(M) x for column-major M (m x n, ld); op N or conj (R).  All threads.
__device__ __forceinline__ double2 cfma(double2 acc, double2 a, double2 x, bool conj) {
  return cadd(acc, conj ? cmulc(a, x) : cmul(a, x));
}

// The per-cluster kernels of the 1-RHS sweeps run one 512-thread workgroup per
// cluster: at the upper levels a colour holds one to six clusters whose Q~ (up
// to n = 512) one workgroup streams alone, so the loads in flight per workgroup
// set the time.
constexpr int SV_NT = 512;
constexpr int SV_NW = SV_NT / 64;

// y[0:m] = M x (conj: conj(M) x) for column-major M (m x n, m <= 512), x in LDS.
// Lanes own rows, the SV_NW wavefronts take interleaved columns with eight
// independent loads in flight per step; partial sums meet in LDS, 64 rows at a
// time.  Every thread of the workgroup must call it (it holds barriers).
__device__ void bv_gemv_n(const double2* M, int64_t ld, int m, int n, const double2* x, double2* y, bool conj) {
  __shared__ double2 red[SV_NW][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int r0 = 0; r0 < m; r0 += 64) {
    const int r = r0 + lane;
    double2 acc = make_double2(0, 0);
    if (r < m) {
      const double2* Mr = M + r;
      int j = w;
      for (; j + 7 * SV_NW < n; j += 8 * SV_NW) {
        double2 a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) a[u] = Mr[(int64_t)(j + SV_NW * u) * ld];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = cfma(acc, a[u], x[j + SV_NW * u], conj);
      }
      for (; j < n; j += SV_NW) acc = cfma(acc, Mr[(int64_t)j * ld], x[j], conj);
    }
    red[w][lane] = acc;
    __syncthreads();
    if (threadIdx.x < 64 && r0 + (int)threadIdx.x < m) {
      double2 t = red[0][threadIdx.x];
#pragma unroll
      for (int q = 1; q < SV_NW; ++q) t = cadd(t, red[q][threadIdx.x]);
      y[r0 + threadIdx.x] = t;
    }
    __syncthreads();
  }
}

// y[0:n] = M^T x (conj: M^H x) for column-major M (m x n), x in LDS: each
// wavefront reduces eight columns at a time (loads of all eight in flight).
__device__ void bv_gemv_t(const double2* M, int64_t ld, int m, int n, const double2* x, double2* y, bool conj) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int j0 = w * 8; j0 < n; j0 += 8 * SV_NW) {
    double2 acc[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] = make_double2(0, 0);
    for (int r = lane; r < m; r += 64) {
      const double2 xv = x[r];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j0 + u < n) acc[u] = cfma(acc[u], M[r + (int64_t)(j0 + u) * ld], xv, conj);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      acc[u].x = wave_sum(acc[u].x);
      acc[u].y = wave_sum(acc[u].y);
    }
    if (lane == 0)
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (j0 + u < n) y[j0 + u] = acc[u];
  }
}

__device__ __forceinline__ void k_sv_fwd_local_body(LevelView v, ColourTasks c, double2* vec, const int64_t* voff,
                                                      int64_t ldv, int nrhs, int adj, const VBlock& VB) {
  __shared__ double2 xs[512], ys[512];
  const int i = c.cl[VB.x];
  const int n = v.n[i], kt = v.kt[i], r = n - kt, rmax = n - v.k[i];
  const double2* Q = v.Q + v.q_off[i];
  const double2* Li = v.LU + v.lu_off[i];
  const double2* Ui = Li + (int64_t)rmax * rmax;
  for (int col = 0; col < nrhs; ++col) {
    double2* b = vec + voff[i] + (int64_t)col * ldv;
    __syncthreads();
    for (int e = threadIdx.x; e < n; e += blockDim.x) xs[e] = b[e];
    __syncthreads();
    bv_gemv_t(Q, n, n, n, xs, ys, !adj);  // Q~^H b  (adj: Q~^T g)
    __syncthreads();
    for (int e = threadIdx.x; e < kt; e += blockDim.x) b[e] = ys[e];
    if (r > 0) {
      if (!adj)
        bv_gemv_n(Li, rmax, r, r, ys + kt, b + kt, false);
      else
        bv_gemv_t(Ui, rmax, r, r, ys + kt, b + kt, true);
    }
  }
}
__global__ void __launch_bounds__(SV_NT) k_sv_fwd_local(LevelView v, ColourTasks c, double2* vec, const int64_t* voff,
                                                      int64_t ldv, int nrhs, int adj) {
  k_sv_fwd_local_body(v, c, vec, voff, ldv, nrhs, adj, vblock());
}
__global__ void __launch_bounds__(SV_NT) k_sv_fwd_local_b(const SweepEntry* E, int ne) {
  VBlock VB;
  const SweepRef e = locate_sweep(E, ne, VB);
  k_sv_fwd_local_body(e.v, e.c, e.vec, e.voff, e.ldv, e.nrhs, e.adj, VB);
}

// Sum over the wavefronts' partial results of the 1-RHS gather kernels.
__device__ __forceinline__ double2 red_sum(const double2 (*red)[128], int t) {
  double2 s = red[0][t];
#pragma unroll
  for (int q = 1; q < SV_NW; ++q) s = cadd(s, red[q][t]);
  return s;
}

__device__ __forceinline__ void k_sv_fwd_gather_body(LevelView v, ColourTasks c, double2* vec, const int64_t* voff,
                                                       int64_t ldv, int nrhs, int adj, const VBlock& VB) {
  __shared__ double2 red[SV_NW][128];
  const int task = VB.x;
  const int a = c.sv_cl[task];
  const int ma = dim_after(v, a, c.colour);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int col = 0; col < nrhs; ++col) {
    for (int rb = 0; rb < ma; rb += 128) {
      double2 acc[2] = {make_double2(0, 0), make_double2(0, 0)};
      for (int e = c.sv_cptr[task]; e < c.sv_cptr[task + 1]; ++e) {
        const int i = c.sv_i[e];
        const int n = v.n[i], kt = v.kt[i], r = n - kt, rmax = n - v.k[i];
        const double2* bi = vec + voff[i] + kt + (int64_t)col * ldv;
        const int off = v.np_off[c.sv_ja[e]];
        if (!adj) {
          // rows on lanes, the r columns of C split over the wavefronts
          const int pr = v.prow[i];
          for (int h = 0; h < 2; ++h) {
            const int row = rb + h * 64 + lane;
            if (row >= ma) continue;
            const double2* C = v.CP + v.cp_off[i] + off + row;
            int q = w;
            for (; q + 3 * SV_NW < r; q += 4 * SV_NW) {
              double2 cv[4], bv[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                cv[u] = C[(int64_t)(q + SV_NW * u) * pr];
                bv[u] = bi[q + SV_NW * u];
              }
#pragma unroll
              for (int u = 0; u < 4; ++u) acc[h] = cadd(acc[h], cmul(cv[u], bv[u]));
            }
            for (; q < r; q += SV_NW) acc[h] = cadd(acc[h], cmul(C[(int64_t)q * pr], bi[q]));
          }
        } else {
          // row dot products: rows split over lanes of the wavefronts, r terms each
          const double2* R = v.RP + v.rp_off[i];
          for (int h = 0; h < 2; ++h) {
            const int row = rb + h * 64 + lane;
            if (row >= ma || w != 0) continue;
            const double2* Rc = R + (int64_t)(off + row) * rmax;
            for (int q = 0; q < r; ++q) acc[h] = cadd(acc[h], cmulc(Rc[q], bi[q]));
          }
        }
      }
      red[w][lane] = acc[0];
      red[w][64 + lane] = acc[1];
      __syncthreads();
      if (threadIdx.x < 128) {
        const int row = rb + threadIdx.x;
        if (row < ma) {
          double2 t = red_sum(red, threadIdx.x);
          double2* ba = vec + voff[a] + row + (int64_t)col * ldv;
          *ba = csub(*ba, t);
        }
      }
      __syncthreads();
    }
  }
}
__global__ void __launch_bounds__(SV_NT) k_sv_fwd_gather(LevelView v, ColourTasks c, double2* vec, const int64_t* voff,
                                                       int64_t ldv, int nrhs, int adj) {
  k_sv_fwd_gather_body(v, c, vec, voff, ldv, nrhs, adj, vblock());
}
__global__ void __launch_bounds__(SV_NT) k_sv_fwd_gather_b(const SweepEntry* E, int ne) {
  VBlock VB;
  const SweepRef e = locate_sweep(E, ne, VB);
  k_sv_fwd_gather_body(e.v, e.c, e.vec, e.voff, e.ldv, e.nrhs, e.adj, VB);
}

__device__ __forceinline__ void k_sv_bwd_partial_body(LevelView v, ColourTasks c, const double2* vec,
                                                        const int64_t* voff, int64_t ldv, int nrhs, int adj,
                                                        double2* part, int nsplit, const VBlock& VB) {
  __shared__ double2 red[SV_NW][128];
  const int i = c.cl[VB.x];
  const int n = v.n[i], kt = v.kt[i], r = n - kt, rmax = n - v.k[i];
  const int chunk = VB.y;
  const int ldp = c.tiles * 64;
  double2* P = part + ((int64_t)VB.x * nsplit + chunk) * ldp * SMALL_RHS;  // ldp x nrhs partial per chunk
  if (r <= 0) return;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int pr = v.prow[i];
  for (int col = 0; col < nrhs; ++col) {
    for (int qb = 0; qb < r; qb += 128) {
      double2 acc[2] = {make_double2(0, 0), make_double2(0, 0)};
      for (int j = v.np_ptr[i] + chunk; j < v.np_ptr[i + 1]; j += nsplit) {
        const int a = v.np_cl[j];
        const int ma = (a == i) ? kt : dim_before(v, a, c.colour);
        const double2* ya = vec + voff[a] + (int64_t)col * ldv;
        const int off = v.np_off[j];
        if (!adj) {
          const double2* R = v.RP + v.rp_off[i] + (int64_t)off * rmax;
          for (int h = 0; h < 2; ++h) {
            const int q = qb + h * 64 + lane;
            if (q >= r) continue;
            int e = w;
            for (; e + 3 * SV_NW < ma; e += 4 * SV_NW) {
              double2 rv[4], yv[4];
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                rv[u] = R[q + (int64_t)(e + SV_NW * u) * rmax];
                yv[u] = ya[e + SV_NW * u];
              }
#pragma unroll
              for (int u = 0; u < 4; ++u) acc[h] = cadd(acc[h], cmul(rv[u], yv[u]));
            }
            for (; e < ma; e += SV_NW) acc[h] = cadd(acc[h], cmul(R[q + (int64_t)e * rmax], ya[e]));
          }
        } else {
          const double2* C = v.CP + v.cp_off[i] + off;
          for (int h = 0; h < 2; ++h) {
            const int q = qb + h * 64 + lane;
            if (q >= r) continue;
            for (int e = w; e < ma; e += SV_NW) acc[h] = cadd(acc[h], cmulc(C[e + (int64_t)q * pr], ya[e]));
          }
        }
      }
      red[w][lane] = acc[0];
      red[w][64 + lane] = acc[1];
      __syncthreads();
      if (threadIdx.x < 128) {
        const int q = qb + threadIdx.x;
        if (q < r)
          P[q + (int64_t)col * ldp] =
              red_sum(red, threadIdx.x);
      }
      __syncthreads();
    }
  }
}
__global__ void __launch_bounds__(SV_NT) k_sv_bwd_partial(LevelView v, ColourTasks c, const double2* vec,
                                                        const int64_t* voff, int64_t ldv, int nrhs, int adj,
                                                        double2* part, int nsplit) {
  k_sv_bwd_partial_body(v, c, vec, voff, ldv, nrhs, adj, part, nsplit, vblock());
}
__global__ void __launch_bounds__(SV_NT) k_sv_bwd_partial_b(const SweepEntry* E, int ne) {
  VBlock VB;
  const SweepRef e = locate_sweep(E, ne, VB);
  k_sv_bwd_partial_body(e.v, e.c, e.vec, e.voff, e.ldv, e.nrhs, e.adj, e.part, e.nsplit, VB);
}

__device__ __forceinline__ void k_sv_bwd_local_body(LevelView v, ColourTasks c, double2* vec, const int64_t* voff,
                                                      int64_t ldv, int nrhs, int adj, const double2* part,
                                                      int nsplit, const VBlock& VB) {
  __shared__ double2 xs[512], ys[512];
  const int i = c.cl[VB.x];
  const int n = v.n[i], kt = v.kt[i], r = n - kt, rmax = n - v.k[i];
  const int ldp = c.tiles * 64;
  const double2* Q = v.Q + v.q_off[i];
  const double2* Li = v.LU + v.lu_off[i];
  const double2* Ui = Li + (int64_t)rmax * rmax;
  const double2* P = part + (int64_t)VB.x * nsplit * ldp * SMALL_RHS;
  for (int col = 0; col < nrhs; ++col) {
    double2* y = vec + voff[i] + (int64_t)col * ldv;
    __syncthreads();
    for (int e = threadIdx.x; e < n; e += blockDim.x) {
      double2 val = y[e];
      if (e >= kt)
        for (int j = 0; j < nsplit; ++j)
          val = csub(val, P[(int64_t)j * ldp * SMALL_RHS + (e - kt) + (int64_t)col * ldp]);
      xs[e] = val;
    }
    __syncthreads();
    if (r > 0) {
      if (!adj)
        bv_gemv_n(Ui, rmax, r, r, xs + kt, ys, false);
      else
        bv_gemv_t(Li, rmax, r, r, xs + kt, ys, true);
      __syncthreads();
      for (int e = threadIdx.x; e < r; e += blockDim.x) xs[kt + e] = ys[e];
      __syncthreads();
    }
    bv_gemv_n(Q, n, n, n, xs, y, !adj);  // conj(Q~) y  (adj: Q~ g)
  }
}
__global__ void __launch_bounds__(SV_NT) k_sv_bwd_local(LevelView v, ColourTasks c, double2* vec, const int64_t* voff,
                                                      int64_t ldv, int nrhs, int adj, const double2* part,
                                                      int nsplit) {
  k_sv_bwd_local_body(v, c, vec, voff, ldv, nrhs, adj, part, nsplit, vblock());
}
__global__ void __launch_bounds__(SV_NT) k_sv_bwd_local_b(const SweepEntry* E, int ne) {
  VBlock VB;
  const SweepRef e = locate_sweep(E, ne, VB);
  k_sv_bwd_local_body(e.v, e.c, e.vec, e.voff, e.ldv, e.nrhs, e.adj, e.part, e.nsplit, VB);
}

void launch_sweep_fwd(const LevelView& v, const ColourTasks& c, double2* vec, const int64_t* voff, int64_t ldv,
                      int nrhs, int adj, double2* scratch, hipStream_t st) {
  if (c.ncl <= 0) return;
  if (nrhs <= SMALL_RHS) {
    hipLaunchKernelGGL(k_sv_fwd_local, dim3(c.ncl), dim3(SV_NT), 0, st, v, c, vec, voff, ldv, nrhs, adj);
    if (c.nsv > 0) hipLaunchKernelGGL(k_sv_fwd_gather, dim3(c.nsv), dim3(SV_NT), 0, st, v, c, vec, voff, ldv, nrhs, adj);
    return;
  }
  const int zb = (nrhs + 63) / 64;
  hipLaunchKernelGGL(k_sw_fwd_local, dim3(c.ncl, 1, zb), dim3(256), 0, st, v, c, vec, voff, ldv, nrhs, adj, scratch);
  if (c.nsv > 0)
    hipLaunchKernelGGL(k_sw_fwd_gather, dim3(c.nsv, c.tiles, zb), dim3(256), 0, st, v, c, vec, voff, ldv, nrhs, adj);
}

void launch_sweep_bwd(const LevelView& v, const ColourTasks& c, double2* vec, const int64_t* voff, int64_t ldv,
                      int nrhs, int adj, double2* part, int nsplit, double2* scratch, hipStream_t st) {
  if (c.ncl <= 0) return;
  if (nrhs <= SMALL_RHS) {
    hipLaunchKernelGGL(k_sv_bwd_partial, dim3(c.ncl, SV_SPLIT), dim3(SV_NT), 0, st, v, c, vec, voff, ldv, nrhs, adj,
                       part, SV_SPLIT);
    hipLaunchKernelGGL(k_sv_bwd_local, dim3(c.ncl), dim3(SV_NT), 0, st, v, c, vec, voff, ldv, nrhs, adj, part, SV_SPLIT);
    return;
  }
  const int zb = (nrhs + 63) / 64;
  hipLaunchKernelGGL(k_sw_bwd_partial, dim3(c.ncl, nsplit, zb), dim3(256), 0, st, v, c, vec, voff, ldv, nrhs, adj, part,
                     nsplit);
  hipLaunchKernelGGL(k_sw_bwd_local, dim3(c.ncl, 1, zb), dim3(256), 0, st, v, c, vec, voff, ldv, nrhs, adj, part, nsplit,
                     scratch);
}

void sweep_stage_entries(int stage, const LevelView& v, const ColourTasks& c, double2* vec, const int64_t* voff,
                         int64_t ldv, int nrhs, int adj, double2* part, int nsplit, double2* scratch,
                         std::vector<std::pair<int, SweepEntry>>& out) {
  if (c.ncl <= 0) return;
  auto add = [&](int kernel, int gx, int gy, int gz, int ns) {
    if (gx <= 0 || gy <= 0 || gz <= 0) return;
    SweepEntry e;
    e.v = v;
    e.c = c;
    e.vec = vec;
    e.voff = voff;
    e.ldv = ldv;
    e.part = part;
    e.scratch = scratch;
    e.nrhs = nrhs;
    e.adj = adj;
    e.nsplit = ns;
    e.gx = gx;
    e.gy = gy;
    e.gz = gz;
    e.first = 0;
    out.emplace_back(kernel, e);
  };
  const bool small = nrhs <= SMALL_RHS;
  const int zb = (nrhs + 63) / 64;
  switch (stage) {
    case SS_FWD_LOCAL:
      if (small)
        add(SK_SV_FWD_LOCAL, c.ncl, 1, 1, 0);
      else
        add(SK_SW_FWD_LOCAL, c.ncl, 1, zb, 0);
      break;
    case SS_FWD_GATHER:
      if (c.nsv <= 0) break;
      if (small)
        add(SK_SV_FWD_GATHER, c.nsv, 1, 1, 0);
      else
        add(SK_SW_FWD_GATHER, c.nsv, c.tiles, zb, 0);
      break;
    case SS_BWD_PARTIAL:
      if (small)
        add(SK_SV_BWD_PARTIAL, c.ncl, SV_SPLIT, 1, SV_SPLIT);
      else
        add(SK_SW_BWD_PARTIAL, c.ncl, nsplit, zb, nsplit);
      break;
    case SS_BWD_LOCAL:
      if (small)
        add(SK_SV_BWD_LOCAL, c.ncl, 1, 1, SV_SPLIT);
      else
        add(SK_SW_BWD_LOCAL, c.ncl, 1, zb, nsplit);
      break;
    default:
      break;
  }
}

void launch_sweep_batched(int kernel, const SweepEntry* entries, int ne, int blocks, hipStream_t st) {
  if (ne <= 0 || blocks <= 0) return;
  const dim3 g(blocks), b256(256), bsv(SV_NT);
  switch (kernel) {
    case SK_SW_FWD_LOCAL: hipLaunchKernelGGL(k_sw_fwd_local_b, g, b256, 0, st, entries, ne); break;
    case SK_SW_FWD_GATHER: hipLaunchKernelGGL(k_sw_fwd_gather_b, g, b256, 0, st, entries, ne); break;
    case SK_SW_BWD_PARTIAL: hipLaunchKernelGGL(k_sw_bwd_partial_b, g, b256, 0, st, entries, ne); break;
    case SK_SW_BWD_LOCAL: hipLaunchKernelGGL(k_sw_bwd_local_b, g, b256, 0, st, entries, ne); break;
    case SK_SV_FWD_LOCAL: hipLaunchKernelGGL(k_sv_fwd_local_b, g, bsv, 0, st, entries, ne); break;
    case SK_SV_FWD_GATHER: hipLaunchKernelGGL(k_sv_fwd_gather_b, g, bsv, 0, st, entries, ne); break;
    case SK_SV_BWD_PARTIAL: hipLaunchKernelGGL(k_sv_bwd_partial_b, g, bsv, 0, st, entries, ne); break;
    case SK_SV_BWD_LOCAL: hipLaunchKernelGGL(k_sv_bwd_local_b, g, bsv, 0, st, entries, ne); break;
    default: break;
  }
}

// up = 1: parent vector = [kept(c1); kept(c2)] ; up = 0: children's kept parts from the parent
__global__ void k_vmerge(const int32_t* kt, const int64_t* cvoff, const int64_t* pvoff, int64_t ldc,
                         int64_t ldp, int nrhs, double2* cvec, double2* pvec, int up, const int32_t* nonempty) {
  const int p = blockIdx.x;
  const int c1 = 2 * p, c2 = 2 * p + 1;
  const int k1 = nonempty[c1] ? kt[c1] : 0, k2 = nonempty[c2] ? kt[c2] : 0;
  for (int col = 0; col < nrhs; ++col) {
    for (int e = threadIdx.x; e < k1 + k2; e += blockDim.x) {
      const int64_t ci = (e < k1) ? cvoff[c1] + e : cvoff[c2] + (e - k1);
      double2* cp = cvec + ci + col * ldc;
      double2* pp = pvec + pvoff[p] + e + col * ldp;
      if (up)
        *pp = *cp;
      else
        *cp = *pp;
    }
  }
}

void launch_vmerge(int np, const int32_t* kt, const int64_t* cvoff, const int64_t* pvoff, int64_t ldc,
                   int64_t ldp, int nrhs, double2* cvec, double2* pvec, int up, const int32_t* nonempty,
                   hipStream_t st) {
  if (np <= 0) return;
  hipLaunchKernelGGL(k_vmerge, dim3(np), dim3(128), 0, st, kt, cvoff, pvoff, ldc, ldp, nrhs, cvec, pvec, up,
                     nonempty);
}

__global__ void k_permute_in(const double2* x, int64_t ldx, const int64_t* perm, const double* scale,
                             int conj_in, int64_t N, int nrhs, double2* out, int64_t ldo) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e % N, col = e / N;
    double2 val = x[perm[t] + col * ldx];
    if (conj_in) val.y = -val.y;
    if (scale) {
      val.x *= scale[t];
      val.y *= scale[t];
    }
    out[t + col * ldo] = val;
  }
}

void launch_permute_in(const double2* x, int64_t ldx, const int64_t* perm, const double* scale, int conj_in,
                       int64_t N, int nrhs, double2* out, int64_t ldo, hipStream_t st) {
  const int64_t tot = N * nrhs;
  if (tot <= 0) return;
  int blocks = (int)imin64(4096, (tot + 255) / 256);
  hipLaunchKernelGGL(k_permute_in, dim3(blocks), dim3(256), 0, st, x, ldx, perm, scale, conj_in, N, nrhs, out,
                     ldo);
}

__global__ void k_permute_out(const double2* in, int64_t ldi, const int64_t* perm, const double* scale,
                              int conj_out, int64_t N, int nrhs, double2* y, int64_t ldy, int accumulate) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t t = e % N, col = e / N;
    double2 val = in[t + col * ldi];
    if (conj_out) val.y = -val.y;
    if (scale) {
      val.x *= scale[t];
      val.y *= scale[t];
    }
    double2* p = y + perm[t] + col * ldy;
    *p = accumulate ? cadd(*p, val) : val;
  }
}

void launch_permute_out(const double2* in, int64_t ldi, const int64_t* perm, const double* scale, int conj_out,
                        int64_t N, int nrhs, double2* y, int64_t ldy, int accumulate, hipStream_t st) {
  const int64_t tot = N * nrhs;
  if (tot <= 0) return;
  int blocks = (int)imin64(4096, (tot + 255) / 256);
  hipLaunchKernelGGL(k_permute_out, dim3(blocks), dim3(256), 0, st, in, ldi, perm, scale, conj_out, N, nrhs, y,
                     ldy, accumulate);
}

// y = M x (conj_trans = 0) or M^H x (1) for an n x n dense M; x and y distinct, ld for both.
// One workgroup per (64-row tile, 64-rhs block).
__global__ void __launch_bounds__(256) k_dense_apply(const double2* M, int64_t n, const double2* x, double2* y,
                                                     int64_t ld, int nrhs, int conj_trans) {
  __shared__ TileSmem<double> s;
  const int tr = blockIdx.x, c0 = blockIdx.y * 64;
  const int m = (int)imin64(64, n - (int64_t)tr * 64), nr = min(64, nrhs - c0);
  TileAcc<double> acc;
  acc.zero();
  const double2* A = conj_trans ? M + (int64_t)tr * 64 * n : M + tr * 64;
  gemm_tile<double, double2>(s, acc, A, n, conj_trans ? OP_C : OP_N, x + (int64_t)c0 * ld, ld, OP_N, m, nr, (int)n);
  store_tile<double, double2>(acc, y + tr * 64 + (int64_t)c0 * ld, ld, m, nr, ST_SET);
}

void launch_dense_apply(const double2* M, int64_t n, const double2* x, double2* y, int64_t ld, int nrhs,
                        int conj_trans, hipStream_t st) {
  if (n <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(k_dense_apply, dim3((unsigned)((n + 63) / 64), (nrhs + 63) / 64), dim3(256), 0, st, M, n, x, y, ld,
                     nrhs, conj_trans);
}

__global__ void k_dense_gemv(const double2* M, int64_t n, const double2* x, double2* y, int64_t ld, int nrhs,
                             int conj_trans) {
  const int col = blockIdx.y;
  for (int64_t row = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; row < n; row += (int64_t)gridDim.x * blockDim.x) {
    double2 acc = make_double2(0, 0);
    const double2* xc = x + col * ld;
    if (!conj_trans)
      for (int64_t e = 0; e < n; ++e) acc = cadd(acc, cmul(M[row + e * n], xc[e]));
    else
      for (int64_t e = 0; e < n; ++e) acc = cadd(acc, cmulc(M[e + row * n], xc[e]));
    y[row + col * ld] = acc;
  }
}

void launch_dense_gemv(const double2* M, int64_t n, const double2* x, double2* y, int64_t ld, int nrhs,
                       int conj_trans, hipStream_t st) {
  if (n <= 0 || nrhs <= 0) return;
  int blocks = (int)imin64(1024, (n + 127) / 128);
  hipLaunchKernelGGL(k_dense_gemv, dim3(blocks, nrhs), dim3(128), 0, st, M, n, x, y, ld, nrhs, conj_trans);
}

// ===========================================================================
// H^2 matrix-vector product pieces
// ===========================================================================
// Block-row GEMV y[0:m] = sum over e of M_e x_e (M_e column-major m x n_e with
// leading dimension m): lanes own rows, the four wavefronts take interleaved
// blocks, eight loads in flight per lane; partial sums meet in LDS.
template <typename BlockOf>
__device__ __forceinline__ void blockrow_gemv(int m, int e0, int e1, BlockOf blk, double2* y) {
  __shared__ double2 red[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int r0 = 0; r0 < m; r0 += 64) {
    const int row = r0 + lane;
    double2 acc = make_double2(0, 0);
    if (row < m) {
      for (int e = e0 + w; e < e1; e += 4) {
        const double2* M;
        const double2* xs;
        int ns;
        blk(e, M, xs, ns);
        M += row;
        int q = 0;
        for (; q + 7 < ns; q += 8) {
          double2 a[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) a[u] = M[(int64_t)(q + u) * m];
#pragma unroll
          for (int u = 0; u < 8; ++u) acc = cadd(acc, cmul(a[u], xs[q + u]));
        }
        for (; q < ns; ++q) acc = cadd(acc, cmul(M[(int64_t)q * m], xs[q]));
      }
    }
    red[w][lane] = acc;
    __syncthreads();
    if (threadIdx.x < 64 && row < m) y[row] = cadd(cadd(red[0][lane], red[1][lane]), cadd(red[2][lane], red[3][lane]));
    __syncthreads();
  }
}

// y_t = sum_{s in near(t)} Z_ts x_s for leaf clusters (row-cluster CSR)
__global__ void __launch_bounds__(256) k_near_mv(const int32_t* rptr, const int32_t* rcol, const int64_t* boff,
                                                 const double2* blocks, const int64_t* cstart,
                                                 const int32_t* csize, const double2* x, double2* y, int64_t ld,
                                                 int nrhs) {
  const int t = blockIdx.x;
  const int m = csize[t];
  for (int col = 0; col < nrhs; ++col)
    blockrow_gemv(m, rptr[t], rptr[t + 1],
                  [&](int e, const double2*& M, const double2*& xs, int& ns) {
                    const int s = rcol[e];
                    ns = csize[s];
                    M = blocks + boff[e];
                    xs = x + cstart[s] + col * ld;
                  },
                  y + cstart[t] + col * ld);
}

void launch_near_mv(int nc, const int32_t* rptr, const int32_t* rcol, const int64_t* boff, const double2* blocks,
                    const int64_t* cstart, const int32_t* csize, const double2* x, double2* y, int64_t ld, int nrhs,
                    hipStream_t st) {
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_near_mv, dim3(nc), dim3(256), 0, st, rptr, rcol, boff, blocks, cstart, csize, x, y, ld,
                     nrhs);
}

// trans = 1: y_t = M_t^T x_t (M_t rows x cols) ; trans = 0: y_t (+)= M_t x_t
__global__ void k_basis_mv(const int32_t* rows, const int32_t* cols, const int64_t* moff, const double2* M,
                           const int64_t* xoff, const double2* x, const int64_t* yoff, double2* y, int64_t ldx,
                           int64_t ldy, int nrhs, int trans, int accumulate) {
  const int t = blockIdx.x;
  const int m = rows[t], n = cols[t];
  const double2* Mt = M + moff[t];
  for (int col = 0; col < nrhs; ++col) {
    const double2* xt = x + xoff[t] + col * ldx;
    double2* yt = y + yoff[t] + col * ldy;
    if (trans) {
      for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double2 acc = make_double2(0, 0);
        for (int i = 0; i < m; ++i) acc = cadd(acc, cmul(Mt[i + (int64_t)j * m], xt[i]));
        yt[j] = accumulate ? cadd(yt[j], acc) : acc;
      }
    } else {
      for (int i = threadIdx.x; i < m; i += blockDim.x) {
        double2 acc = make_double2(0, 0);
        for (int j = 0; j < n; ++j) acc = cadd(acc, cmul(Mt[i + (int64_t)j * m], xt[j]));
        yt[i] = accumulate ? cadd(yt[i], acc) : acc;
      }
    }
  }
}

void launch_basis_mv(int nc, const int32_t* rows, const int32_t* cols, const int64_t* moff, const double2* M,
                     const int64_t* xoff, const double2* x, const int64_t* yoff, double2* y, int64_t ldx,
                     int64_t ldy, int nrhs, int trans, int accumulate, hipStream_t st) {
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_basis_mv, dim3(nc), dim3(128), 0, st, rows, cols, moff, M, xoff, x, yoff, y, ldx, ldy, nrhs,
                     trans, accumulate);
}

// yhat_t = sum_{s in adm(t)} S_ts xhat_s
__global__ void __launch_bounds__(256) k_coupling_mv(const int32_t* rptr, const int32_t* rcol, const int64_t* soff,
                                                     const int32_t* kr, const int32_t* kc, const double2* S,
                                                     const int64_t* xoff, const double2* x, const int64_t* yoff,
                                                     double2* y, int64_t ld, int nrhs) {
  const int t = blockIdx.x;
  const int m = kr[t];
  for (int col = 0; col < nrhs; ++col)
    blockrow_gemv(m, rptr[t], rptr[t + 1],
                  [&](int e, const double2*& M, const double2*& xs, int& ns) {
                    const int s = rcol[e];
                    ns = kc[s];
                    M = S + soff[e];
                    xs = x + xoff[s] + col * ld;
                  },
                  y + yoff[t] + col * ld);
}

void launch_coupling_mv(int nc, const int32_t* rptr, const int32_t* rcol, const int64_t* soff, const int32_t* kr,
                        const int32_t* kc, const double2* S, const int64_t* xoff, const double2* x,
                        const int64_t* yoff, double2* y, int64_t ld, int nrhs, hipStream_t st) {
  if (nc <= 0) return;
  hipLaunchKernelGGL(k_coupling_mv, dim3(nc), dim3(256), 0, st, rptr, rcol, soff, kr, kc, S, xoff, x, yoff, y, ld,
                     nrhs);
}

// ===========================================================================
// Refinement helpers
// ===========================================================================
__global__ void k_residual(const double2* b, int64_t ldb, const double2* ax, int64_t lda, double2* r, int64_t ldr,
                           int64_t N, int nrhs) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % N, c = e / N;
    r[i + c * ldr] = csub(b[i + c * ldb], ax[i + c * lda]);
  }
}

void launch_residual(const double2* b, int64_t ldb, const double2* ax, int64_t lda, double2* r, int64_t ldr,
                     int64_t N, int nrhs, hipStream_t st) {
  int blocks = (int)imin64(4096, (N * nrhs + 255) / 256);
  hipLaunchKernelGGL(k_residual, dim3(blocks), dim3(256), 0, st, b, ldb, ax, lda, r, ldr, N, nrhs);
}

__global__ void k_axpy_cols(const double2* d, int64_t ldd, double2* x, int64_t ldx, int64_t N, int nrhs) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N * nrhs;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % N, c = e / N;
    x[i + c * ldx] = cadd(x[i + c * ldx], d[i + c * ldd]);
  }
}

void launch_axpy_cols(const double2* d, int64_t ldd, double2* x, int64_t ldx, int64_t N, int nrhs,
                      hipStream_t st) {
  int blocks = (int)imin64(4096, (N * nrhs + 255) / 256);
  hipLaunchKernelGGL(k_axpy_cols, dim3(blocks), dim3(256), 0, st, d, ldd, x, ldx, N, nrhs);
}

__global__ void __launch_bounds__(256) k_col_norms(const double2* x, int64_t ld, int64_t N, double* out) {
  __shared__ double red[4];
  const int c = blockIdx.x;
  double part = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) part += cabs2(x[i + c * ld]);
  const double s = block_sum256(part, red);
  if (threadIdx.x == 0) out[c] = sqrt(s);
}

void launch_col_norms(const double2* x, int64_t ld, int64_t N, int nrhs, double* out, hipStream_t st) {
  if (nrhs <= 0) return;
  hipLaunchKernelGGL(k_col_norms, dim3(nrhs), dim3(256), 0, st, x, ld, N, out);
}

// dL/dchi_j = sum over columns of Re(conj(lam_j - g_j) x_j) / chi_j: column j
// of A is chi_j (K e_j + c e_j) + e_j, so dA/dchi_j = (A e_j - e_j) / chi_j,
// and lam^H A = g^H for lam = A^-H g.
__global__ void k_contrast_grad(const double2* x, const double2* g, const double2* lam, int64_t ld, int nrhs,
                                const double* chi, int64_t N, double* grad) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < N; j += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int c = 0; c < nrhs; ++c) {
      const int64_t e = j + (int64_t)c * ld;
      const double2 d = csub(lam[e], g[e]);
      acc += d.x * x[e].x + d.y * x[e].y;
    }
    grad[j] = acc / chi[j];
  }
}

void launch_contrast_grad(const double2* x, const double2* g, const double2* lam, int64_t ld, int nrhs,
                          const double* chi, int64_t N, double* grad, hipStream_t st) {
  if (N <= 0) return;
  const int blocks = (int)imin64(4096, (N + 255) / 256);
  hipLaunchKernelGGL(k_contrast_grad, dim3(blocks), dim3(256), 0, st, x, g, lam, ld, nrhs, chi, N, grad);
}

// ===========================================================================
// Launches shared by several independent problems: the workgroups of one launch
// are dealt to the problems' entries (BatchEntry, sorted by `first`); every kernel
// body runs exactly as in the problem's own launch.
// ===========================================================================
// The entries one problem contributes to a stage of a colour, with the grids and
// arguments its own launchers (launch_schur, launch_gram_fill, ...) would use.
void batch_stage_entries(int stage, const LevelView& v, const ColourTasks& c, bool mixed, bool mixed_flush,
                         double2* buf, int64_t aux, int i0, std::vector<std::pair<int, BatchEntry>>& out) {
  auto add = [&](int kernel, int gx, int gy, int gz, double2* b, int64_t a, int i) {
    if (gx <= 0 || gy <= 0 || gz <= 0) return;
    BatchEntry e;
    e.v = v;
    e.c = c;
    e.buf = b;
    e.aux = a;
    e.i0 = i;
    e.gx = gx;
    e.gy = gy;
    e.gz = gz;
    e.first = 0;
    out.emplace_back(kernel, e);
  };
  const int t2 = c.tiles * c.tiles;
  switch (stage) {
    case BS_SCHUR:
      if (c.nsc > 0) add(mixed_flush ? BK_SCHUR_MIXED : BK_SCHUR_FP64, c.nsc, t2, 1, nullptr, 0, 0);
      break;
    case BS_SCHUR_REDUCE:
      if (c.nsc > 0 && c.ngrp > 0) add(BK_SCHUR_REDUCE, c.ngrp, t2, 4, nullptr, 0, 0);
      break;
    case BS_GRAM:
      add(BK_GRAM_FILL, c.ncl, t2, GRAM_SPLIT, buf, aux, 0);
      break;
    case BS_GRAM_REDUCE:
      add(BK_GRAM_FILL_REDUCE, c.ncl, GRAM_RED_BLOCKS, 1, buf, aux, 0);
      break;
    case BS_XFORM0:
    case BS_XFORM1:
    case BS_XFORM2:
      add(BK_XFORM, c.ncl, t2, 1, nullptr, 0, stage - BS_XFORM0);
      break;
    case BS_STEP0: {
      const int k = i0 <= 64 ? BK_STEP0_1 : i0 <= 128 ? BK_STEP0_2 : i0 <= 256 ? BK_STEP0_4 : BK_STEP0_8;
      add(k, c.ncl, 1, 1, buf, 0, i0);
      break;
    }
    case BS_PROJ0:
      if (c.tiles == 1)
        add(mixed ? BK_PROJ_FUSED_MIXED : BK_PROJ_FUSED, c.npj, 1, 1, nullptr, 0, 0);
      else
        add(mixed ? BK_PROJ_MIXED : BK_PROJ, c.npj, t2, 1, buf, 0, 0);
      break;
    case BS_PROJ1:
      if (c.tiles > 1) add(mixed ? BK_PROJ_MIXED : BK_PROJ, c.npj, t2, 1, buf, 0, 1);
      break;
    case BS_LU:
      add(i0 <= LU_REG_MAX ? BK_LU_REG : BK_LU_BIG, c.ncl, 1, 1, buf, 0, i0);
      break;
    case BS_PANELS:
      add(BK_PANELS, c.npn, t2, 2, nullptr, 0, 0);
      break;
    default:
      break;
  }
}

void launch_batched(int kernel, const BatchEntry* entries, int ne, int blocks, hipStream_t st) {
  if (ne <= 0 || blocks <= 0) return;
  const dim3 g(blocks), b256(256);
  switch (kernel) {
    case BK_SCHUR_FP64: hipLaunchKernelGGL(k_schur_fp64_b, g, b256, 0, st, entries, ne); break;
    case BK_SCHUR_MIXED: hipLaunchKernelGGL(k_schur_mixed_b, g, b256, 0, st, entries, ne); break;
    case BK_SCHUR_REDUCE: hipLaunchKernelGGL(k_schur_reduce_b, g, b256, 0, st, entries, ne); break;
    case BK_GRAM_FILL: hipLaunchKernelGGL(k_gram_fill_b, g, b256, 0, st, entries, ne); break;
    case BK_GRAM_FILL_REDUCE: hipLaunchKernelGGL(k_gram_fill_reduce_b, g, b256, 0, st, entries, ne); break;
    case BK_XFORM: hipLaunchKernelGGL(k_xform_b, g, b256, 0, st, entries, ne); break;
    case BK_STEP0_1: hipLaunchKernelGGL(k_step0_eig_b<1>, g, dim3(S0_NT), 0, st, entries, ne); break;
    case BK_STEP0_2: hipLaunchKernelGGL(k_step0_eig_b<2>, g, dim3(S0_NT), 0, st, entries, ne); break;
    case BK_STEP0_4: hipLaunchKernelGGL(k_step0_eig_b<4>, g, dim3(S0_NT), 0, st, entries, ne); break;
    case BK_STEP0_8: hipLaunchKernelGGL(k_step0_eig_b<8>, g, dim3(S0_NT), 0, st, entries, ne); break;
    case BK_PROJ: hipLaunchKernelGGL(k_proj_b, g, b256, 0, st, entries, ne); break;
    case BK_PROJ_MIXED: hipLaunchKernelGGL(k_proj_mixed_b, g, b256, 0, st, entries, ne); break;
    case BK_PROJ_FUSED: hipLaunchKernelGGL(k_proj_fused_b, g, b256, 0, st, entries, ne); break;
    case BK_PROJ_FUSED_MIXED: hipLaunchKernelGGL(k_proj_fused_mixed_b, g, b256, 0, st, entries, ne); break;
    case BK_LU_REG: hipLaunchKernelGGL(k_lu_reg_b, g, dim3(LU_NT), 0, st, entries, ne); break;
    case BK_LU_BIG: hipLaunchKernelGGL(k_lu_big_b, g, b256, 0, st, entries, ne); break;
    case BK_PANELS: hipLaunchKernelGGL(k_panels_b, g, b256, 0, st, entries, ne); break;
    default: break;
  }
}

// ===========================================================================
// Fixed scratch of the allocation-free solve (h2_solve_noalloc): the sweep's
// per-level vectors, its final-block vectors and the backward gather's partial
// sums.  Every call on a device shares that device's copy.
// ===========================================================================
static __device__ __align__(256) double2 scratch[NOALLOC_SCRATCH_ELEMS];

double2* noalloc_scratch(hipError_t* err) {
  constexpr int MAX_DEV = 64;
  static std::mutex mu;
  static double2* ptr[MAX_DEV] = {};
  int dev = -1;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= MAX_DEV) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(mu);
  if (!ptr[dev]) {
    // the array's name in host code is only a host-side stand-in: take the
    // device address of this device's copy
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess) return nullptr;
    ptr[dev] = static_cast<double2*>(p);
  }
  *err = hipSuccess;
  return ptr[dev];
}

}  // namespace h2
