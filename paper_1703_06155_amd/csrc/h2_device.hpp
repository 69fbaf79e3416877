// Device building blocks for gfx950: complex helpers, wavefront reductions and
// the 64x64 complex MFMA tile engine used by every batched contraction.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "h2_kernels.hpp"

namespace h2 {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename R>
struct cplx_t;
template <>
struct cplx_t<double> {
  typedef double2 type;
};
template <>
struct cplx_t<float> {
  typedef float2 type;
};

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cmulc(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// Wavefront reductions on the DPP network (no LDS round trips): quad
// permutations and row rotations combine the 16 lanes of a row, row_bcast:15 and
// row_bcast:31 carry the row results up to lane 63, whose value every lane then
// reads.  All 64 lanes must be active.
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, ROW_MASK, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double lane63_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<0xb1>(v);        // quad_perm [1,0,3,2]
  v += dpp_f64<0x4e>(v);        // quad_perm [2,3,0,1]
  v += dpp_f64<0x124>(v);       // row_ror:4
  v += dpp_f64<0x128>(v);       // row_ror:8
  v += dpp_f64<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f64<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return lane63_f64(v);
}
__device__ __forceinline__ int wave_min_int(int v) {
  v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0xb1, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x4e, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x124, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x128, 0xf, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x142, 0xa, 0xf, false));
  v = min(v, __builtin_amdgcn_update_dpp(0x7fffffff, v, 0x143, 0xc, 0xf, false));
  return __builtin_amdgcn_readlane(v, 63);
}
__device__ __forceinline__ int wave_sum_int(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0xb1, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x4e, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x124, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);
  return __builtin_amdgcn_readlane(v, 63);
}
// maximum of non-negative values (lanes outside a DPP source read 0)
__device__ __forceinline__ double wave_max_nonneg(double v) {
  v = fmax(v, dpp_f64<0xb1>(v));
  v = fmax(v, dpp_f64<0x4e>(v));
  v = fmax(v, dpp_f64<0x124>(v));
  v = fmax(v, dpp_f64<0x128>(v));
  v = fmax(v, dpp_f64<0x142, 0xa>(v));
  v = fmax(v, dpp_f64<0x143, 0xc>(v));
  return lane63_f64(v);
}

// Workgroup-wide sum for 256 threads; `red` holds >= 4 doubles of LDS.
__device__ __forceinline__ double block_sum256(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------------------
// MFMA wrappers.  The operands are passed swapped (B fragment first) so that
// the 16x16 accumulator holds C^T, i.e. 16 consecutive rows of a column-major
// C per quarter wave: lane l, element v <-> C(row = l % 16, col = acc_col(l, v)).
// The accumulator's row order differs between the two instructions (measured
// on gfx950): f64 16x16x4 interleaves rows as l / 16 + 4 v, f32 16x16x4
// blocks them as 4 (l / 16) + v.
// ---------------------------------------------------------------------------
__device__ __forceinline__ d4 mfma16(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma16(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename R>
__device__ __forceinline__ int acc_col(int lane, int v);
template <>
__device__ __forceinline__ int acc_col<double>(int lane, int v) {
  return (lane >> 4) + 4 * v;
}
template <>
__device__ __forceinline__ int acc_col<float>(int lane, int v) {
  return 4 * (lane >> 4) + v;
}

template <typename R>
struct acc_t;
template <>
struct acc_t<double> {
  typedef d4 type;
};
template <>
struct acc_t<float> {
  typedef f4 type;
};


constexpr int TM = 64;   // tile rows
constexpr int TN = 64;   // tile cols
constexpr int TK = 16;   // k step
constexpr int TPAD = 1;  // LDS row padding (elements)

template <typename R>
struct TileSmem {
  R are[TK][TM + TPAD];
  R aim[TK][TM + TPAD];
  R bre[TK][TN + TPAD];
  R bim[TK][TN + TPAD];
};

template <typename R>
struct TileAcc {
  typename acc_t<R>::type re[2][2], im[2][2];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        re[t][u] = typename acc_t<R>::type{0, 0, 0, 0};
        im[t][u] = typename acc_t<R>::type{0, 0, 0, 0};
      }
  }
};

// Per-thread staging of one TK slab: 4 elements of op(A) and 4 of op(B).
template <typename CT>
struct SlabRegs {
  CT a[4], b[4];
};

// Global -> registers for the slab starting at k0 (zero outside [0,m) x [0,K) / [0,K) x [0,n)).
template <typename CT>
__device__ __forceinline__ void slab_fetch(SlabRegs<CT>& r, const CT* __restrict__ A, int64_t lda, int opA,
                                           const CT* __restrict__ B, int64_t ldb, int opB, int m, int n, int K,
                                           int k0) {
  const int t = threadIdx.x;
  if (opA == OP_N || opA == OP_R) {
    const int i = t & 63;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + (t >> 6) + 4 * e;
      r.a[e] = (i < m && k < K) ? A[i + (int64_t)k * lda] : CT{0, 0};
    }
  } else {
    const int k = k0 + (t & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = (t >> 4) + 16 * e;
      r.a[e] = (i < m && k < K) ? A[k + (int64_t)i * lda] : CT{0, 0};
    }
  }
  if (opB == OP_N || opB == OP_R) {
    const int k = k0 + (t & 15);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = (t >> 4) + 16 * e;
      r.b[e] = (j < n && k < K) ? B[k + (int64_t)j * ldb] : CT{0, 0};
    }
  } else {
    const int j = t & 63;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int k = k0 + (t >> 6) + 4 * e;
      r.b[e] = (j < n && k < K) ? B[j + (int64_t)k * ldb] : CT{0, 0};
    }
  }
}

// Registers -> LDS in the layout mma_slab reads (conjugation applied here).
template <typename R, typename CT>
__device__ __forceinline__ void slab_store(TileSmem<R>& s, const SlabRegs<CT>& r, int opA, int opB) {
  const int t = threadIdx.x;
  const bool ca = (opA == OP_C || opA == OP_R), cb = (opB == OP_C || opB == OP_R);
  if (opA == OP_N || opA == OP_R) {
    const int i = t & 63;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int kk = (t >> 6) + 4 * e;
      s.are[kk][i] = r.a[e].x;
      s.aim[kk][i] = ca ? -r.a[e].y : r.a[e].y;
    }
  } else {
    const int kk = t & 15;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = (t >> 4) + 16 * e;
      s.are[kk][i] = r.a[e].x;
      s.aim[kk][i] = ca ? -r.a[e].y : r.a[e].y;
    }
  }
  if (opB == OP_N || opB == OP_R) {
    const int kk = t & 15;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int j = (t >> 4) + 16 * e;
      s.bre[kk][j] = r.b[e].x;
      s.bim[kk][j] = cb ? -r.b[e].y : r.b[e].y;
    }
  } else {
    const int j = t & 63;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int kk = (t >> 6) + 4 * e;
      s.bre[kk][j] = r.b[e].x;
      s.bim[kk][j] = cb ? -r.b[e].y : r.b[e].y;
    }
  }
}

// Load a 64 x TK tile of op(A) and a TK x 64 tile of op(B) straight into LDS
// (generated-entry kernels write LDS themselves and use mma_slab directly).
template <typename R, typename CT>
__device__ __forceinline__ void load_a(TileSmem<R>& s, const CT* __restrict__ A, int64_t lda, int op, int m, int K,
                                       int k0) {
  const int t = threadIdx.x;
  if (op == OP_N || op == OP_R) {
    const int i = t & 63;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int kk = (t >> 6) + 4 * e;
      const int k = k0 + kk;
      CT v{0, 0};
      if (i < m && k < K) v = A[i + (int64_t)k * lda];
      s.are[kk][i] = v.x;
      s.aim[kk][i] = (op == OP_R) ? -v.y : v.y;
    }
  } else {
    const int kk = t & 15;
    const int k = k0 + kk;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = (t >> 4) + 16 * e;
      CT v{0, 0};
      if (i < m && k < K) v = A[k + (int64_t)i * lda];
      s.are[kk][i] = v.x;
      s.aim[kk][i] = (op == OP_C) ? -v.y : v.y;
    }
  }
}

// acc += op(A_tile) * op(B_tile) for the first nk (<= TK, uniform over the
// block) k-columns of one slab resident in LDS (zero beyond its K range, so only
// whole 4-wide MFMA steps past nk are skipped).  The tile's mt x nt active 16 x 16
// output blocks (block k at row block k % mt, column block k / mt) are dealt to
// the four wavefronts in contiguous runs of ceil(mt nt / 4), so no wavefront
// carries more than that; wavefront w keeps its j-th block in accumulator slot j
// (re[j >> 1][j & 1]).
template <typename R>
__device__ __forceinline__ void mma_slab_bal(const TileSmem<R>& s, TileAcc<R>& acc, int nk, int mt, int nt) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int cnt = mt * nt, per = (cnt + 3) >> 2, k0 = w * per;
#pragma unroll
  for (int q = 0; q < TK / 4; ++q) {
    if (q * 4 >= nk) break;
    const int kk = q * 4 + lk;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kb = k0 + j;
      if (j >= per || kb >= cnt) continue;
      const int rb = kb % mt, cb = kb / mt;
      const R ar = s.are[kk][rb * 16 + li], ai = s.aim[kk][rb * 16 + li];
      const R br = s.bre[kk][cb * 16 + li], bi = s.bim[kk][cb * 16 + li];
      auto& re = acc.re[j >> 1][j & 1];
      auto& im = acc.im[j >> 1][j & 1];
      re = mfma16(br, ar, re);
      re = mfma16(bi, -ai, re);
      im = mfma16(br, ai, im);
      im = mfma16(bi, ar, im);
    }
  }
}

// C[0:m, 0:n] -= acc for the blocks mma_slab_bal assigned to this wavefront.
template <typename R, typename CT>
__device__ __forceinline__ void store_tile_bal_sub(const TileAcc<R>& acc, CT* C, int64_t ldc, int m, int n, int mt,
                                                   int nt) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int cnt = mt * nt, per = (cnt + 3) >> 2, k0 = w * per;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int kb = k0 + j;
    if (j >= per || kb >= cnt) continue;
    const int rb = kb % mt, cb = kb / mt;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = rb * 16 + (lane & 15), jj = cb * 16 + acc_col<R>(lane, v);
      if (i < m && jj < n) {
        CT* p = C + i + (int64_t)jj * ldc;
        const CT o = *p;
        *p = CT{o.x - acc.re[j >> 1][j & 1][v], o.y - acc.im[j >> 1][j & 1][v]};
      }
    }
  }
}

// C[0:m, 0:n] = acc for the blocks mma_slab_bal assigned to this wavefront
// (together the four wavefronts cover every 16 x 16 block of the m x n tile).
template <typename R, typename CT>
__device__ __forceinline__ void store_tile_bal_set(const TileAcc<R>& acc, CT* C, int64_t ldc, int m, int n, int mt,
                                                   int nt) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int cnt = mt * nt, per = (cnt + 3) >> 2, k0 = w * per;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int kb = k0 + j;
    if (j >= per || kb >= cnt) continue;
    const int rb = kb % mt, cb = kb / mt;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = rb * 16 + (lane & 15), jj = cb * 16 + acc_col<R>(lane, v);
      if (i < m && jj < n) C[i + (int64_t)jj * ldc] = CT{acc.re[j >> 1][j & 1][v], acc.im[j >> 1][j & 1][v]};
    }
  }
}

// acc += op(A)[0:m, 0:K] * op(B)[0:K, 0:n] (m, n <= 64), with the next slab's
// global loads in flight while the current slab is multiplied.
template <typename R, typename CT>
__device__ __forceinline__ void gemm_tile(TileSmem<R>& s, TileAcc<R>& acc, const CT* A, int64_t lda, int opA,
                                          const CT* B, int64_t ldb, int opB, int m, int n, int K) {
  if (K <= 0) return;
  const int mt = (m + 15) >> 4, nt = (n + 15) >> 4;
  SlabRegs<CT> r;
  slab_fetch<CT>(r, A, lda, opA, B, ldb, opB, m, n, K, 0);
  for (int k0 = 0; k0 < K; k0 += TK) {
    __syncthreads();
    slab_store<R, CT>(s, r, opA, opB);
    __syncthreads();
    if (k0 + TK < K) slab_fetch<CT>(r, A, lda, opA, B, ldb, opB, m, n, K, k0 + TK);
    mma_slab_bal<R>(s, acc, min(TK, K - k0), mt, nt);
  }
}

// C[0:m, 0:n] (op)= acc, C column-major with leading dimension ldc, for the
// 16 x 16 blocks mma_slab_bal dealt to this wavefront (the same m, n).
template <typename R, typename CT>
__device__ __forceinline__ void store_tile(const TileAcc<R>& acc, CT* C, int64_t ldc, int m, int n,
                                           int mode) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int mt = (m + 15) >> 4, nt = (n + 15) >> 4;
  const int cnt = mt * nt, per = (cnt + 3) >> 2, k0 = w * per;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int kb = k0 + j;
    if (j >= per || kb >= cnt) continue;
    const int rb = kb % mt, cb = kb / mt;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = rb * 16 + (lane & 15), jj = cb * 16 + acc_col<R>(lane, v);
      if (i < m && jj < n) {
        CT* p = C + i + (int64_t)jj * ldc;
        const R xr = acc.re[j >> 1][j & 1][v], xi = acc.im[j >> 1][j & 1][v];
        if (mode == ST_SET) {
          *p = CT{xr, xi};
        } else {
          const CT o = *p;
          if (mode == ST_ADD)
            *p = CT{o.x + xr, o.y + xi};
          else
            *p = CT{o.x - xr, o.y - xi};
        }
      }
    }
  }
}

}  // namespace h2
