// Complex GEMM with FP32 operands evaluated on 16-bit matrix cores (CDNA4
// 16x16x32 bf16 / f16 MFMA) with FP32 accumulation, by splitting each FP32
// value x into a leading 16-bit part h = low(x) and a trailing part
// l = low((x - h) * S):  x ~ h + l / S.  A real product is taken as three
// MFMA products, h_a h_b + (h_a l_b + l_a h_b) / S (the l_a l_b term is below
// the precision of the split), accumulated in two FP32 accumulators.
//
//   bf16 (8-bit significand, FP32 exponent range): S = 1; about 16 significant
//        bits per operand.
//   f16 (11-bit significand, narrow exponent range): S = 2^11 keeps the
//        trailing part in the normal range; about 22 significant bits.  The
//        operands must be bounded by 1 in magnitude (true for right-canonical
//        site tensors and for transfer-matrix environments, which are images
//        of contractions); values below 2^-14 lose relative precision but keep
//        an absolute error near 2^-24.
//
// The problem functors are those of cgemm_kernel (gemm_core.h) with T = float;
// the tile loop, XCD remap and operand handles follow cgemm_kernel, with the
// split done when a staged FP32 tile is written to LDS.
//
// MFMA 16x16x32 operand layout (wave64), lane l, j = 0..7:
//   A fragment A[l % 16][8 (l / 16) + j], B fragment B[8 (l / 16) + j][l % 16],
//   accumulator element v holds D[4 (l / 16) + v][l % 16]
// (checked on the device by mps_selftest_mfma).
#pragma once

#include <hip/hip_runtime.h>

#include "gemm_core.h"

namespace mps {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));

template <typename L> struct split_traits;
template <> struct split_traits<__bf16> {
  using V8 = bf16x8_t;
  static constexpr float S = 1.0f;
  __device__ static f4_t mfma(V8 a, V8 b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct split_traits<_Float16> {
  using V8 = f16x8_t;
  static constexpr float S = 2048.0f;
  __device__ static f4_t mfma(V8 a, V8 b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

// k index of element j of lane l's A (and B) fragment; its row (column) is l % 16.
__device__ __forceinline__ int frag32_k(int lane, int j) { return 8 * (lane >> 4) + j; }

// Sign flip of all eight 16-bit values.
template <typename V8>
__device__ __forceinline__ V8 neg8(V8 v) {
  typedef unsigned int u4_t __attribute__((ext_vector_type(4)));
  u4_t u = __builtin_bit_cast(u4_t, v);
  u ^= 0x80008000u;
  return __builtin_bit_cast(V8, u);
}

template <class P, typename L, int BM, int BN>
__global__ __launch_bounds__(256) void cgemm_split_kernel(P p, int tiles_m, int tiles_n, int total,
                                                          int g8) {
  static_assert(sizeof(typename P::T) == 4, "split GEMM takes FP32 operands");
  using C2 = float2;
  using Tr = split_traits<L>;
  using V8 = typename Tr::V8;
  constexpr int BK = 32;
  constexpr int KP = BK + 8;  // LDS row length (16-bit values): rows stay 16-byte aligned
  constexpr int NT = 256;
  constexpr int A_EL = BM * BK / NT;
  constexpr int B_EL = BK * BN / NT;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  static_assert(A_EL * NT == BM * BK && B_EL * NT == BK * BN, "tile/threads");

  // [0] leading real, [1] leading imaginary, [2] trailing real, [3] trailing imaginary
  __shared__ __attribute__((aligned(16))) L As[4][BM][KP];
  __shared__ __attribute__((aligned(16))) L Bs[4][BN][KP];

  const int logical = xcd_remap(blockIdx.x, g8);
  if (logical >= total) return;
  const int per_item = tiles_m * tiles_n;
  const int item = logical / per_item;
  const int t = logical - item * per_item;
  const int tm = t / tiles_n;
  const int tn = t - tm * tiles_n;
  const typename P::Ctx ctx = p.context(item);
  int M, N, K;
  P::dims(ctx, M, N, K);
  const int m0 = tm * BM, n0 = tn * BN;
  if (m0 >= M || n0 >= N) return;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * WM;
  const int wn = (wave & 1) * WN;
  const int lr = lane & 15;
  const int lk = lane >> 4;

  C2 ra[A_EL], rb[B_EL];
  typename P::RowA ha[A_EL];
  typename P::ColB hb[B_EL];
  auto a_coord = [&](int e, int& ii, int& kk) {
    const int idx = tid + e * NT;
    if (P::A_CONTIG_K) { kk = idx % BK; ii = idx / BK; }
    else { ii = idx % BM; kk = idx / BM; }
  };
  auto b_coord = [&](int e, int& kk, int& jj) {
    const int idx = tid + e * NT;
    if (P::B_CONTIG_N) { jj = idx % BN; kk = idx / BN; }
    else { kk = idx % BK; jj = idx / BK; }
  };
#pragma unroll
  for (int e = 0; e < A_EL; ++e) {
    int ii, kk;
    a_coord(e, ii, kk);
    if (m0 + ii < M) ha[e] = P::rowA(ctx, m0 + ii);
  }
#pragma unroll
  for (int e = 0; e < B_EL; ++e) {
    int kk, jj;
    b_coord(e, kk, jj);
    if (n0 + jj < N) hb[e] = P::colB(ctx, n0 + jj);
  }
  auto load_tiles = [&](int k0) {
#pragma unroll
    for (int e = 0; e < A_EL; ++e) {
      int ii, kk;
      a_coord(e, ii, kk);
      const int gi = m0 + ii, gk = k0 + kk;
      C2 v = make_float2(0.f, 0.f);
      if (gi < M && gk < K) v = P::loadA(ctx, ha[e], gi, gk);
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < B_EL; ++e) {
      int kk, jj;
      b_coord(e, kk, jj);
      const int gk = k0 + kk, gj = n0 + jj;
      C2 v = make_float2(0.f, 0.f);
      if (gk < K && gj < N) v = P::loadB(ctx, hb[e], gk, gj);
      rb[e] = v;
    }
  };
  auto split = [](float x, L& h, L& l) {
    h = (L)x;
    l = (L)((x - (float)h) * Tr::S);
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int e = 0; e < A_EL; ++e) {
      int ii, kk;
      a_coord(e, ii, kk);
      split(ra[e].x, As[0][ii][kk], As[2][ii][kk]);
      split(ra[e].y, As[1][ii][kk], As[3][ii][kk]);
    }
#pragma unroll
    for (int e = 0; e < B_EL; ++e) {
      int kk, jj;
      b_coord(e, kk, jj);
      split(rb[e].x, Bs[0][jj][kk], Bs[2][jj][kk]);
      split(rb[e].y, Bs[1][jj][kk], Bs[3][jj][kk]);
    }
  };

  f4_t hr[FM][FN], hi[FM][FN], xr[FM][FN], xi[FM][FN];  // leading / cross accumulators
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) hr[i][j][v] = hi[i][j][v] = xr[i][j][v] = xi[i][j][v] = 0.f;

  load_tiles(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    store_tiles();
    __syncthreads();
    if (k0 + BK < K) load_tiles(k0 + BK);
    V8 a[FM][4], b[FN][4];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int c = 0; c < 4; ++c) a[i][c] = *(const V8*)&As[c][wm + i * 16 + lr][frag32_k(lane, 0)];
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) b[j][c] = *(const V8*)&Bs[c][wn + j * 16 + lr][frag32_k(lane, 0)];
#pragma unroll
    for (int i = 0; i < FM; ++i) {
      const V8 nih = neg8(a[i][1]), nil = neg8(a[i][3]);
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        // real: ar br - ai bi;  imaginary: ar bi + ai br
        hr[i][j] = Tr::mfma(a[i][0], b[j][0], hr[i][j]);
        hr[i][j] = Tr::mfma(nih, b[j][1], hr[i][j]);
        xr[i][j] = Tr::mfma(a[i][0], b[j][2], xr[i][j]);
        xr[i][j] = Tr::mfma(a[i][2], b[j][0], xr[i][j]);
        xr[i][j] = Tr::mfma(nih, b[j][3], xr[i][j]);
        xr[i][j] = Tr::mfma(nil, b[j][1], xr[i][j]);
        hi[i][j] = Tr::mfma(a[i][0], b[j][1], hi[i][j]);
        hi[i][j] = Tr::mfma(a[i][1], b[j][0], hi[i][j]);
        xi[i][j] = Tr::mfma(a[i][0], b[j][3], xi[i][j]);
        xi[i][j] = Tr::mfma(a[i][2], b[j][1], xi[i][j]);
        xi[i][j] = Tr::mfma(a[i][1], b[j][2], xi[i][j]);
        xi[i][j] = Tr::mfma(a[i][3], b[j][0], xi[i][j]);
      }
    }
  }

  constexpr float inv_s = 1.0f / Tr::S;
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm + i * 16 + acc_row<float>(lk, v);
        const int col = n0 + wn + j * 16 + lr;
        if (row < M && col < N)
          P::store(ctx, row, col, hr[i][j][v] + xr[i][j][v] * inv_s, hi[i][j][v] + xi[i][j][v] * inv_s);
      }
}

template <typename L, int BM, int BN, class P>
inline hipError_t launch_cgemm_split(const P& p, int items, int max_m, int max_n, hipStream_t s) {
  if (items <= 0 || max_m <= 0 || max_n <= 0) return hipSuccess;
  const int tiles_m = (max_m + BM - 1) / BM;
  const int tiles_n = (max_n + BN - 1) / BN;
  const long long total = (long long)items * tiles_m * tiles_n;
  if (total > 0x7fffff00LL) return hipErrorInvalidValue;
  const int g8 = (int)((total + 7) / 8 * 8);
  hipLaunchKernelGGL((cgemm_split_kernel<P, L, BM, BN>), dim3(g8), dim3(256), 0, s, p, tiles_m, tiles_n,
                     (int)total, g8);
  return hipGetLastError();
}

}  // namespace mps
