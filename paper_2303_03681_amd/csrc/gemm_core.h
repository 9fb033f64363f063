// Batched complex GEMM on CDNA4 matrix cores (FP64 16x16x4 and FP32 16x16x4).
//
// One kernel template serves every dense contraction of the method: the
// two-site product (Methods Eq. C), the site update C V^+ (Eq. Bl), the two
// halves of the transfer-matrix update sum_{ss'} sigma_{ss'} A^{s+} L A^{s'}
// (Eq. expec2) and the closing traces.  A "problem" functor supplies, per
// batch item, the sizes and the element addressing of op(A) (M x K), op(B)
// (K x N) and the output, so index permutations, conjugation and the Pauli
// letter's block swap and phase are folded into the operand fetch instead of
// being materialised.
//
// Problem interface: typedef T (compute type), Ctx (per-item state), RowA
// and ColB (per-row / per-column handles, e.g. a row pointer), constexpr
// A_CONTIG_K / B_CONTIG_N (which index is contiguous in memory, to pick a
// coalesced load order) and REAL_ONLY, plus
//   Ctx context(int item) const;   static void dims(const Ctx&, int& M, int& N, int& K);
//   static RowA rowA(const Ctx&, int i);   static ColB colB(const Ctx&, int j);
//   static C2 loadA(const Ctx&, RowA, int i, int k);  static C2 loadB(const Ctx&, ColB, int k, int j);
//   static void store(const Ctx&, int i, int j, T re, T im);
// Each thread's rows of A and columns of B are fixed for the whole K loop,
// so their handles are computed once.  The core only calls the loads and
// stores with in-range indices.
//
// Tile: BM x BN per workgroup of 256 threads (4 wave64s in a 2x2 grid, each
// wave owning (BM/2) x (BN/2) as 16x16 MFMA blocks), K staged through LDS in
// chunks of BK with the next chunk prefetched into registers.  Complex
// products use four real MFMAs (re*re - im*im, re*im + im*re) into separate
// real and imaginary accumulators; REAL_ONLY problems skip the imaginary one.
//
// MFMA operand layout (16x16x4, wave64), lane l:
//   A fragment A[l % 16][l / 16], B fragment B[l / 16][l % 16];
//   accumulator element v of lane l holds D[row][l % 16] with
//     FP32: row = 4 * (l / 16) + v,   FP64: row = 4 * v + l / 16
//   (acc_row below).  mps_selftest_mfma() checks both on the device.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace mps {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

template <typename T> struct acc_of;
template <> struct acc_of<double> { using type = d4_t; };
template <> struct acc_of<float> { using type = f4_t; };

// Row of the 16x16 block held by accumulator element v of a lane in group lk = lane / 16.
template <typename T> __device__ __forceinline__ int acc_row(int lk, int v);
template <> __device__ __forceinline__ int acc_row<double>(int lk, int v) { return 4 * v + lk; }
template <> __device__ __forceinline__ int acc_row<float>(int lk, int v) { return 4 * lk + v; }

__device__ __forceinline__ d4_t mfma_16x16x4(double a, double b, d4_t c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4_t mfma_16x16x4(float a, float b, f4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Workgroups are dispatched round-robin over the 8 XCDs.  Remap so that
// consecutive logical tiles (same batch item, sharing operand rows) land on
// the same XCD and hit its L2.  `g8` is the grid size rounded up to 8.
__device__ __forceinline__ int xcd_remap(int b, int g8) { return (b & 7) * (g8 >> 3) + (b >> 3); }

template <class P, int BM, int BN, int BK>
__global__ __launch_bounds__(256) void cgemm_kernel(P p, int tiles_m, int tiles_n, int total, int g8) {
  using T = typename P::T;
  using C2 = typename cplx_of<T>::type;
  using Acc = typename acc_of<T>::type;
  constexpr int PAD = 1;
  constexpr int NT = 256;
  constexpr int A_EL = BM * BK / NT;
  constexpr int B_EL = BK * BN / NT;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  static_assert(A_EL * NT == BM * BK && B_EL * NT == BK * BN, "tile/threads");
  static_assert(BK % 4 == 0 && WM % 16 == 0 && WN % 16 == 0, "tile shape");

  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];

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
    const int gi = m0 + ii;
    if (gi < M) ha[e] = P::rowA(ctx, gi);
  }
#pragma unroll
  for (int e = 0; e < B_EL; ++e) {
    int kk, jj;
    b_coord(e, kk, jj);
    const int gj = n0 + jj;
    if (gj < N) hb[e] = P::colB(ctx, gj);
  }
  // Tiles wholly inside M x N skip the per-element bounds checks for full
  // K-chunks (uniform per workgroup and chunk).
  const bool inside = m0 + BM <= M && n0 + BN <= N;
  auto load_tiles = [&](int k0) {
    if (inside && k0 + BK <= K) {
#pragma unroll
      for (int e = 0; e < A_EL; ++e) {
        int ii, kk;
        a_coord(e, ii, kk);
        ra[e] = P::loadA(ctx, ha[e], m0 + ii, k0 + kk);
      }
#pragma unroll
      for (int e = 0; e < B_EL; ++e) {
        int kk, jj;
        b_coord(e, kk, jj);
        rb[e] = P::loadB(ctx, hb[e], k0 + kk, n0 + jj);
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < A_EL; ++e) {
      int ii, kk;
      a_coord(e, ii, kk);
      const int gi = m0 + ii, gk = k0 + kk;
      C2 v;
      v.x = T(0);
      v.y = T(0);
      if (gi < M && gk < K) v = P::loadA(ctx, ha[e], gi, gk);
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < B_EL; ++e) {
      int kk, jj;
      b_coord(e, kk, jj);
      const int gk = k0 + kk, gj = n0 + jj;
      C2 v;
      v.x = T(0);
      v.y = T(0);
      if (gk < K && gj < N) v = P::loadB(ctx, hb[e], gk, gj);
      rb[e] = v;
    }
  };
  auto store_tiles = [&]() {
#pragma unroll
    for (int e = 0; e < A_EL; ++e) {
      int ii, kk;
      a_coord(e, ii, kk);
      As[0][kk][ii] = ra[e].x;
      As[1][kk][ii] = ra[e].y;
    }
#pragma unroll
    for (int e = 0; e < B_EL; ++e) {
      int kk, jj;
      b_coord(e, kk, jj);
      Bs[0][kk][jj] = rb[e].x;
      Bs[1][kk][jj] = rb[e].y;
    }
  };

  Acc acc_r[FM][FN], acc_i[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc_r[i][j][v] = T(0);
        acc_i[i][j][v] = T(0);
      }

  load_tiles(0);
  for (int k0 = 0; k0 < K; k0 += BK) {
    __syncthreads();
    store_tiles();
    __syncthreads();
    if (k0 + BK < K) load_tiles(k0 + BK);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T ar[FM], ai[FM], br[FN], bi[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) {
        ar[i] = As[0][kk + lk][wm + i * 16 + lr];
        ai[i] = As[1][kk + lk][wm + i * 16 + lr];
      }
#pragma unroll
      for (int j = 0; j < FN; ++j) {
        br[j] = Bs[0][kk + lk][wn + j * 16 + lr];
        bi[j] = Bs[1][kk + lk][wn + j * 16 + lr];
      }
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) {
          acc_r[i][j] = mfma_16x16x4(ar[i], br[j], acc_r[i][j]);
          acc_r[i][j] = mfma_16x16x4(-ai[i], bi[j], acc_r[i][j]);
          if (!P::REAL_ONLY) {
            acc_i[i][j] = mfma_16x16x4(ar[i], bi[j], acc_i[i][j]);
            acc_i[i][j] = mfma_16x16x4(ai[i], br[j], acc_i[i][j]);
          }
        }
    }
  }

#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm + i * 16 + acc_row<T>(lk, v);
        const int col = n0 + wn + j * 16 + lr;
        if (row < M && col < N) P::store(ctx, row, col, acc_r[i][j][v], acc_i[i][j][v]);
      }
}

// Host-side launcher: grid = items x tiles, rounded up to a multiple of 8
// for the XCD remap.
template <int BM, int BN, int BK, class P>
inline hipError_t launch_cgemm(const P& p, int items, int max_m, int max_n, hipStream_t s) {
  if (items <= 0 || max_m <= 0 || max_n <= 0) return hipSuccess;
  const int tiles_m = (max_m + BM - 1) / BM;
  const int tiles_n = (max_n + BN - 1) / BN;
  const long long total = (long long)items * tiles_m * tiles_n;
  if (total > 0x7fffff00LL) return hipErrorInvalidValue;
  const int g8 = (int)((total + 7) / 8 * 8);
  hipLaunchKernelGGL((cgemm_kernel<P, BM, BN, BK>), dim3(g8), dim3(256), 0, s, p, tiles_m, tiles_n,
                     (int)total, g8);
  return hipGetLastError();
}

}  // namespace mps
