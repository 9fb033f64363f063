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
// The problem functors are those of cgemm_kernel (gemm_core.h) with T = float,
// plus loadA8 / loadB8, which fetch the eight consecutive k of one thread's
// row (column) in a full K-chunk and return the operation (SPLIT_* bits) that
// maps the split planes of the fetched values to those of the operand: a
// conjugation or a Pauli phase that is uniform over the eight values costs a
// sign flip or a swap of whole planes instead of work on every element.
// Negation and the exchange of real and imaginary parts commute exactly with
// the split, so the planes equal those of the per-element fetch (up to the
// sign of zero residuals, which no product sum sees).  The tile
// loop, XCD remap and operand handles follow cgemm_kernel, with the split done
// when a staged FP32 tile is written to LDS (8 consecutive k per thread, each
// 16-bit plane stored as one 16-byte vector), into the second of two LDS
// buffers while the matrix cores take the first.
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

typedef float f32x8_t __attribute__((ext_vector_type(8)));

// Plane operations returned by loadA8 / loadB8, applied in this order.
constexpr int SPLIT_SWAP = 1;    // exchange the real and imaginary planes
constexpr int SPLIT_NEG_RE = 2;  // negate the real planes
constexpr int SPLIT_NEG_IM = 4;  // negate the imaginary planes

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
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;

  // Two buffers; in each, [0] leading real, [1] leading imaginary, [2]
  // trailing real, [3] trailing imaginary.  While the matrix cores work on one
  // K-chunk, the next chunk is split and stored into the other buffer.
  __shared__ __attribute__((aligned(16))) L As[2][4][BM][KP];
  __shared__ __attribute__((aligned(16))) L Bs[2][4][BN][KP];

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

  // Staging: each thread moves 8 consecutive k of one row of A and one
  // column of B.  The operand's contiguous index runs across neighbouring
  // threads (so global loads coalesce), and each of the four 16-bit planes of
  // the 8 values goes to LDS as one 16-byte store.
  constexpr int KC = BK / 8;
  static_assert(BM * KC == NT && BN * KC == NT, "one row (column) and 8 k per thread");
  const int a_i = P::A_CONTIG_K ? tid / KC : tid % BM;
  const int a_k = 8 * (P::A_CONTIG_K ? tid % KC : tid / BM);
  const int b_j = P::B_CONTIG_N ? tid % BN : tid / KC;
  const int b_k = 8 * (P::B_CONTIG_N ? tid / BN : tid % KC);
  C2 ra[8], rb[8];
  int opa = 0, opb = 0;  // plane operations of the staged values
  typename P::RowA ha{};
  typename P::ColB hb{};
  if (m0 + a_i < M) ha = P::rowA(ctx, m0 + a_i);
  if (n0 + b_j < N) hb = P::colB(ctx, n0 + b_j);
  // Tiles wholly inside M x N (every tile of the saturated bonds) skip the
  // per-element bounds checks for full K-chunks; the choice is uniform per
  // workgroup and chunk.
  const bool inside = m0 + BM <= M && n0 + BN <= N;
  auto load_tiles = [&](int k0) {
    const int gi = m0 + a_i, gj = n0 + b_j;
    if (inside && k0 + BK <= K) {
      opa = P::loadA8(ctx, ha, gi, k0 + a_k, ra);
      opb = P::loadB8(ctx, hb, k0 + b_k, gj, rb);
      return;
    }
    opa = opb = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int ga = k0 + a_k + j, gb = k0 + b_k + j;
      ra[j] = (gi < M && ga < K) ? P::loadA(ctx, ha, gi, ga) : make_float2(0.f, 0.f);
      rb[j] = (gb < K && gj < N) ? P::loadB(ctx, hb, gb, gj) : make_float2(0.f, 0.f);
    }
  };
  // The eight values of each plane as one vector: paired conversions give
  // the leading parts, which are converted back exactly for the residuals.
  auto split8 = [](const C2 (&v)[8], V8& rh, V8& ih, V8& rl, V8& il) {
    f32x8_t xr, xi;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      xr[j] = v[j].x;
      xi[j] = v[j].y;
    }
    rh = __builtin_convertvector(xr, V8);
    ih = __builtin_convertvector(xi, V8);
    rl = __builtin_convertvector((xr - __builtin_convertvector(rh, f32x8_t)) * Tr::S, V8);
    il = __builtin_convertvector((xi - __builtin_convertvector(ih, f32x8_t)) * Tr::S, V8);
  };
  // op is uniform over the eight values of a thread (and, for the
  // environment problems, over a wave): negations and swaps of whole planes.
  auto plane_op = [](int op, V8& p0, V8& p1, V8& p2, V8& p3) {
    if (op & SPLIT_SWAP) {
      const V8 t0 = p0, t2 = p2;
      p0 = p1;
      p1 = t0;
      p2 = p3;
      p3 = t2;
    }
    if (op & SPLIT_NEG_RE) {
      p0 = neg8(p0);
      p2 = neg8(p2);
    }
    if (op & SPLIT_NEG_IM) {
      p1 = neg8(p1);
      p3 = neg8(p3);
    }
  };
  auto store_tiles = [&](int buf) {
    V8 p0, p1, p2, p3;
    split8(ra, p0, p1, p2, p3);
    plane_op(opa, p0, p1, p2, p3);
    *(V8*)&As[buf][0][a_i][a_k] = p0;
    *(V8*)&As[buf][1][a_i][a_k] = p1;
    *(V8*)&As[buf][2][a_i][a_k] = p2;
    *(V8*)&As[buf][3][a_i][a_k] = p3;
    split8(rb, p0, p1, p2, p3);
    plane_op(opb, p0, p1, p2, p3);
    *(V8*)&Bs[buf][0][b_j][b_k] = p0;
    *(V8*)&Bs[buf][1][b_j][b_k] = p1;
    *(V8*)&Bs[buf][2][b_j][b_k] = p2;
    *(V8*)&Bs[buf][3][b_j][b_k] = p3;
  };

  f4_t hr[FM][FN], hi[FM][FN], xr[FM][FN], xi[FM][FN];  // leading / cross accumulators
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) hr[i][j][v] = hi[i][j][v] = xr[i][j][v] = xi[i][j][v] = 0.f;

  load_tiles(0);
  store_tiles(0);
  __syncthreads();
  int cur = 0;
  for (int k0 = 0; k0 < K; k0 += BK) {
    const bool more = k0 + BK < K;
    if (more) load_tiles(k0 + BK);
    V8 a[FM][4], b[FN][4];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int c = 0; c < 4; ++c) a[i][c] = *(const V8*)&As[cur][c][wm + i * 16 + lr][frag32_k(lane, 0)];
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int c = 0; c < 4; ++c) b[j][c] = *(const V8*)&Bs[cur][c][wn + j * 16 + lr][frag32_k(lane, 0)];
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
    // the other buffer was last read before the previous barrier
    if (more) store_tiles(cur ^ 1);
    __syncthreads();
    cur ^= 1;
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
