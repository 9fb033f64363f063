// One two-qubit gate per workgroup, with the bond dimensions read from and
// written to device memory, so consecutive gates of a circuit queue on the
// stream without the host learning each new rank.  For bonds whose two-site
// matrix C~ is at most 128 x 128 (bond capacity <= 64 on both sides).
//
//   Eq. (C)   C = sum_{i'j'} Q B_q^{i'} B_{q+1}^{j'}          -> scratch (L2-resident)
//   Eq. (C~)  rows of lambda C, held in registers
//   Alg. 1    one-sided Jacobi on those rows until a sweep makes no rotation
//   Eq. (svd) sigma = row norms, stable descending order, truncation rank k
//   Eq. (Bl)  B_{q+1} <- V_k^+,  B_q <- C V_k / ||sigma_1..k||,  lambda <- sigma_k / ||sigma_1..k||
//
// Jacobi layout: 8 waves; wave w holds two blocks of 8 rows ("top" and
// "bottom"), each lane E elements of every row (e = lane + 64 k).  A sweep is
// a round-robin over the nb blocks: in round r the blocks at positions
// w and nb-1-w meet in wave w (position 0 fixed, the others advance by one),
// so every block pair meets once per sweep; round 0 also pairs the rows
// inside each block.  Within a wave the 64 cross pairs of its two blocks run
// as 8 sub-rounds of 8 disjoint pairs whose reductions interleave.  Between
// rounds, blocks move through LDS in two phases (tops, then bottoms), so at
// most nb/2 block slots are needed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <utility>

#include "internal.h"
#include "jacobi_ops.h"
#include "wave_ops.h"

namespace mps {

namespace {

constexpr int FW = 8;      // waves per workgroup
constexpr int FB = 8;      // rows per block
constexpr int FMAXN = 128; // rows (2 D_l) and row length (2 D_r) limit
constexpr int FVS = 65;    // LDS row stride (double2) of the staged V^+ (bank spread)

// Position p of the block round-robin in round r holds block pos_id(p, r).
__device__ __forceinline__ int pos_id(int p, int r, int nb) {
  return p == 0 ? 0 : 1 + ((p - 1 + r) % (nb - 1));
}

// Player at position p in sub-round s of the 8-player circle method.
constexpr int rr8(int p, int s) { return p == 0 ? 0 : 1 + ((p - 1 + s) % 7); }
constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a < b ? b : a; }

// ---------------------------------------------------------------------------
// Eight pairs at a time.  The 32 per-lane partial sums (x^+x, y^+y, Re x^+y,
// Im x^+y of 8 pairs) are reduce-scattered over the wave (each lane ends with
// one full sum instead of all 32), gathered so that every lane holds the four
// sums of one pair, and Algorithm 1's rotation of that pair is computed lane-
// parallel (8 pairs per instruction stream); the coefficients then go to
// scalar registers for the vector updates.

// Which register block (0 top, 1 bottom) and row each pair of a group uses.
template <int S>
struct CrossPairs {  // (top[i], bottom[(i + S) % 8])
  static constexpr int xa(int) { return 0; }
  static constexpr int xr(int i) { return i; }
  static constexpr int ya(int) { return 1; }
  static constexpr int yr(int i) { return (i + S) % FB; }
};

template <int S>
struct IntraPairs {  // circle-method sub-round S inside the top (i < 4) and bottom block
  static constexpr int xa(int i) { return i < 4 ? 0 : 1; }
  static constexpr int xr(int i) { return cmin(rr8(i % 4, S), rr8(7 - i % 4, S)); }
  static constexpr int ya(int i) { return xa(i); }
  static constexpr int yr(int i) { return cmax(rr8(i % 4, S), rr8(7 - i % 4, S)); }
};

template <int E, int A>
__device__ __forceinline__ double2 (&blk(double2 (&T)[FB][E], double2 (&B)[FB][E]))[FB][E] {
  if constexpr (A == 0) return T;
  else return B;
}

// One reduce-scatter stage: keep the half of v selected by this lane's bit,
// add the partner's copy of it (the partner keeps the other half).
template <int H>
__device__ __forceinline__ double rs_pick(const double (&v)[2 * H], int j, bool hi, bool send) {
  return (hi != send) ? v[H + j] : v[j];
}

template <int E, class P, int I>
__device__ __forceinline__ void partials_one(double2 (&T)[FB][E], double2 (&B)[FB][E], double (&v)[16]) {
  double2 (&X)[FB][E] = blk<E, P::xa(I)>(T, B);
  double2 (&Y)[FB][E] = blk<E, P::ya(I)>(T, B);
  pair_partials_xy<E>(X[P::xr(I)], Y[P::yr(I)], v[I], v[8 + I]);
}

// Tracked squared norms live in LDS, 16 per wave (wn[0..7] top rows,
// wn[8..15] bottom rows): index of row r of block A.
template <int A>
constexpr int nidx(int r) { return A * FB + r; }

// This lane's pair (lane & 7) picks its two tracked norms.
template <class P, int I>
__device__ __forceinline__ void pick_idx(int li, int& ix, int& iy) {
  if (li == I) {
    ix = nidx<P::xa(I)>(P::xr(I));
    iy = nidx<P::ya(I)>(P::yr(I));
  }
}

template <int E, class P, int I>
__device__ __forceinline__ int apply_one(double2 (&T)[FB][E], double2 (&B)[FB][E], double* wn, int lane,
                                         uint64_t act, const Rot& mine, double dn, bool x_is_i) {
  // pair I is held (real part) by lane I after the reduce-scatter
  if (!((act >> I) & 1)) return 0;
  Rot rt;
  rt.c = readlane_d(mine.c, I);
  rt.ar = readlane_d(mine.ar, I);
  rt.ai = readlane_d(mine.ai, I);
  rt.br = readlane_d(mine.br, I);
  rt.bi = readlane_d(mine.bi, I);
  const double d = readlane_d(dn, I);
  double2 (&X)[FB][E] = blk<E, P::xa(I)>(T, B);
  double2 (&Y)[FB][E] = blk<E, P::ya(I)>(T, B);
  pair_apply<E>(X[P::xr(I)], Y[P::yr(I)], rt);
  if (lane == 0) {
    wn[nidx<P::xa(I)>(P::xr(I))] += x_is_i ? d : -d;
    wn[nidx<P::ya(I)>(P::yr(I))] -= x_is_i ? d : -d;
  }
  return 1;
}

// Eight disjoint pairs with tracked squared norms: the 16 partial sums of
// x^+y are reduce-scattered (lane bits 3, 2, 1, 0 by DPP, then full sums over
// bits 4 and 5), so lane l holds component (l >> 3) & 1 (Re, Im) of pair
// l & 7; the other component comes by a swizzle and every lane computes the
// rotation of its pair (eight at once).
template <int E, class P, int... I>
__device__ __forceinline__ int rot8_impl(double2 (&T)[FB][E], double2 (&B)[FB][E], double* wn,
                                         bool x_is_i, double eps, double floor, int lane,
                                         std::integer_sequence<int, I...>) {
  double v[16];  // v[8c + i]: component c (0 Re, 1 Im) of x_i^+ y_i
  (partials_one<E, P, I>(T, B, v), ...);
  double v8[8], v4[4], v2[2];
  {
    const bool hi = (lane >> 3) & 1;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      v8[j] = rs_pick<8>(v, j, hi, false) + dpp_mov<0x140>(rs_pick<8>(v, j, hi, true));
  }
  {
    const bool hi = (lane >> 2) & 1;
#pragma unroll
    for (int j = 0; j < 4; ++j)
      v4[j] = rs_pick<4>(v8, j, hi, false) + dpp_mov<0x141>(rs_pick<4>(v8, j, hi, true));
  }
  {
    const bool hi = (lane >> 1) & 1;
#pragma unroll
    for (int j = 0; j < 2; ++j)
      v2[j] = rs_pick<2>(v4, j, hi, false) + dpp_mov<0x4E>(rs_pick<2>(v4, j, hi, true));
  }
  double x;
  {
    const bool hi = lane & 1;
    x = rs_pick<1>(v2, 0, hi, false) + dpp_mov<0xB1>(rs_pick<1>(v2, 0, hi, true));
  }
  x += swizzle<swz(16)>(x);
  x += __shfl_xor(x, 32, 64);  // the same bits in every lane that holds this sum
  const double other = swizzle<swz(8)>(x);
  const bool im_lane = (lane >> 3) & 1;
  const int li = lane & 7;
  int ix = 0, iy = 0;
  (pick_idx<P, I>(li, ix, iy), ...);
  const double bxx = wn[ix], byy = wn[iy];
  const double br = im_lane ? other : x, bi = im_lane ? x : other;
  const uint64_t act = __ballot(pair_needs_rot(bxx, byy, br, bi, eps, floor)) & 0xFFull;
  if (act == 0) return 0;  // no pair rotates: skip the rotation formula
  Rot mine{1.0, 0.0, 0.0, 0.0, 0.0};
  double dn = 0.0;
  pair_rot_coeffs(bxx, byy, br, bi, x_is_i, mine, &dn);
  return (apply_one<E, P, I>(T, B, wn, lane, act, mine, dn, x_is_i) + ...);
}

template <int E, class P>
__device__ __forceinline__ int rot8(double2 (&T)[FB][E], double2 (&B)[FB][E], double* wn, bool x_is_i,
                                    double eps, double floor, int lane) {
  return rot8_impl<E, P>(T, B, wn, x_is_i, eps, floor, lane, std::make_integer_sequence<int, 8>{});
}

template <int E, int... S>
__device__ __forceinline__ int cross_all_impl(double2 (&T)[FB][E], double2 (&B)[FB][E], double* wn,
                                              bool top_is_i, double eps, double floor, int lane,
                                              std::integer_sequence<int, S...>) {
  return (rot8<E, CrossPairs<S>>(T, B, wn, top_is_i, eps, floor, lane) + ...);
}

template <int E, int... S>
__device__ __forceinline__ int intra_all_impl(double2 (&T)[FB][E], double2 (&B)[FB][E], double* wn,
                                              double eps, double floor, int lane,
                                              std::integer_sequence<int, S...>) {
  return (rot8<E, IntraPairs<S>>(T, B, wn, true, eps, floor, lane) + ...);
}

template <int E>
__device__ __forceinline__ int cross_all(double2 (&T)[FB][E], double2 (&B)[FB][E], double* wn,
                                         bool top_is_i, double eps, double floor, int lane) {
  return cross_all_impl<E>(T, B, wn, top_is_i, eps, floor, lane, std::make_integer_sequence<int, 8>{});
}

template <int E>
__device__ __forceinline__ int intra_all(double2 (&T)[FB][E], double2 (&B)[FB][E], double* wn,
                                         double eps, double floor, int lane) {
  return intra_all_impl<E>(T, B, wn, eps, floor, lane, std::make_integer_sequence<int, 7>{});
}

// Fresh squared norms of the 16 rows a wave holds, into the wave's LDS row wn.
template <int E>
__device__ __forceinline__ void row_norms(const double2 (&T)[FB][E], const double2 (&B)[FB][E],
                                          double* wn, int lane) {
  double v[2 * FB];
#pragma unroll
  for (int t = 0; t < FB; ++t) {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      a += T[t][k].x * T[t][k].x + T[t][k].y * T[t][k].y;
      b += B[t][k].x * B[t][k].x + B[t][k].y * B[t][k].y;
    }
    v[t] = a;
    v[FB + t] = b;
  }
  wave_sum_n<2 * FB>(v);
#pragma unroll
  for (int t = 0; t < 2 * FB; ++t)
    if (lane == t) wn[t] = v[t];
}

template <int E>
__device__ __forceinline__ void blk_store(const double2 (&X)[FB][E], double2* slot, int lane) {
#pragma unroll
  for (int t = 0; t < FB; ++t)
#pragma unroll
    for (int k = 0; k < E; ++k) slot[(t * E + k) * 64 + lane] = X[t][k];
}

template <int E>
__device__ __forceinline__ void blk_load(double2 (&X)[FB][E], const double2* slot, int lane) {
#pragma unroll
  for (int t = 0; t < FB; ++t)
#pragma unroll
    for (int k = 0; k < E; ++k) X[t][k] = slot[(t * E + k) * 64 + lane];
}

// Advance the round-robin by one round: position p <- position p + 1 for
// p = 1 .. nb-2, position nb-1 <- position 1.  In waves: top(w) <- top(w+1)
// for 1 <= w <= nwa-2, top(nwa-1) <- bottom(nwa-1), bottom(w) <- bottom(w-1)
// for w >= 1, bottom(0) <- top(1); top(0) stays.  Every wave of the
// workgroup calls this (it holds the barriers).
template <int E>
__device__ __forceinline__ void advance(double2 (&T)[FB][E], double2 (&B)[FB][E], double2* xs,
                                        int wv, int nwa, int lane) {
  constexpr int SLOT = FB * 64 * E;
  __syncthreads();
  if (wv >= 1 && wv < nwa) blk_store<E>(T, xs + (size_t)(wv - 1) * SLOT, lane);
  __syncthreads();
  if (wv >= 1 && wv <= nwa - 2) blk_load<E>(T, xs + (size_t)wv * SLOT, lane);
  if (wv == nwa - 1) {
#pragma unroll
    for (int t = 0; t < FB; ++t)
#pragma unroll
      for (int k = 0; k < E; ++k) T[t][k] = B[t][k];
  }
  __syncthreads();
  if (wv <= nwa - 2) blk_store<E>(B, xs + (size_t)(wv + 1) * SLOT, lane);
  __syncthreads();
  if (wv >= 1 && wv < nwa) blk_load<E>(B, xs + (size_t)wv * SLOT, lane);
  if (wv == 0) blk_load<E>(B, xs, lane);
}

// Algorithm 1 on the rows held in T and B (nb blocks, positions as set up by
// the caller: wave w holds blocks w and nb-1-w): sweeps until one makes no
// rotation.  Returns the sweeps used, or 0 if max_sweeps were not enough.
// The block arrangement is the initial one again on return.  s_rot: two ints
// of shared memory, zero on entry; norms: FW x 16 doubles of shared memory.
// Every thread of the workgroup calls this.
template <int E>
__device__ __forceinline__ int jacobi_sweeps(double2 (&T)[FB][E], double2 (&B)[FB][E], double2* xs,
                                             int* s_rot, double* norms, int nb, int max_sweeps,
                                             double eps, double floor) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double* wn = norms + wv * 2 * FB;
  const int nwa = nb / 2;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    int rot = 0;
    for (int r = 0; r < nb - 1; ++r) {
      if (wv < nwa) {
        // squared norms, fresh for every round and then tracked through its rotations
        row_norms<E>(T, B, wn, lane);
        if (r == 0) rot += intra_all<E>(T, B, wn, eps, floor, lane);
        const bool top_is_i = pos_id(wv, r, nb) < pos_id(nb - 1 - wv, r, nb);
        rot += cross_all<E>(T, B, wn, top_is_i, eps, floor, lane);
      }
      if (nb > 2) advance<E>(T, B, xs, wv, nwa, lane);
    }
    if (lane == 0 && rot) atomicAdd(&s_rot[sw & 1], rot);
    __syncthreads();
    const int total = s_rot[sw & 1];
    __syncthreads();
    if (threadIdx.x == 0) s_rot[sw & 1] = 0;  // reused two sweeps on, after more barriers
    if (total == 0) return sw + 1;
  }
  return 0;
}

__device__ __forceinline__ void set_status(const FusedGate& g, int code) {
  g.status[1] = g.gate;
  __threadfence();
  g.status[0] = code;
}

}  // namespace

// Workgroup-shared scalars of one gate.
struct FusedShared {
  double norms[FW * 2 * FB];  // tracked squared row norms of the Jacobi sweeps
  double sig[FMAXN];
  int perm[FMAXN];
  int rank[FMAXN];
  double part[FW];
  int rot[2];
  int k;
  double inv;
  int ok;
};

// One two-qubit gate by the whole workgroup; xs is the dynamic LDS (block
// slots, then the staged V^+).  Every thread returns at the same point.
template <int E>
__device__ __forceinline__ void gate_body(const FusedGate& g, double2* xs, FusedShared& sh) {
  double* s_sig = sh.sig;
  int* s_perm = sh.perm;
  int* s_rank = sh.rank;
  double* s_part = sh.part;
  int* s_rot = sh.rot;
  int& s_k = sh.k;
  double& s_inv = sh.inv;
  int& s_ok = sh.ok;

  if (g.status[0] != 0) return;  // an earlier gate of this run failed: apply nothing
  const int Dl = g.dims[g.q], Dm = g.dims[g.q + 1], Dr = g.dims[g.q + 2];
  const int n = 2 * Dl, m = 2 * Dr;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  double2* C = g.c;

  // ---- Eq. (C): C[(i,a)][(j,r)] = sum_{i'j'} Q[2i+j][2i'+j'] (B_q^{i'} B_{q+1}^{j'})[a][r]
  double2 u[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) u[i] = g.u[i];
  for (int idx = threadIdx.x; idx < Dl * Dr; idx += FW * 64) {
    const int a = idx / Dr, r = idx - a * Dr;
    const double2* x0 = g.bq + (size_t)a * Dm;
    const double2* x1 = g.bq + (size_t)(Dl + a) * Dm;
    const double2* y0 = g.bq1 + r;
    const double2* y1 = g.bq1 + (size_t)Dm * Dr + r;
    double2 t[4] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0), make_double2(0.0, 0.0),
                    make_double2(0.0, 0.0)};
    for (int b = 0; b < Dm; ++b) {
      const double2 a0 = x0[b], a1 = x1[b], b0 = y0[(size_t)b * Dr], b1 = y1[(size_t)b * Dr];
      t[0].x += a0.x * b0.x - a0.y * b0.y; t[0].y += a0.x * b0.y + a0.y * b0.x;
      t[1].x += a0.x * b1.x - a0.y * b1.y; t[1].y += a0.x * b1.y + a0.y * b1.x;
      t[2].x += a1.x * b0.x - a1.y * b0.y; t[2].y += a1.x * b0.y + a1.y * b0.x;
      t[3].x += a1.x * b1.x - a1.y * b1.y; t[3].y += a1.x * b1.y + a1.y * b1.x;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double2 v = cmul(u[(2 * i + j) * 4 + k], t[k]);
          acc.x += v.x;
          acc.y += v.y;
        }
        C[(size_t)(i * Dl + a) * m + j * Dr + r] = acc;
      }
  }
  __syncthreads();

  // ---- Eq. (C~): rows lambda_a C[(i,a)] into registers; ||C~||_F^2 in a fixed order
  int nb = (n + FB - 1) / FB;
  nb = nb < 2 ? 2 : nb + (nb & 1);
  const int nwa = nb / 2;
  double2 T[FB][E], B[FB][E];
  double part = 0.0;
  {
    const int gt = wv * FB, gb = (nb - 1 - wv) * FB;
#pragma unroll
    for (int t = 0; t < FB; ++t)
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const int e = lane + 64 * k;
        double2 vt = make_double2(0.0, 0.0), vb = make_double2(0.0, 0.0);
        if (wv < nwa && e < m) {
          const int rt = gt + t, rb = gb + t;
          if (rt < n) {
            const double l = g.lam_l[rt % Dl];
            const double2 cv = C[(size_t)rt * m + e];
            vt = make_double2(l * cv.x, l * cv.y);
          }
          if (rb < n) {
            const double l = g.lam_l[rb % Dl];
            const double2 cv = C[(size_t)rb * m + e];
            vb = make_double2(l * cv.x, l * cv.y);
          }
        }
        T[t][k] = vt;
        B[t][k] = vb;
        part += vt.x * vt.x + vt.y * vt.y + vb.x * vb.x + vb.y * vb.y;
      }
  }
  part = wave_sum(part);
  if (lane == 0) s_part[wv] = part;
  if (threadIdx.x == 0) {
    s_rot[0] = 0;
    s_rot[1] = 0;
  }
  __syncthreads();
  double fro2 = 0.0;
#pragma unroll
  for (int w = 0; w < FW; ++w) fro2 += s_part[w];
  if (!isfinite(fro2)) {
    if (threadIdx.x == 0) set_status(g, 1);
    return;
  }
  const double eps = g.eps_scale * (double)m;
  const double floor = eps * eps * fro2;

  // ---- Algorithm 1
  const int done = jacobi_sweeps<E>(T, B, xs, s_rot, sh.norms, nb, g.max_sweeps, eps, floor);
  if (!done) {
    if (threadIdx.x == 0) set_status(g, 2);
    return;
  }

  // ---- sigma_i = ||row_i||, stable descending order, truncation
  {
    double nrm[2 * FB];
#pragma unroll
    for (int t = 0; t < FB; ++t) {
      double a = 0.0, b = 0.0;
#pragma unroll
      for (int k = 0; k < E; ++k) {
        a += T[t][k].x * T[t][k].x + T[t][k].y * T[t][k].y;
        b += B[t][k].x * B[t][k].x + B[t][k].y * B[t][k].y;
      }
      nrm[t] = a;
      nrm[FB + t] = b;
    }
    wave_sum_n<2 * FB>(nrm);
    if (wv < nwa && lane < 2 * FB) {
      double v = 0.0;
#pragma unroll
      for (int t = 0; t < 2 * FB; ++t)
        if (lane == t) v = nrm[t];
      const int row = lane < FB ? wv * FB + lane : (nb - 1 - wv) * FB + (lane - FB);
      if (row < n) s_sig[row] = sqrt(v);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += FW * 64) {
    const double si = s_sig[i];
    int rk = 0;
    for (int j = 0; j < n; ++j) {
      const double sj = s_sig[j];
      rk += (sj > si) || (sj == si && j < i);
    }
    s_perm[rk] = i;
    s_rank[i] = rk;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    bool bad = false;
    for (int a = 0; a < n; ++a) {
      const double sv = s_sig[s_perm[a]];
      if (!isfinite(sv)) bad = true;
      tot += sv * sv;
    }
    const double nrm = sqrt(tot);
    int k = 0;
    while (k < n && s_sig[s_perm[k]] > g.cutoff * nrm) ++k;
    const int capk = min(g.cap_k, min(n, m));
    if (k < 1) k = 1;
    if (k > capk) k = capk;
    double kept2 = 0.0, disc2 = 0.0;
    for (int a = 0; a < n; ++a) {
      const double sv = s_sig[s_perm[a]];
      if (a < k) kept2 += sv * sv;
      else disc2 += sv * sv;
    }
    const double kept = sqrt(kept2);
    s_ok = !(bad || !(kept > 0.0) || !isfinite(kept));
    s_inv = s_ok ? 1.0 / kept : 0.0;
    s_k = k;
    if (s_ok) {
      *g.disc += tot > 0.0 ? disc2 / tot : 0.0;
      *g.sweeps += done;
    } else {
      set_status(g, 1);
    }
  }
  __syncthreads();
  if (!s_ok) return;
  const int k = s_k;
  const double inv = s_inv;

  // ---- Eq. (Bl): B_{q+1} <- V_k^+ as [j][p][r];  lambda_{q+1} <- sigma_k / ||sigma_k||
  if (wv < nwa) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int base = h == 0 ? wv * FB : (nb - 1 - wv) * FB;
#pragma unroll
      for (int t = 0; t < FB; ++t) {
        const int row = base + t;
        if (row >= n) continue;
        const int p = s_rank[row];
        if (p >= k) continue;
        const double sv = s_sig[row];
        const double is = sv > 0.0 ? 1.0 / sv : 0.0;
#pragma unroll
        for (int kk = 0; kk < E; ++kk) {
          const int e = lane + 64 * kk;
          if (e < m) {
            const double2 x = h == 0 ? T[t][kk] : B[t][kk];
            const int j = e >= Dr ? 1 : 0, r = e - j * Dr;
            g.bq1[((size_t)j * k + p) * Dr + r] = make_double2(x.x * is, x.y * is);
          }
        }
      }
    }
  }
  for (int p = threadIdx.x; p < k; p += FW * 64) g.lam_m[p] = s_sig[s_perm[p]] * inv;

  // ---- Eq. (Bl): B_q[(i,a)][p] = inv sum_e C[(i,a)][e] conj(V^+[p][e]), 64 columns at a
  // time, V^+ read back from the rows just stored in B_{q+1}
  for (int p0 = 0; p0 < k; p0 += 64) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < m * 64; idx += FW * 64) {
      const int e = idx >> 6, pp = idx & 63, p = p0 + pp;
      double2 v = make_double2(0.0, 0.0);
      if (p < k) {
        const int j = e >= Dr ? 1 : 0, r = e - j * Dr;
        const double2 x = g.bq1[((size_t)j * k + p) * Dr + r];
        v = make_double2(x.x * inv, -x.y * inv);
      }
      xs[e * FVS + pp] = v;
    }
    __syncthreads();
    // wave w: rows 16w .. 16w+15 of B_q; lane: column p0 + lane
    const int r0 = wv * 16;
    if (r0 < n) {
      double2 acc[16];
#pragma unroll
      for (int rr = 0; rr < 16; ++rr) acc[rr] = make_double2(0.0, 0.0);
      for (int e = 0; e < m; ++e) {
        const double2 v = xs[e * FVS + lane];
#pragma unroll
        for (int rr = 0; rr < 16; ++rr) {
          const int row = min(r0 + rr, n - 1);
          const double2 cv = C[(size_t)row * m + e];
          acc[rr].x += cv.x * v.x - cv.y * v.y;
          acc[rr].y += cv.x * v.y + cv.y * v.x;
        }
      }
      const int p = p0 + lane;
      if (p < k) {
#pragma unroll
        for (int rr = 0; rr < 16; ++rr)
          if (r0 + rr < n) g.bq[(size_t)(r0 + rr) * k + p] = acc[rr];
      }
    }
  }
  if (threadIdx.x == 0) g.dims[g.q + 1] = k;
}

// Register width from the actual row length 2 D_r.
__device__ __forceinline__ void gate_any(const FusedGate& g, double2* xs, FusedShared& sh) {
  if (2 * g.dims[g.q + 2] <= 64) gate_body<1>(g, xs, sh);
  else gate_body<2>(g, xs, sh);
}

__global__ __launch_bounds__(FW * 64) void gate2q_fused_kernel(FusedGate g) {
  extern __shared__ double2 xs[];
  __shared__ FusedShared sh;
  gate_any(g, xs, sh);
}

// One step of several gate lists: workgroup f applies gate g0 + step of run
// f (Eq. 1q in place, or a two-qubit gate by gate_any) unless its list is
// exhausted or an earlier gate of the run failed.  The host enqueues the
// steps in order on one stream.
__global__ __launch_bounds__(FW * 64) void fused_step_kernel(const FusedRun* runs, int64_t step) {
  extern __shared__ double2 xs[];
  __shared__ FusedShared sh;
  const FusedRun r = runs[blockIdx.x];
  const int64_t gi = r.g0 + step;
  if (gi >= r.g1 || r.status[0] != 0) return;
  const int q = r.q0[gi];
  const double2* u = r.u + (size_t)gi * 16;
  if (r.q1[gi] < 0) {
    double2* b = r.sites[q];
    const int count = r.dims[q] * r.dims[q + 1];
    const double2 u00 = u[0], u01 = u[1], u10 = u[2], u11 = u[3];
    for (int i = threadIdx.x; i < count; i += FW * 64) {
      const double2 x0 = b[i], x1 = b[count + i];
      const double2 a = cmul(u00, x0), bb = cmul(u01, x1), c = cmul(u10, x0), d = cmul(u11, x1);
      b[i] = make_double2(a.x + bb.x, a.y + bb.y);
      b[count + i] = make_double2(c.x + d.x, c.y + d.y);
    }
    return;
  }
  const FusedGate g{r.sites[q], r.sites[q + 1], r.lam[q], r.lam[q + 1], u, r.dims, r.c, r.status,
                    r.disc, r.sweeps, q, (int)gi, r.cap[q + 1], r.max_sweeps, r.cutoff, r.eps_scale};
  gate_any(g, xs, sh);
}

// Eq. (1q) with the bond dimensions read on the device.
__global__ void gate1q_dev_kernel(double2* b, const double2* u, const int* dims, const int* status,
                                  int q) {
  if (status[0] != 0) return;
  const int count = dims[q] * dims[q + 1];
  const double2 u00 = u[0], u01 = u[1], u10 = u[2], u11 = u[3];
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    const double2 x0 = b[i], x1 = b[count + i];
    const double2 a = cmul(u00, x0), bb = cmul(u01, x1), c = cmul(u10, x0), d = cmul(u11, x1);
    b[i] = make_double2(a.x + bb.x, a.y + bb.y);
    b[count + i] = make_double2(c.x + d.x, c.y + d.y);
  }
}

// Algorithm 1 alone on matrices of at most 128 rows of at most 128 complex
// elements (one workgroup per item, all sweeps in one launch): rows it.w
// (n x m, row-major) are rotated in place; *it.sweeps_done receives the
// sweeps used, or -max_sweeps if they were not enough; ||w||_F^2 is read
// from *it.fro2.
template <int E>
__device__ __forceinline__ void jacobi_small_body(const JacItem& it, int max_sweeps, double eps_scale,
                                                  double2* xs, int* s_rot, double* norms) {
  const int n = it.n, m = it.m;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  int nb = (n + FB - 1) / FB;
  nb = nb < 2 ? 2 : nb + (nb & 1);
  const int nwa = nb / 2;
  double2 T[FB][E], B[FB][E];
#pragma unroll
  for (int t = 0; t < FB; ++t)
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int e = lane + 64 * k, rt = wv * FB + t, rb = (nb - 1 - wv) * FB + t;
      const bool ok = wv < nwa && e < m;
      T[t][k] = ok && rt < n ? it.w[(size_t)rt * m + e] : make_double2(0.0, 0.0);
      B[t][k] = ok && rb < n ? it.w[(size_t)rb * m + e] : make_double2(0.0, 0.0);
    }
  const double eps = eps_scale * (double)m;
  const double floor = eps * eps * (*it.fro2);
  const int done = jacobi_sweeps<E>(T, B, xs, s_rot, norms, nb, max_sweeps, eps, floor);
  if (wv < nwa) {
#pragma unroll
    for (int t = 0; t < FB; ++t)
#pragma unroll
      for (int k = 0; k < E; ++k) {
        const int e = lane + 64 * k, rt = wv * FB + t, rb = (nb - 1 - wv) * FB + t;
        if (e < m) {
          if (rt < n) it.w[(size_t)rt * m + e] = T[t][k];
          if (rb < n) it.w[(size_t)rb * m + e] = B[t][k];
        }
      }
  }
  if (threadIdx.x == 0) *it.sweeps_done = done > 0 ? done : -max_sweeps;
}

__global__ __launch_bounds__(FW * 64) void jacobi_small_kernel(const JacItem* items, int max_sweeps,
                                                               double eps_scale) {
  extern __shared__ double2 xs[];
  __shared__ int s_rot[2];
  __shared__ double norms[FW * 2 * FB];
  const JacItem it = items[blockIdx.x];
  if (threadIdx.x == 0) {
    s_rot[0] = 0;
    s_rot[1] = 0;
  }
  __syncthreads();
  if (it.m <= 64) jacobi_small_body<1>(it, max_sweeps, eps_scale, xs, s_rot, norms);
  else jacobi_small_body<2>(it, max_sweeps, eps_scale, xs, s_rot, norms);
}

size_t fused_lds_bytes() {
  const size_t slots = (size_t)FW * FB * 64 * 2 * sizeof(double2);
  const size_t vstage = (size_t)FMAXN * FVS * sizeof(double2);
  return std::max(slots, vstage);
}

hipError_t configure_fused_lds() {
  hipError_t e = hipFuncSetAttribute((const void*)gate2q_fused_kernel,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)fused_lds_bytes());
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute((const void*)fused_step_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                          (int)fused_lds_bytes());
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)jacobi_small_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)(FW * FB * 64 * 2 * sizeof(double2)));
}

hipError_t launch_gate2q_fused(const FusedGate& g, int max_len, hipStream_t s) {
  if (max_len > FMAXN) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gate2q_fused_kernel, dim3(1), dim3(FW * 64), fused_lds_bytes(), s, g);
  return hipGetLastError();
}

hipError_t launch_fused_step(const FusedRun* runs_dev, int n_runs, int64_t step, hipStream_t s) {
  if (n_runs <= 0) return hipSuccess;
  hipLaunchKernelGGL(fused_step_kernel, dim3(n_runs), dim3(FW * 64), fused_lds_bytes(), s, runs_dev,
                     step);
  return hipGetLastError();
}

hipError_t launch_jacobi_small(const JacItem* items_dev, int items, int max_sweeps, double eps_scale,
                               hipStream_t s) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_small_kernel, dim3(items), dim3(FW * 64), FW * FB * 64 * 2 * sizeof(double2),
                     s, items_dev, max_sweeps, eps_scale);
  return hipGetLastError();
}

hipError_t launch_gate1q_dev(double2* b, const double2* u, const int* dims, const int* status, int q,
                             int max_count, hipStream_t s) {
  const int blocks = std::max(1, std::min(64, (max_count + 255) / 256));
  hipLaunchKernelGGL(gate1q_dev_kernel, dim3(blocks), dim3(256), 0, s, b, u, dims, status, q);
  return hipGetLastError();
}

}  // namespace mps
