// Device kernels of the MPS energy evaluation (gfx950).
//
//   init_product     product state B^s = delta_{s,b} (Methods, UCC: HF reference)
//   gate1q           Eq. (1q)
//   theta + mix      Eq. (C) as one batched MFMA GEMM, then the 4x4 gate mix and
//                    the lambda row scale of Eq. (C~)
//   jacobi_*         Algorithm 1 (one-sided Jacobi), block-parallel round-robin
//   finalize         sigma_i = ||a_i||, stable descending sort, truncation,
//                    normalised vectors -> B~_{q+1} = V (Eq. Bl) or canonical tensors
//   trunc            Eq. (Bl): B~_q = C V^+, an MFMA GEMM
//   canon_*          the GEMMs of the two canonicalisation sweeps
//   env_gemm1/2      Eq. (expec2) transfer update L' = sum sigma A^{s+} L A^{s'}
//   gram             closing traces Tr(L R) for all (prefix, suffix) pairs at a bond
//   energy           compensated FP64 sum_k c_k <P_k> in string order
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "gemm_core.h"
#include "gemm_split.h"
#include "internal.h"
#include "jacobi_ops.h"
#include "wave_ops.h"

namespace mps {

namespace {

inline int cdiv(long long a, long long b) { return (int)((a + b - 1) / b); }

}  // namespace

// =================================================================== state

__global__ void init_product_kernel(double2* const* sites, double* const* lam, const uint8_t* bits,
                                    int n) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) {
    const int b = bits[q] ? 1 : 0;
    sites[q][0] = make_double2(b == 0 ? 1.0 : 0.0, 0.0);
    sites[q][1] = make_double2(b == 1 ? 1.0 : 0.0, 0.0);
  }
  if (q <= n) lam[q][0] = 1.0;
}

hipError_t launch_init_product(double2* const* sites, double* const* lam0, const uint8_t* bits,
                               int n, hipStream_t s) {
  hipLaunchKernelGGL(init_product_kernel, dim3(cdiv(n + 1, 256)), dim3(256), 0, s, sites, lam0,
                     bits, n);
  return hipGetLastError();
}

// Eq. (1q): B^s <- sum_s' Q_{ss'} B^{s'}; count = Dl * Dr elements per physical index.
__global__ void gate1q_kernel(double2* b, const double2* u, int count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double2 x0 = b[i], x1 = b[count + i];
  const double2 u00 = u[0], u01 = u[1], u10 = u[2], u11 = u[3];
  const double2 a = cmul(u00, x0), bb = cmul(u01, x1), c = cmul(u10, x0), d = cmul(u11, x1);
  b[i] = make_double2(a.x + bb.x, a.y + bb.y);
  b[count + i] = make_double2(c.x + d.x, c.y + d.y);
}

hipError_t launch_gate1q(double2* b, const double2* u, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(gate1q_kernel, dim3(cdiv(count, 256)), dim3(256), 0, s, b, u, count);
  return hipGetLastError();
}

// =================================================================== Eq. (C)

struct ThetaP {
  using T = double;
  using Ctx = ThetaItem;
  static constexpr bool A_CONTIG_K = true, B_CONTIG_N = true, REAL_ONLY = false;
  const ThetaItem* items;
  __device__ Ctx context(int i) const { return items[i]; }
  __device__ static void dims(const Ctx& c, int& M, int& N, int& K) {
    M = 2 * c.dl;
    N = 2 * c.dr;
    K = c.dm;
  }
  using RowA = const double2*;
  using ColB = const double2*;
  __device__ static RowA rowA(const Ctx& c, int i) { return c.bl + (size_t)i * c.dm; }
  __device__ static ColB colB(const Ctx& c, int j) {
    const int s = j >= c.dr;
    return c.br + (size_t)s * c.dm * c.dr + (j - s * c.dr);
  }
  __device__ static double2 loadA(const Ctx&, RowA r, int, int k) { return r[k]; }
  __device__ static double2 loadB(const Ctx& c, ColB b, int k, int) { return b[(size_t)k * c.dr]; }
  __device__ static void store(const Ctx& c, int i, int j, double re, double im) {
    c.theta[(size_t)i * (2 * c.dr) + j] = make_double2(re, im);
  }
};

hipError_t launch_theta(const ThetaItem* items_dev, int items, int max_rows, int max_cols,
                        hipStream_t s) {
  ThetaP p{items_dev};
  return launch_cgemm<64, 64, 16>(p, items, max_rows, max_cols, s);
}

// C^{t1 t2}_{l r} = sum_{s1 s2} Q[(t1 t2),(s1 s2)] Theta[(s1,l),(s2,r)]  (Eq. C)
// W = lambda_l C                                                       (Eq. C~)
// One thread per (l, r); ||W||_F^2 accumulated per item.
__global__ __launch_bounds__(256) void mix_kernel(const MixItem* items, int per_item_blocks) {
  const int item = blockIdx.x / per_item_blocks;
  const int blk = blockIdx.x - item * per_item_blocks;
  const MixItem it = items[item];
  const int dl = it.dl, dr = it.dr;
  const int idx = blk * 256 + threadIdx.x;
  double local = 0.0;
  if (idx < dl * dr) {
    const int l = idx / dr, r = idx - (idx / dr) * dr;
    const size_t ld = 2 * (size_t)dr;
    double2 th[4];
#pragma unroll
    for (int s1 = 0; s1 < 2; ++s1)
#pragma unroll
      for (int s2 = 0; s2 < 2; ++s2) th[s1 * 2 + s2] = it.c[(size_t)(s1 * dl + l) * ld + s2 * dr + r];
    const double lam = it.lam[l];
#pragma unroll
    for (int t1 = 0; t1 < 2; ++t1)
#pragma unroll
      for (int t2 = 0; t2 < 2; ++t2) {
        double2 acc = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double2 v = cmul(it.q[(t1 * 2 + t2) * 4 + k], th[k]);
          acc.x += v.x;
          acc.y += v.y;
        }
        const size_t o = (size_t)(t1 * dl + l) * ld + t2 * dr + r;
        it.c[o] = acc;
        const double2 wv = make_double2(lam * acc.x, lam * acc.y);
        it.w[o] = wv;
        local += wv.x * wv.x + wv.y * wv.y;
      }
  }
  local = wave_sum(local);
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = local;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(it.fro2, part[0] + part[1] + part[2] + part[3]);
}

hipError_t launch_mix(const MixItem* items_dev, int items, int max_dldr, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  const int per = cdiv(max_dldr, 256);
  hipLaunchKernelGGL(mix_kernel, dim3(items * per), dim3(256), 0, s, items_dev, per);
  return hipGetLastError();
}

// =================================================================== Algorithm 1

// Rotate local vectors i and j (one wave): b_ii, b_jj, b_ij by wave
// reductions, then, if |b_ij| > eps sqrt(b_ii b_jj) and |b_ij| > floor,
//   tau = (b_ii - b_jj) / (2|b_ij|), t = sign(tau) / (|tau| + sqrt(1 + tau^2)),
//   c = 1/sqrt(1+t^2), s = t c, e = b_ij / |b_ij|,
//   a_i <- c a_i + s conj(e) a_j,   a_j <- c a_j - s e a_i.
__device__ __forceinline__ bool jacobi_pair(double2* xi, double2* xj, int m, int lane, double eps,
                                            double floor) {
  double bii = 0.0, bjj = 0.0, br = 0.0, bi = 0.0;
  for (int e = lane; e < m; e += 64) {
    const double2 a = xi[e], b = xj[e];
    bii += a.x * a.x + a.y * a.y;
    bjj += b.x * b.x + b.y * b.y;
    br += a.x * b.x + a.y * b.y;
    bi += a.x * b.y - a.y * b.x;
  }
  bii = wave_sum(bii);
  bjj = wave_sum(bjj);
  br = wave_sum(br);
  bi = wave_sum(bi);
  const double mag = sqrt(br * br + bi * bi);
  if (!(mag > floor) || !(mag > eps * sqrt(bii * bjj))) return false;
  const double tau = (bii - bjj) / (2.0 * mag);
  const double at = fabs(tau);
  const double sg = tau >= 0.0 ? 1.0 : -1.0;
  const double t = at > 1e100 ? sg * (0.5 / at) : sg / (at + sqrt(1.0 + tau * tau));
  const double c = 1.0 / sqrt(1.0 + t * t);
  const double s = t * c;
  const double er = br / mag, ei = bi / mag;
  for (int e = lane; e < m; e += 64) {
    const double2 a = xi[e], b = xj[e];
    // conj(e) b and e a
    const double cbr = er * b.x + ei * b.y, cbi = er * b.y - ei * b.x;
    const double ear = er * a.x - ei * a.y, eai = er * a.y + ei * a.x;
    xi[e] = make_double2(c * a.x + s * cbr, c * a.y + s * cbi);
    xj[e] = make_double2(c * b.x - s * ear, c * b.y - s * eai);
  }
  return true;
}

// One sweep over all pairs of the nloc local vectors in round-robin order
// (nloc - 1 rounds of nloc/2 disjoint pairs, one pair per wave at a time).
// gidx gives each local vector's global index (-1 = absent); pairs are
// oriented so the lower global index plays the role of i.
__device__ int jacobi_local_sweep(double2* sm, const int* gidx, int nloc, int m, double eps,
                                  double floor, int* s_rot) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int nwaves = blockDim.x >> 6;
  if (threadIdx.x == 0) *s_rot = 0;
  __syncthreads();
  for (int ir = 0; ir < nloc - 1; ++ir) {
    for (int pp = wave; pp < nloc / 2; pp += nwaves) {
      int i = (pp == 0) ? 0 : 1 + ((pp - 1 + ir) % (nloc - 1));
      int j = 1 + ((nloc - 2 - pp + ir) % (nloc - 1));
      const int gi = gidx[i], gj = gidx[j];
      if (gi < 0 || gj < 0) continue;
      if (gi > gj) {
        const int tmp = i;
        i = j;
        j = tmp;
      }
      if (jacobi_pair(sm + (size_t)i * m, sm + (size_t)j * m, m, lane, eps, floor) && lane == 0)
        atomicAdd(s_rot, 1);
    }
    __syncthreads();
  }
  return *s_rot;
}

// Block mode: one workgroup per block pair of round `round`; the pair's
// 2*wblk vectors are staged in LDS, swept once, and written back.  Each block
// is a contiguous run of vectors, so staging is two flat, coalesced copies.
__global__ __launch_bounds__(512) void jacobi_block_kernel(const JacItem* items, int max_pairs,
                                                           int round, int sweep, double eps_scale) {
  extern __shared__ double2 sm[];
  __shared__ int gidx[256];
  __shared__ int s_rot;
  const int item = blockIdx.x / max_pairs;
  const int p = blockIdx.x - item * max_pairs;
  const JacItem it = items[item];
  const int nb = it.nb;
  if (p >= nb / 2 || round >= nb - 1) return;
  if (sweep > 0 && it.rot[(sweep - 1) * it.rot_stride] == 0) return;  // converged
  const int w = it.wblk, m = it.m, n = it.n;
  const int bp = (p == 0) ? 0 : 1 + ((p - 1 + round) % (nb - 1));
  const int bq = 1 + ((nb - 2 - p + round) % (nb - 1));
  const int nloc = 2 * w;
  for (int lv = threadIdx.x; lv < nloc; lv += blockDim.x) {
    const int g = lv < w ? bp * w + lv : bq * w + (lv - w);
    gidx[lv] = g < n ? g : -1;
  }
  const int vp = max(0, min(w, n - bp * w)), vq = max(0, min(w, n - bq * w));
  const size_t cp = (size_t)vp * m, cq = (size_t)vq * m, wm = (size_t)w * m;
  const double2* srcp = it.w + (size_t)bp * w * m;
  const double2* srcq = it.w + (size_t)bq * w * m;
#pragma unroll 4
  for (size_t i = threadIdx.x; i < wm; i += 512) sm[i] = i < cp ? srcp[i] : make_double2(0.0, 0.0);
#pragma unroll 4
  for (size_t i = threadIdx.x; i < wm; i += 512) sm[wm + i] = i < cq ? srcq[i] : make_double2(0.0, 0.0);
  __syncthreads();
  const double eps = eps_scale * (double)m;
  const double floor = eps * eps * (*it.fro2);
  const int rot = jacobi_local_sweep(sm, gidx, nloc, m, eps, floor, &s_rot);
  if (rot > 0) {
    double2* dstp = it.w + (size_t)bp * w * m;
    double2* dstq = it.w + (size_t)bq * w * m;
#pragma unroll 4
    for (size_t i = threadIdx.x; i < cp; i += 512) dstp[i] = sm[i];
#pragma unroll 4
    for (size_t i = threadIdx.x; i < cq; i += 512) dstq[i] = sm[wm + i];
    if (threadIdx.x == 0) atomicAdd(&it.rot[sweep * it.rot_stride], rot);
  }
}

// ---------------------------------------------------------------------------
// Register-resident block Jacobi on blocks of JW = 8 vectors; each lane keeps
// E elements (e = lane + 64 k) of the vectors its wave holds, so dot products
// and rotations never touch LDS.  A sweep is one launch for the 28 pairs
// inside every block (circle method, both vectors of a wave move each inner
// round), then one launch per outer round of the block round-robin, each
// pairing every block with exactly one other and taking the 64 cross pairs
// of the two (resident vectors stay, travellers move one wave along per
// inner round).  Over one sweep every pair of the matrix is visited once.
constexpr int JW = 8;

template <int E>
struct RegVec {
  double2 v[E];
};

// Row pointers of the Jacobi work matrices are global memory: typed so, the
// loads and stores are global (not flat) instructions with immediate offsets.
typedef double __attribute__((ext_vector_type(2))) dvec2;
typedef __attribute__((address_space(1))) dvec2 gdvec2;

// Every lane loads (unconditionally, from inside the row: indices past the
// row end are clamped to its last element; src is always a row of the
// matrix) and zeroes what lies outside the row or belongs to a padding row,
// so the loads need no branches.
template <int E>
__device__ __forceinline__ void rv_load(RegVec<E>& r, const double2* src, int valid, int m, int lane) {
  const gdvec2* g = (const gdvec2*)src;
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int e = lane + 64 * k;
    const dvec2 v = g[e < m ? e : m - 1];
    const bool keep = valid && e < m;
    r.v[k] = make_double2(keep ? v.x : 0.0, keep ? v.y : 0.0);
  }
}

template <int E>
__device__ __forceinline__ void rv_store(const RegVec<E>& r, double2* dst, int m, int lane) {
  gdvec2* g = (gdvec2*)dst;
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const int e = lane + 64 * k;
    if (e < m) g[e] = dvec2{r.v[k].x, r.v[k].y};
  }
}

template <int E>
__device__ __forceinline__ void rv_to_lds(const RegVec<E>& r, double2* slot, int lane) {
#pragma unroll
  for (int k = 0; k < E; ++k) slot[64 * k + lane] = r.v[k];
}

template <int E>
__device__ __forceinline__ void rv_from_lds(RegVec<E>& r, const double2* slot, int lane) {
#pragma unroll
  for (int k = 0; k < E; ++k) r.v[k] = slot[64 * k + lane];
}

// Algorithm 1's pair step on register vectors x and y; the one with the lower
// global index plays a_i.  One code path for both orientations:
//   x' = c x + alpha y,  y' = c y + beta x  with (alpha, beta) =
//   (s conj(e), -s e) if x is a_i, (-s e, s conj(e)) if y is a_i.
template <int E>
__device__ __forceinline__ bool jacobi_pair_ordered(RegVec<E>& x, int gx, RegVec<E>& y, int gy,
                                                    double eps, double floor) {
  if (gx < 0 || gy < 0) return false;
  double bxx = 0.0, byy = 0.0, br = 0.0, bi = 0.0;  // x^+ x, y^+ y, x^+ y
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const double2 a = x.v[k], b = y.v[k];
    bxx += a.x * a.x + a.y * a.y;
    byy += b.x * b.x + b.y * b.y;
    br += a.x * b.x + a.y * b.y;
    bi += a.x * b.y - a.y * b.x;
  }
  bxx = wave_sum(bxx);
  byy = wave_sum(byy);
  br = wave_sum(br);
  bi = wave_sum(bi);
  const bool x_is_i = gx < gy;
  const double bii = x_is_i ? bxx : byy, bjj = x_is_i ? byy : bxx;
  const double mag = sqrt(br * br + bi * bi);
  if (!(mag > floor) || !(mag > eps * sqrt(bii * bjj))) return false;
  const double tau = (bii - bjj) / (2.0 * mag);
  const double at = fabs(tau);
  const double sg = tau >= 0.0 ? 1.0 : -1.0;
  const double t = at > 1e100 ? sg * (0.5 / at) : sg / (at + sqrt(1.0 + tau * tau));
  const double c = 1.0 / sqrt(1.0 + t * t);
  const double s = t * c;
  // e = b_ij / |b_ij| with b_ij = x^+ y (x is a_i) or y^+ x = conj(x^+ y)
  const double er = br / mag, ei = x_is_i ? bi / mag : -bi / mag;
  // s conj(e) and -s e
  const double pr = s * er, pi = -s * ei, qr = -s * er, qi = -s * ei;
  const double ar = wave_uniform(x_is_i ? pr : qr), ai = wave_uniform(x_is_i ? pi : qi);
  const double brr = wave_uniform(x_is_i ? qr : pr), bri = wave_uniform(x_is_i ? qi : pi);
  const double cu = wave_uniform(c);
#pragma unroll
  for (int k = 0; k < E; ++k) {
    const double2 a = x.v[k], b = y.v[k];
    x.v[k] = make_double2(cu * a.x + (ar * b.x - ai * b.y), cu * a.y + (ar * b.y + ai * b.x));
    y.v[k] = make_double2(cu * b.x + (brr * a.x - bri * a.y), cu * b.y + (brr * a.y + bri * a.x));
  }
  return true;
}

// Common prologue of the register kernels: which block pair this workgroup
// owns, or false if it has nothing to do (padding pair, converged item).
struct RegCtx {
  JacItem it;
  int bp, bq;
  double eps, floor;
};

__device__ __forceinline__ bool reg_prologue(const JacItem* items, int max_pairs, int round,
                                             int sweep, double eps_scale, RegCtx& c) {
  const int item = blockIdx.x / max_pairs;
  const int p = blockIdx.x - item * max_pairs;
  c.it = items[item];
  const int nb = c.it.nb;
  if (p >= nb / 2 || round >= nb - 1) return false;
  if (sweep > 0 && c.it.rot[(sweep - 1) * c.it.rot_stride] == 0) return false;  // converged
  c.bp = (p == 0) ? 0 : 1 + ((p - 1 + round) % (nb - 1));
  c.bq = 1 + ((nb - 2 - p + round) % (nb - 1));
  c.eps = eps_scale * (double)c.it.m;
  c.floor = c.eps * c.eps * (*c.it.fro2);
  return true;
}

template <int E>
__device__ __forceinline__ void reg_epilogue(const RegCtx& c, int rot, int* s_rot, const RegVec<E>& x,
                                             int gx, const RegVec<E>& y, int gy, int sweep) {
  const int lane = threadIdx.x & 63;
  if (lane == 0 && rot) atomicAdd(s_rot, rot);
  __syncthreads();
  if (*s_rot > 0) {
    if (gx >= 0) rv_store<E>(x, c.it.w + (size_t)gx * c.it.m, c.it.m, lane);
    if (gy >= 0) rv_store<E>(y, c.it.w + (size_t)gy * c.it.m, c.it.m, lane);
    if (threadIdx.x == 0) atomicAdd(&c.it.rot[sweep * c.it.rot_stride], *s_rot);
  }
}

// Circle method over the 2W rows that W waves hold (wave w: positions w and
// 2W - 1 - w): every pair of them is visited once in 2W - 1 steps; after
// each step positions 1..2W-1 advance by one through 2 x W LDS slots
// (position 0 fixed), in C chunks of E / C elements per lane so that the
// slots take 2 W 64 (E / C) elements.  gx, gy follow the rows (global
// indices, -1 padding).
template <int E, int W, int C>
__device__ __forceinline__ int circle_pairs(RegVec<E>& x, int& gx, RegVec<E>& y, int& gy, double2* slots,
                                            int* g_top, int* g_bot, double eps, double floor, int lane,
                                            int wv) {
  static_assert(E % C == 0, "chunks must divide the elements per lane");
  constexpr int EC = E / C;
  double2* top = slots;
  double2* bot = slots + (size_t)W * 64 * EC;
  int rot = 0;
  for (int t = 0; t < 2 * W - 1; ++t) {
    rot += jacobi_pair_ordered<E>(x, gx, y, gy, eps, floor);
    int nx = gx, ny = gy;
#pragma unroll
    for (int c = 0; c < C; ++c) {
#pragma unroll
      for (int k = 0; k < EC; ++k) {
        top[((size_t)wv * EC + k) * 64 + lane] = x.v[c * EC + k];
        bot[((size_t)wv * EC + k) * 64 + lane] = y.v[c * EC + k];
      }
      if (c == 0 && lane == 0) {
        g_top[wv] = gx;
        g_bot[wv] = gy;
      }
      __syncthreads();
      // new pos j+1 <- old pos j for j = 1..2W-2, new pos 1 <- old pos 2W-1, pos 0 fixed
      const double2* sx = wv >= 2 ? top + (size_t)(wv - 1) * EC * 64 : (wv == 1 ? bot : nullptr);
      const double2* sy = wv <= W - 2 ? bot + (size_t)(wv + 1) * EC * 64 : top + (size_t)(W - 1) * EC * 64;
      if (sx) {
#pragma unroll
        for (int k = 0; k < EC; ++k) x.v[c * EC + k] = sx[(size_t)k * 64 + lane];
      }
#pragma unroll
      for (int k = 0; k < EC; ++k) y.v[c * EC + k] = sy[(size_t)k * 64 + lane];
      if (c == 0) {
        if (wv >= 2) nx = g_top[wv - 1];
        if (wv == 1) nx = g_bot[0];
        ny = wv <= W - 2 ? g_bot[wv + 1] : g_top[W - 1];
      }
      __syncthreads();
    }
    gx = nx;
    gy = ny;
  }
  return rot;
}

// The 28 pairs inside each block of 8 rows, one 4-wave workgroup per block
// (rows b*8 + w and b*8 + 7 - w on wave w), for every block of every item.
// Run before outer round 0 of a sweep, whose cross pairs the cross kernel
// then takes: over the sweep every pair of the matrix is visited once.  The
// rows move through LDS in two halves (32 KB at E = 8), so that LDS allows
// as many resident workgroups as the registers do.
constexpr int IW = JW / 2;
template <int E>
constexpr int intra_chunks() { return E >= 2 ? 2 : 1; }

template <int E>
__global__ __launch_bounds__(IW * 64) void jacobi_reg_intra_kernel(const JacItem* items, int max_blocks,
                                                                   int sweep, double eps_scale) {
  extern __shared__ double2 slots[];  // 2 * IW slots of 64 * E / intra_chunks<E>() elements
  __shared__ int s_rot;
  __shared__ int g_top[IW], g_bot[IW];
  const int item = blockIdx.x / max_blocks;
  const int b = blockIdx.x - item * max_blocks;
  const JacItem it = items[item];
  if (b >= it.nb) return;
  if (sweep > 0 && it.rot[(sweep - 1) * it.rot_stride] == 0) return;  // converged
  const int m = it.m, n = it.n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_rot = 0;
  const double eps = eps_scale * (double)m;
  const double floor = eps * eps * (*it.fro2);
  RegVec<E> x, y;
  int gx = b * JW + wv, gy = b * JW + (JW - 1 - wv);
  gx = gx < n ? gx : -1;
  gy = gy < n ? gy : -1;
  rv_load<E>(x, it.w + (size_t)max(gx, 0) * m, gx >= 0, m, lane);
  rv_load<E>(y, it.w + (size_t)max(gy, 0) * m, gy >= 0, m, lane);
  const int rot = circle_pairs<E, IW, intra_chunks<E>()>(x, gx, y, gy, slots, g_top, g_bot, eps, floor, lane, wv);
  if (lane == 0 && rot) atomicAdd(&s_rot, rot);
  __syncthreads();
  if (s_rot > 0) {
    if (gx >= 0) rv_store<E>(x, it.w + (size_t)gx * m, m, lane);
    if (gy >= 0) rv_store<E>(y, it.w + (size_t)gy * m, m, lane);
    if (threadIdx.x == 0) atomicAdd(&it.rot[sweep * it.rot_stride], s_rot);
  }
}

// Two disjoint pairs (x0, y0), (x1, y1) with their squared norms tracked:
// only x^+y is reduced (4 partial sums, reduce-scattered over lane bits 3
// and 2, then full sums over bits 1, 0, 4, 5), so lane l holds component
// (l >> 3) & 1 (Re, Im) of pair (l >> 2) & 1; the other component comes by a
// swizzle, the rotation is computed lane-parallel and the norms move by
// +-t |b_ij| (Algorithm 1 recomputes them; the caller does so at every
// launch, so at most a few updates accumulate).
template <int E>
__device__ __forceinline__ int rot2n(RegVec<E>& x0, RegVec<E>& y0, double& nx0, double& ny0,
                                     RegVec<E>& x1, RegVec<E>& y1, double& nx1, double& ny1,
                                     bool x_is_i, double eps, double floor, int lane) {
  double v[4];  // v[2c + i]: component c (0 Re, 1 Im) of pair i
  pair_partials_xy<E>(x0.v, y0.v, v[0], v[2]);
  pair_partials_xy<E>(x1.v, y1.v, v[1], v[3]);
  double v2[2], x;
  {
    const bool hi = (lane >> 3) & 1;
#pragma unroll
    for (int j = 0; j < 2; ++j)
      v2[j] = (hi ? v[2 + j] : v[j]) + dpp_mov<0x140>(hi ? v[j] : v[2 + j]);
  }
  {
    const bool hi = (lane >> 2) & 1;
    x = (hi ? v2[1] : v2[0]) + dpp_mov<0x141>(hi ? v2[0] : v2[1]);
  }
  x += dpp_mov<0x4E>(x);
  x += dpp_mov<0xB1>(x);
  x += swizzle<swz(16)>(x);
  x += __shfl_xor(x, 32, 64);
  const double other = swizzle<swz(8)>(x);
  const bool im_lane = (lane >> 3) & 1;
  const bool p1 = (lane >> 2) & 1;
  const double bxx = p1 ? nx1 : nx0, byy = p1 ? ny1 : ny0;
  const double br = im_lane ? other : x, bi = im_lane ? x : other;
  const uint64_t act = __ballot(pair_needs_rot(bxx, byy, br, bi, eps, floor));
  if (!(act & 17ull)) return 0;  // neither pair rotates: skip the rotation formula
  Rot mine{1.0, 0.0, 0.0, 0.0, 0.0};
  double dn = 0.0;
  pair_rot_coeffs(bxx, byy, br, bi, x_is_i, mine, &dn);
  int rot = 0;
  // pair i is held (Re component) by lane 4 i
  if (act & 1ull) {
    const Rot rt{readlane_d(mine.c, 0), readlane_d(mine.ar, 0), readlane_d(mine.ai, 0),
                 readlane_d(mine.br, 0), readlane_d(mine.bi, 0)};
    const double d = readlane_d(dn, 0);
    pair_apply<E>(x0.v, y0.v, rt);
    nx0 += x_is_i ? d : -d;
    ny0 -= x_is_i ? d : -d;
    ++rot;
  }
  if (act & 16ull) {
    const Rot rt{readlane_d(mine.c, 4), readlane_d(mine.ar, 4), readlane_d(mine.ai, 4),
                 readlane_d(mine.br, 4), readlane_d(mine.bi, 4)};
    const double d = readlane_d(dn, 4);
    pair_apply<E>(x1.v, y1.v, rt);
    nx1 += x_is_i ? d : -d;
    ny1 -= x_is_i ? d : -d;
    ++rot;
  }
  return rot;
}

template <int E>
__device__ __forceinline__ double rv_norm2(const RegVec<E>& r) {
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < E; ++k) s += r.v[k].x * r.v[k].x + r.v[k].y * r.v[k].y;
  return wave_sum(s);
}

// Every outer round: the 64 cross pairs of blocks bp and bq on CW = 4 waves.
// Wave w keeps resident rows bp*8 + 2w, 2w + 1 and holds two travellers from
// block bq, which move one wave along per step through LDS (4 steps) with
// their squared norms; each step is two sub-steps of two disjoint pairs.
constexpr int CW = 4;

template <int E>
__global__ __launch_bounds__(CW * 64, 2) void jacobi_reg_cross_kernel(const JacItem* items, int max_pairs,
                                                                      int round, int sweep,
                                                                      double eps_scale) {
  extern __shared__ double2 slots[];  // CW slots of two travellers (2 x 64 E elements)
  __shared__ double s_tn[CW][2];      // the travellers' squared norms
  __shared__ int s_rot;
  RegCtx c;
  if (!reg_prologue(items, max_pairs, round, sweep, eps_scale, c)) return;
  const int m = c.it.m, n = c.it.n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) s_rot = 0;
  RegVec<E> r0, r1, t0, t1;
  const int g0 = c.bp * JW + 2 * wv, g1 = g0 + 1;
  rv_load<E>(r0, c.it.w + (size_t)min(g0, n - 1) * m, g0 < n, m, lane);
  rv_load<E>(r1, c.it.w + (size_t)min(g1, n - 1) * m, g1 < n, m, lane);
  int src = wv;  // home wave of the travellers held
  {
    const int h0 = c.bq * JW + 2 * src, h1 = h0 + 1;
    rv_load<E>(t0, c.it.w + (size_t)min(h0, n - 1) * m, h0 < n, m, lane);
    rv_load<E>(t1, c.it.w + (size_t)min(h1, n - 1) * m, h1 < n, m, lane);
  }
  double nr0 = rv_norm2<E>(r0), nr1 = rv_norm2<E>(r1), nt0 = rv_norm2<E>(t0), nt1 = rv_norm2<E>(t1);
  const bool x_is_i = c.bp < c.bq;
  int rot = 0;
  for (int st = 0; st < CW; ++st) {
    rot += rot2n<E>(r0, t0, nr0, nt0, r1, t1, nr1, nt1, x_is_i, c.eps, c.floor, lane);
    rot += rot2n<E>(r0, t1, nr0, nt1, r1, t0, nr1, nt0, x_is_i, c.eps, c.floor, lane);
    if (st == CW - 1) break;
    double2* mine = slots + (size_t)wv * 2 * 64 * E;
    rv_to_lds<E>(t0, mine, lane);
    rv_to_lds<E>(t1, mine + 64 * E, lane);
    if (lane == 0) {
      s_tn[wv][0] = nt0;
      s_tn[wv][1] = nt1;
    }
    __syncthreads();
    const int from = (wv + CW - 1) % CW;
    const double2* prev = slots + (size_t)from * 2 * 64 * E;
    rv_from_lds<E>(t0, prev, lane);
    rv_from_lds<E>(t1, prev + 64 * E, lane);
    nt0 = s_tn[from][0];
    nt1 = s_tn[from][1];
    src = (src + CW - 1) % CW;
    __syncthreads();
  }
  if (lane == 0 && rot) atomicAdd(&s_rot, rot);
  __syncthreads();
  if (s_rot > 0) {
    const int h0 = c.bq * JW + 2 * src, h1 = h0 + 1;
    if (g0 < n) rv_store<E>(r0, c.it.w + (size_t)g0 * m, m, lane);
    if (g1 < n) rv_store<E>(r1, c.it.w + (size_t)g1 * m, m, lane);
    if (h0 < n) rv_store<E>(t0, c.it.w + (size_t)h0 * m, m, lane);
    if (h1 < n) rv_store<E>(t1, c.it.w + (size_t)h1 * m, m, lane);
    if (threadIdx.x == 0) atomicAdd(&c.it.rot[sweep * c.it.rot_stride], s_rot);
  }
}

template <int E>
hipError_t launch_reg_e(const JacItem* items_dev, int items, int max_pairs, int round, int sweep,
                        double eps_scale, hipStream_t s) {
  if (round == 0) {  // in-block pairs of every block first (nb = 2 * pairs blocks per item)
    hipLaunchKernelGGL(jacobi_reg_intra_kernel<E>, dim3(items * 2 * max_pairs), dim3(IW * 64),
                       2 * IW * 64 * (E / intra_chunks<E>()) * sizeof(double2), s, items_dev, 2 * max_pairs,
                       sweep, eps_scale);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(jacobi_reg_cross_kernel<E>, dim3(items * max_pairs), dim3(CW * 64),
                     CW * 2 * 64 * E * sizeof(double2), s, items_dev, max_pairs, round, sweep, eps_scale);
  return hipGetLastError();
}

// Rows of 513..1024 elements (E = 16, 64 registers per row and lane): a wave
// keeps one resident row of block bp in registers and takes its partners
// from LDS, where the eight rows of block bq sit (128 KB).  Cross rounds are
// eight steps; at step st wave w pairs its resident row with LDS row
// (w + st) % 8, a permutation, so no row is touched twice in a step.  Outer
// round 0 first sweeps the 28 pairs inside each block (block bp, then bq, in
// LDS, circle method, four waves with both rows in registers), then the 64
// cross pairs, so that every pair is visited once per outer sweep as with
// the shorter rows.
template <int E, int NW>
__device__ __forceinline__ int lds_intra_block(double2* lds, int b, int n, double eps, double floor, int wv,
                                               int lane) {
  int rot = 0;
  for (int t = 0; t < NW - 1; ++t) {
    if (wv < NW / 2) {
      auto pos = [&](int k) { return k == 0 ? 0 : 1 + (k - 1 + t) % (NW - 1); };
      const int a = pos(wv), bb = pos(NW - 1 - wv);
      const int ga = b * NW + a, gb = b * NW + bb;
      RegVec<E> x, y;
      rv_from_lds<E>(x, lds + (size_t)a * 64 * E, lane);
      rv_from_lds<E>(y, lds + (size_t)bb * 64 * E, lane);
      if (jacobi_pair_ordered<E>(x, ga < n ? ga : -1, y, gb < n ? gb : -1, eps, floor)) {
        rv_to_lds<E>(x, lds + (size_t)a * 64 * E, lane);
        rv_to_lds<E>(y, lds + (size_t)bb * 64 * E, lane);
        ++rot;
      }
    }
    __syncthreads();
  }
  return rot;
}

// Blocks of NW rows on NW waves: each wave keeps one resident row of block bp
// in registers and takes its partners from LDS, where the NW rows of block bq
// sit (NW * 64 E complex values).  Cross rounds are NW steps; at step st wave
// w pairs its resident row with LDS row (w + st) % NW, a permutation, so no
// row is touched twice in a step.  Outer round 0 first sweeps the pairs
// inside each block (block bp, then bq, in LDS, circle method, NW / 2 waves
// with both rows in registers), then the cross pairs, so that every pair is
// visited once per outer sweep.  Used with E = 16 (513..1024-long rows) and
// NW = 8, the block size of the other register kernels.
template <int E, int NW>
__global__ __launch_bounds__(NW * 64, 1) void jacobi_reg_lds_kernel(const JacItem* items, int max_pairs,
                                                                    int round, int sweep, double eps_scale) {
  extern __shared__ double2 lds[];  // NW rows of 64 E elements
  __shared__ int s_rot;
  RegCtx c;
  if (!reg_prologue(items, max_pairs, round, sweep, eps_scale, c)) return;
  const int m = c.it.m, n = c.it.n;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // the block pair in units of NW rows (the prologue's indices are in units of the item's blocks)
  const int bp = c.bp, bq = c.bq;
  if (threadIdx.x == 0) s_rot = 0;
  int rot = 0;
  auto block_to_lds = [&](int b) {
    const int g = b * NW + wv;
    const double2* src = c.it.w + (size_t)min(g, n - 1) * m;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int e = lane + 64 * k;
      lds[(size_t)wv * 64 * E + 64 * k + lane] = (g < n && e < m) ? src[e] : make_double2(0.0, 0.0);
    }
  };
  const int gx = bp * NW + wv;
  if (round == 0) {
    // block bp's own pairs in LDS; its rows go back to memory (each lane
    // rewrites and later rereads only its own elements) so that no resident
    // row is held while the other block's pairs take two rows per wave
    block_to_lds(bp);
    __syncthreads();
    rot += lds_intra_block<E, NW>(lds, bp, n, c.eps, c.floor, wv, lane);
    if (gx < n)
      for (int k = 0; k < E; ++k) {
        const int e = lane + 64 * k;
        if (e < m) c.it.w[(size_t)gx * m + e] = lds[(size_t)wv * 64 * E + 64 * k + lane];
      }
    __syncthreads();  // every row is read before block bq overwrites LDS
  }
  block_to_lds(bq);
  __syncthreads();
  if (round == 0) rot += lds_intra_block<E, NW>(lds, bq, n, c.eps, c.floor, wv, lane);
  RegVec<E> x;  // resident row wv of block bp
  rv_load<E>(x, c.it.w + (size_t)min(gx, n - 1) * m, gx < n, m, lane);
  for (int st = 0; st < NW; ++st) {
    const int j = (wv + st) % NW;
    const int gy = bq * NW + j;
    RegVec<E> y;
    rv_from_lds<E>(y, lds + (size_t)j * 64 * E, lane);
    if (jacobi_pair_ordered<E>(x, gx < n ? gx : -1, y, gy < n ? gy : -1, c.eps, c.floor)) {
      rv_to_lds<E>(y, lds + (size_t)j * 64 * E, lane);
      ++rot;
    }
    __syncthreads();
  }
  if (lane == 0 && rot) atomicAdd(&s_rot, rot);
  __syncthreads();
  if (s_rot > 0) {
    if (gx < n) rv_store<E>(x, c.it.w + (size_t)gx * m, m, lane);
    const int gq = bq * NW + wv;
    if (gq < n)
      for (int k = 0; k < E; ++k) {
        const int e = lane + 64 * k;
        if (e < m) c.it.w[(size_t)gq * m + e] = lds[(size_t)wv * 64 * E + 64 * k + lane];
      }
    if (threadIdx.x == 0) atomicAdd(&c.it.rot[sweep * c.it.rot_stride], s_rot);
  }
}

constexpr size_t kWideLds = (size_t)8 * 64 * 16 * sizeof(double2);  // 128 KB

// Rows of 513..1024 elements: E = 16, 8-row blocks.  (The same design with
// E = 8 and 16-row blocks, half the rounds of the 8-row register blocks, was
// slower than jacobi_reg_cross_kernel on 512-long rows: 159 against 101 ms
// per saturated 50-qubit D = 256 layer.)
hipError_t launch_jacobi_wide(const JacItem* items_dev, int items, int max_pairs, int round, int sweep,
                              double eps_scale, hipStream_t s) {
  if (items <= 0 || max_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL((jacobi_reg_lds_kernel<16, 8>), dim3(items * max_pairs), dim3(8 * 64), kWideLds, s,
                     items_dev, max_pairs, round, sweep, eps_scale);
  return hipGetLastError();
}

hipError_t launch_jacobi_reg(const JacItem* items_dev, int items, int max_pairs, int round,
                             int sweep, double eps_scale, int max_m, hipStream_t s) {
  if (items <= 0 || max_pairs <= 0) return hipSuccess;
  if (max_m <= 64) return launch_reg_e<1>(items_dev, items, max_pairs, round, sweep, eps_scale, s);
  if (max_m <= 128) return launch_reg_e<2>(items_dev, items, max_pairs, round, sweep, eps_scale, s);
  if (max_m <= 256) return launch_reg_e<4>(items_dev, items, max_pairs, round, sweep, eps_scale, s);
  if (max_m <= 512) return launch_reg_e<8>(items_dev, items, max_pairs, round, sweep, eps_scale, s);
  return hipErrorInvalidValue;
}

// Single mode: the whole matrix fits in LDS; sweep until a sweep performs no
// rotation or max_sweeps is reached.
__global__ __launch_bounds__(512) void jacobi_single_kernel(const JacItem* items, int max_sweeps,
                                                            double eps_scale) {
  extern __shared__ double2 sm[];
  __shared__ int gidx[1024];
  __shared__ int s_rot;
  const JacItem it = items[blockIdx.x];
  const int n = it.n, m = it.m;
  const int nloc = (n + 1) & ~1;
  for (int lv = threadIdx.x; lv < nloc; lv += blockDim.x) gidx[lv] = lv < n ? lv : -1;
  for (int idx = threadIdx.x; idx < n * m; idx += blockDim.x) sm[idx] = it.w[idx];
  __syncthreads();
  const double eps = eps_scale * (double)m;
  const double floor = eps * eps * (*it.fro2);
  int done = -max_sweeps;
  int any = 0;
  for (int sw = 0; sw < max_sweeps; ++sw) {
    const int rot = jacobi_local_sweep(sm, gidx, nloc, m, eps, floor, &s_rot);
    __syncthreads();
    any += rot;
    if (rot == 0) {
      done = sw + 1;
      break;
    }
  }
  if (any > 0)
    for (int idx = threadIdx.x; idx < n * m; idx += blockDim.x) it.w[idx] = sm[idx];
  if (threadIdx.x == 0) *it.sweeps_done = done;
}

hipError_t configure_jacobi_lds(size_t bytes) {
  const void* fns[] = {(const void*)jacobi_block_kernel, (const void*)jacobi_single_kernel,
                       (const void*)jacobi_reg_intra_kernel<1>, (const void*)jacobi_reg_intra_kernel<2>,
                       (const void*)jacobi_reg_intra_kernel<4>, (const void*)jacobi_reg_intra_kernel<8>,
                       (const void*)jacobi_reg_cross_kernel<1>, (const void*)jacobi_reg_cross_kernel<2>,
                       (const void*)jacobi_reg_cross_kernel<4>, (const void*)jacobi_reg_cross_kernel<8>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e != hipSuccess) return e;
  }
  if (bytes >= kWideLds) {
    const void* lf[] = {(const void*)jacobi_reg_lds_kernel<16, 8>};
    for (const void* f : lf) {
      hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kWideLds);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_jacobi_block(const JacItem* items_dev, int items, int max_pairs, int round,
                               int sweep, double eps_scale, size_t lds_bytes, hipStream_t s) {
  if (items <= 0 || max_pairs <= 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_block_kernel, dim3(items * max_pairs), dim3(512), lds_bytes, s,
                     items_dev, max_pairs, round, sweep, eps_scale);
  return hipGetLastError();
}

hipError_t launch_jacobi_single(const JacItem* items_dev, int items, int max_sweeps,
                                double eps_scale, size_t lds_bytes, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(jacobi_single_kernel, dim3(items), dim3(512), lds_bytes, s, items_dev,
                     max_sweeps, eps_scale);
  return hipGetLastError();
}

// sigma_i = ||a_i||, stable descending sort, k = min(cap, #{sigma > cutoff ||sigma||}) >= 1,
// normalised output vectors (Algorithm 1's final loop and sort; truncation of Eq. svd).
__global__ __launch_bounds__(1024) void finalize_kernel(const FinItem* items) {
  __shared__ double sig[1024];
  __shared__ int perm[1024];
  __shared__ int s_k;
  __shared__ double s_inv;
  const FinItem it = items[blockIdx.x];
  const int n = it.n, m = it.m;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int v = wave; v < n; v += 16) {
    double acc = 0.0;
    for (int e = lane; e < m; e += 64) {
      const double2 x = it.w[(size_t)v * m + e];
      acc += x.x * x.x + x.y * x.y;
    }
    acc = wave_sum(acc);
    if (lane == 0) sig[v] = sqrt(acc);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double si = sig[i];
    int r = 0;
    for (int j = 0; j < n; ++j) {
      const double sj = sig[j];
      r += (sj > si) || (sj == si && j < i);
    }
    perm[r] = i;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double tot = 0.0;
    bool bad = false;
    for (int a = 0; a < n; ++a) {
      const double sv = sig[perm[a]];
      if (!isfinite(sv)) bad = true;
      tot += sv * sv;
    }
    const double nrm = sqrt(tot);
    int k = 0;
    while (k < n && sig[perm[k]] > it.cutoff * nrm) ++k;
    if (k < 1) k = 1;
    if (k > it.cap) k = it.cap;
    double kept2 = 0.0, disc2 = 0.0;
    for (int a = 0; a < n; ++a) {
      const double sv = sig[perm[a]];
      if (a < k) kept2 += sv * sv;
      else disc2 += sv * sv;
    }
    const double kept = sqrt(kept2);
    if (bad || !(kept > 0.0) || !isfinite(kept)) {
      *it.status_out = 1;
      s_inv = 0.0;
    } else {
      *it.status_out = 0;
      s_inv = 1.0 / kept;
    }
    *it.k_out = k;
    *it.scale_out = s_inv;
    *it.disc_out = tot > 0.0 ? disc2 / tot : 0.0;
    s_k = k;
  }
  __syncthreads();
  const int k = s_k;
  const double inv = s_inv;
  if (it.mode == FIN_LEFT) {
    for (int idx = threadIdx.x; idx < m * k; idx += blockDim.x) {
      const int e = idx / k, a = idx - (idx / k) * k;
      const double sv = sig[perm[a]];
      const double2 x = it.w[(size_t)perm[a] * m + e];
      it.vec_out[idx] = sv > 0.0 ? make_double2(x.x / sv, x.y / sv) : make_double2(0.0, 0.0);
    }
  } else {
    for (int a = threadIdx.x; a < k; a += blockDim.x) it.lam_out[a] = sig[perm[a]] * inv;
    const int half = m / 2;
    for (int idx = threadIdx.x; idx < k * m; idx += blockDim.x) {
      const int a = idx / m, e = idx - (idx / m) * m;
      const int s = e / half, r = e - s * half;
      const double sv = sig[perm[a]];
      const double2 x = it.w[(size_t)perm[a] * m + e];
      it.vec_out[((size_t)s * k + a) * half + r] =
          sv > 0.0 ? make_double2(x.x / sv, x.y / sv) : make_double2(0.0, 0.0);
    }
  }
}

hipError_t launch_finalize(const FinItem* items_dev, int items, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3(items), dim3(1024), 0, s, items_dev);
  return hipGetLastError();
}

// =================================================================== Eq. (Bl)

struct TruncP {
  using T = double;
  using Ctx = TruncItem;
  static constexpr bool A_CONTIG_K = true, B_CONTIG_N = false, REAL_ONLY = false;
  const TruncItem* items;
  __device__ Ctx context(int i) const {
    TruncItem t = items[i];
    if (t.k_dev) t.k = min(t.k, *t.k_dev);
    return t;
  }
  __device__ static void dims(const Ctx& c, int& M, int& N, int& K) {
    M = c.rows;
    N = c.k;
    K = 2 * c.dr;
  }
  using RowA = const double2*;
  using ColB = const double2*;
  __device__ static RowA rowA(const Ctx& c, int i) { return c.c + (size_t)i * (2 * c.dr); }
  __device__ static ColB colB(const Ctx& c, int j) { return c.v + (size_t)j * c.dr; }
  __device__ static double2 loadA(const Ctx&, RowA r, int, int k) { return r[k]; }
  __device__ static double2 loadB(const Ctx& c, ColB b, int k, int) {
    const int s = k >= c.dr;
    const double2 v = b[(size_t)s * c.k * c.dr + (k - s * c.dr)];
    return make_double2(v.x, -v.y);
  }
  __device__ static void store(const Ctx& c, int i, int j, double re, double im) {
    const double sc = *c.scale;
    c.out[(size_t)i * c.k + j] = make_double2(re * sc, im * sc);
  }
};

hipError_t launch_trunc(const TruncItem* items_dev, int items, int max_rows, int max_k,
                        hipStream_t s) {
  TruncP p{items_dev};
  return launch_cgemm<64, 64, 16>(p, items, max_rows, max_k, s);
}

// =================================================================== canonical form

struct CanonLeftP {  // W[beta][(s,alpha)] = sum_g B[s][g][beta] T[alpha][g]
  using T = double;
  using Ctx = CanonLeftItem;
  static constexpr bool A_CONTIG_K = false, B_CONTIG_N = false, REAL_ONLY = false;
  const CanonLeftItem* items;
  __device__ Ctx context(int i) const { return items[i]; }
  __device__ static void dims(const Ctx& c, int& M, int& N, int& K) {
    M = c.db;
    N = c.r;
    K = c.dg;
  }
  using RowA = const double2*;
  using ColB = const double2*;
  __device__ static RowA rowA(const Ctx& c, int i) { return c.b + (size_t)c.s * c.dg * c.db + i; }
  __device__ static ColB colB(const Ctx& c, int j) { return c.t + (size_t)j * c.dg; }
  __device__ static double2 loadA(const Ctx& c, RowA r, int, int k) { return r[(size_t)k * c.db]; }
  __device__ static double2 loadB(const Ctx&, ColB b, int k, int) { return b[k]; }
  __device__ static void store(const Ctx& c, int i, int j, double re, double im) {
    c.w[(size_t)i * (2 * c.r) + c.s * c.r + j] = make_double2(re, im);
  }
};

struct CanonCarryLeftP {  // T'[a][beta] = sum_e conj(A[e][a]) W0[beta][e]
  using T = double;
  using Ctx = CanonCarryLeftItem;
  static constexpr bool A_CONTIG_K = false, B_CONTIG_N = false, REAL_ONLY = false;
  const CanonCarryLeftItem* items;
  __device__ Ctx context(int i) const { return items[i]; }
  __device__ static void dims(const Ctx& c, int& M, int& N, int& K) {
    M = c.k;
    N = c.db;
    K = c.m;
  }
  using RowA = const double2*;
  using ColB = const double2*;
  __device__ static RowA rowA(const Ctx& c, int i) { return c.a + i; }
  __device__ static ColB colB(const Ctx& c, int j) { return c.w0 + (size_t)j * c.m; }
  __device__ static double2 loadA(const Ctx& c, RowA r, int, int k) {
    const double2 v = r[(size_t)k * c.k];
    return make_double2(v.x, -v.y);
  }
  __device__ static double2 loadB(const Ctx&, ColB b, int k, int) { return b[k]; }
  __device__ static void store(const Ctx& c, int i, int j, double re, double im) {
    c.t[(size_t)i * c.db + j] = make_double2(re, im);
  }
};

struct CanonRightP {  // W[alpha][(s,b')] = sum_beta A[s][alpha][beta] T[beta][b']
  using T = double;
  using Ctx = CanonRightItem;
  static constexpr bool A_CONTIG_K = true, B_CONTIG_N = true, REAL_ONLY = false;
  const CanonRightItem* items;
  __device__ Ctx context(int i) const { return items[i]; }
  __device__ static void dims(const Ctx& c, int& M, int& N, int& K) {
    M = c.dl;
    N = c.r;
    K = c.dm;
  }
  using RowA = const double2*;
  using ColB = const double2*;
  __device__ static RowA rowA(const Ctx& c, int i) { return c.a + ((size_t)c.s * c.dl + i) * c.dm; }
  __device__ static ColB colB(const Ctx& c, int j) { return c.t + j; }
  __device__ static double2 loadA(const Ctx&, RowA r, int, int k) { return r[k]; }
  __device__ static double2 loadB(const Ctx& c, ColB b, int k, int) { return b[(size_t)k * c.r]; }
  __device__ static void store(const Ctx& c, int i, int j, double re, double im) {
    c.w[(size_t)i * (2 * c.r) + c.s * c.r + j] = make_double2(re, im);
  }
};

hipError_t launch_canon_left(const CanonLeftItem* items_dev, int items, int max_db, int max_r,
                             hipStream_t s) {
  CanonLeftP p{items_dev};
  return launch_cgemm<64, 64, 16>(p, items, max_db, max_r, s);
}
hipError_t launch_canon_carry_left(const CanonCarryLeftItem* items_dev, int items, int max_k,
                                   int max_db, hipStream_t s) {
  CanonCarryLeftP p{items_dev};
  return launch_cgemm<64, 64, 16>(p, items, max_k, max_db, s);
}
hipError_t launch_canon_right(const CanonRightItem* items_dev, int items, int max_dl, int max_r,
                              hipStream_t s) {
  CanonRightP p{items_dev};
  return launch_cgemm<64, 64, 16>(p, items, max_dl, max_r, s);
}

__global__ __launch_bounds__(256) void fro2_kernel(const double2* w, int count, double* out) {
  double acc = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < count; i += gridDim.x * 256) {
    const double2 x = w[i];
    acc += x.x * x.x + x.y * x.y;
  }
  acc = wave_sum(acc);
  __shared__ double part[4];
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(out, part[0] + part[1] + part[2] + part[3]);
}

hipError_t launch_fro2(const double2* w, int count, double* out, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int blocks = cdiv(count, 256);
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(fro2_kernel, dim3(blocks), dim3(256), 0, s, w, count, out);
  return hipGetLastError();
}

__global__ void copy_kernel(double2* dst, const double2* src, size_t count) {
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < count; i += (size_t)gridDim.x * 256)
    dst[i] = src[i];
}

hipError_t launch_copy(double2* dst, const double2* src, size_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  size_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dst, src, count);
  return hipGetLastError();
}

// =================================================================== fixed scratch

// Device scratch of the entry point that allocates nothing
// (mps_jacobi_svd_noalloc).  Each device holds its own copy of the array at
// its own address; host code reaches it only through the address
// hipGetSymbolAddress returns for the current device, looked up once per
// device and kept.  Every call on a device shares its copy.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kScratchDevices] = {};
}  // namespace

hipError_t scratch_address(void** out) {
  *out = nullptr;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Zero-fill of a device region (a kernel, not a memset node: callers may
// capture it in a graph).
__global__ void zero_kernel(uint64_t* dst, size_t words) {
  for (size_t i = blockIdx.x * (size_t)256 + threadIdx.x; i < words; i += (size_t)gridDim.x * 256)
    dst[i] = 0;
}

hipError_t launch_zero(void* dst, size_t bytes, hipStream_t s) {
  const size_t words = (bytes + 7) / 8;
  if (words == 0) return hipSuccess;
  size_t blocks = (words + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, (uint64_t*)dst, words);
  return hipGetLastError();
}

// One site of the statevector contraction of Eq. (mps):
//   out[(a, s)][beta] = sum_alpha in[a][alpha] B^s[alpha][beta],
// `in` holding `amps` rows of D_l amplitudes-with-open-bond, `out` 2 amps rows
// of D_r.  Row index a is the bit string of the sites already contracted,
// the earliest site most significant, so qubit 0 ends as the top bit.
__global__ void sv_site_kernel(const double2* in, const double2* b, double2* out, int64_t amps, int dl,
                               int dr) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  const int64_t total = amps * 2 * dr;
  if (i >= total) return;
  const int beta = (int)(i % dr);
  const int64_t as = i / dr;
  const int sbit = (int)(as & 1);
  const int64_t a = as >> 1;
  const double2* row = in + a * dl;
  const double2* col = b + (size_t)sbit * dl * dr + beta;
  double re = 0.0, im = 0.0;
  for (int al = 0; al < dl; ++al) {
    const double2 x = row[al], y = col[(size_t)al * dr];
    re += x.x * y.x - x.y * y.y;
    im += x.x * y.y + x.y * y.x;
  }
  out[i] = make_double2(re, im);
}

hipError_t launch_sv_site(const double2* in, const double2* b, double2* out, int64_t amps, int dl, int dr,
                          hipStream_t s) {
  const int64_t total = amps * 2 * dr;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(sv_site_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, in, b, out, amps,
                     dl, dr);
  return hipGetLastError();
}

__global__ void fill_ident_kernel(double2* dst, int d) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < d * d) dst[i] = make_double2((i / d) == (i % d) ? 1.0 : 0.0, 0.0);
}

hipError_t launch_fill_ident(double2* dst, int d, hipStream_t s) {
  if (d <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_ident_kernel, dim3(cdiv((long long)d * d, 256)), dim3(256), 0, s, dst, d);
  return hipGetLastError();
}

// =================================================================== Eq. (expec2)

// X = L [A^0 | A^1]: (Dl x Dl)(Dl x 2Dr); one item per parent, the site A and
// the dims the launch's or (items of several MPSs in one launch) the item's.
template <typename TT>
struct EnvG1P {
  using T = TT;
  using C2 = typename cplx_of<TT>::type;
  struct Ctx {
    const C2* l;
    C2* x;
    const C2* site;
    int dl, dr;
  };
  static constexpr bool A_CONTIG_K = true, B_CONTIG_N = true, REAL_ONLY = false;
  const EnvParent<C2>* items;
  const C2* site;
  int dl, dr;
  __device__ Ctx context(int i) const {
    const EnvParent<C2> e = items[i];
    if (e.site) return Ctx{e.l, e.x, e.site, e.dl, e.dr};
    return Ctx{e.l, e.x, site, dl, dr};
  }
  __device__ static void dims(const Ctx& c, int& M, int& N, int& K) {
    M = c.dl;
    N = 2 * c.dr;
    K = c.dl;
  }
  using RowA = const C2*;
  using ColB = const C2*;
  __device__ static RowA rowA(const Ctx& c, int i) { return c.l + (size_t)i * c.dl; }
  __device__ static ColB colB(const Ctx& c, int j) {
    const int s = j >= c.dr;
    return c.site + (size_t)s * c.dl * c.dr + (j - s * c.dr);
  }
  __device__ static C2 loadA(const Ctx&, RowA r, int, int k) { return r[k]; }
  __device__ static C2 loadB(const Ctx& c, ColB b, int k, int) { return b[(size_t)k * c.dr]; }
  // Eight consecutive k (k + 7 < K) for the 16-bit split GEMM; the return
  // value is the operation on the split planes that turns the loaded values
  // into the operand (SPLIT_SWAP, SPLIT_NEG_RE, SPLIT_NEG_IM bits; none here).
  __device__ __forceinline__ static int loadA8(const Ctx&, RowA r, int, int k, C2 (&o)[8]) {
#pragma unroll
    for (int t = 0; t < 8; ++t) o[t] = r[k + t];
    return 0;
  }
  __device__ __forceinline__ static int loadB8(const Ctx& c, ColB b, int k, int, C2 (&o)[8]) {
    const C2* q = b + (size_t)k * c.dr;
#pragma unroll
    for (int t = 0; t < 8; ++t) o[t] = q[(size_t)t * c.dr];
    return 0;
  }
  __device__ static void store(const Ctx& c, int i, int j, TT re, TT im) {
    C2 v;
    v.x = re;
    v.y = im;
    c.x[(size_t)i * (2 * c.dr) + j] = v;
  }
};

// L' = sum_s A^{s+} Y^s with Y^s = sum_s' sigma_{ss'} X^{s'}: a block swap
// (X, Y letters) and a phase (Y: -i, +i; Z: +1, -1) folded into the B fetch.
template <typename TT>
struct EnvG2P {
  using T = TT;
  using C2 = typename cplx_of<TT>::type;
  struct Ctx {
    const C2* x;
    C2* out;
    const C2* site;
    int dl, dr, letter;
  };
  static constexpr bool A_CONTIG_K = false, B_CONTIG_N = true, REAL_ONLY = false;
  const EnvChild<C2>* items;
  const C2* site;
  int dl, dr;
  __device__ Ctx context(int i) const {
    const EnvChild<C2> e = items[i];
    if (e.site) return Ctx{e.x, e.out, e.site, e.dl, e.dr, e.letter};
    return Ctx{e.x, e.out, site, dl, dr, e.letter};
  }
  __device__ static void dims(const Ctx& c, int& M, int& N, int& K) {
    M = c.dr;
    N = c.dr;
    K = 2 * c.dl;
  }
  using RowA = const C2*;
  using ColB = const C2*;
  __device__ static RowA rowA(const Ctx& c, int i) { return c.site + i; }
  __device__ static ColB colB(const Ctx& c, int j) { return c.x + j; }
  __device__ static C2 loadA(const Ctx& c, RowA r, int, int k) {
    // element (beta, (s, alpha)) of [A^0+ | A^1+] is conj(A[s][alpha][beta]); k = s*dl + alpha
    C2 v = r[(size_t)k * c.dr];
    v.y = -v.y;
    return v;
  }
  __device__ static C2 loadB(const Ctx& c, ColB b, int k, int) {
    const int s = k >= c.dl;
    const int a = k - s * c.dl;
    const int flip = (c.letter == 1 || c.letter == 2) ? 1 : 0;
    const C2 v = b[(size_t)a * (2 * c.dr) + (s ^ flip) * c.dr];
    C2 o = v;
    if (c.letter == 2) {  // Y: s=0 -> -i X^1, s=1 -> +i X^0
      if (s == 0) { o.x = v.y; o.y = -v.x; }
      else { o.x = -v.y; o.y = v.x; }
    } else if (c.letter == 3 && s == 1) {
      o.x = -v.x;
      o.y = -v.y;
    }
    return o;
  }
  // Eight consecutive k as in EnvG1P: the conjugation, and the letter's
  // phase when all eight share one s, become sign flips and a swap of the
  // split planes (exact: the split commutes with negation); eight k across
  // the s boundary are loaded one by one.
  __device__ __forceinline__ static int loadA8(const Ctx& c, RowA r, int, int k, C2 (&o)[8]) {
    const C2* q = r + (size_t)k * c.dr;
#pragma unroll
    for (int t = 0; t < 8; ++t) o[t] = q[(size_t)t * c.dr];
    return SPLIT_NEG_IM;
  }
  __device__ __forceinline__ static int loadB8(const Ctx& c, ColB b, int k, int j, C2 (&o)[8]) {
    const int s = k >= c.dl;
    const int a = k - s * c.dl;
    if (a + 7 >= c.dl) {
#pragma unroll
      for (int t = 0; t < 8; ++t) o[t] = loadB(c, b, k + t, j);
      return 0;
    }
    const int flip = (c.letter == 1 || c.letter == 2) ? 1 : 0;
    const C2* q = b + (size_t)a * (2 * c.dr) + (s ^ flip) * c.dr;
#pragma unroll
    for (int t = 0; t < 8; ++t) o[t] = q[(size_t)t * (2 * c.dr)];
    if (c.letter == 2) return s == 0 ? (SPLIT_SWAP | SPLIT_NEG_IM) : (SPLIT_SWAP | SPLIT_NEG_RE);
    if (c.letter == 3 && s == 1) return SPLIT_NEG_RE | SPLIT_NEG_IM;
    return 0;
  }
  __device__ static void store(const Ctx& c, int i, int j, TT re, TT im) {
    C2 v;
    v.x = re;
    v.y = im;
    c.out[(size_t)i * c.dr + j] = v;
  }
};

// One environment GEMM with tile shape kEnvTileShape[tile] (all shapes give
// bitwise-identical results: every output element accumulates its K range in
// the same order of 16x16x4 steps whatever the tile).
template <class P>
hipError_t launch_env_tile(const P& p, int tile, int count, int m, int n, hipStream_t s) {
  switch (tile) {
    case 0: return launch_cgemm<64, 64, 16>(p, count, m, n, s);
    case 1: return launch_cgemm<32, 32, 16>(p, count, m, n, s);
    case 2: return launch_cgemm<128, 64, 16>(p, count, m, n, s);
    case 3: return launch_cgemm<64, 128, 16>(p, count, m, n, s);
    case 4: return launch_cgemm<64, 64, 32>(p, count, m, n, s);
    case 5: return launch_cgemm<32, 64, 16>(p, count, m, n, s);
    case 6: return launch_cgemm<128, 128, 16>(p, count, m, n, s);
    case 7: return launch_cgemm<128, 128, 8>(p, count, m, n, s);
    default: return hipErrorInvalidValue;
  }
}
static_assert(kEnvTiles == 8, "launch_env_tile covers every tile shape");

hipError_t launch_env_gemm1_c128(const EnvParent<double2>* items, int count, const double2* site,
                                 int dl, int dr, hipStream_t s, int tile) {
  EnvG1P<double> p{items, site, dl, dr};
  return launch_env_tile(p, tile, count, dl, 2 * dr, s);
}
hipError_t launch_env_gemm2_c128(const EnvChild<double2>* items, int count, const double2* site,
                                 int dl, int dr, hipStream_t s, int tile) {
  EnvG2P<double> p{items, site, dl, dr};
  return launch_env_tile(p, tile, count, dr, dr, s);
}
hipError_t launch_env_gemm1_c64(const EnvParent<float2>* items, int count, const float2* site,
                                int dl, int dr, hipStream_t s, int tile) {
  EnvG1P<float> p{items, site, dl, dr};
  return launch_env_tile(p, tile, count, dl, 2 * dr, s);
}
hipError_t launch_env_gemm2_c64(const EnvChild<float2>* items, int count, const float2* site,
                                int dl, int dr, hipStream_t s, int tile) {
  EnvG2P<float> p{items, site, dl, dr};
  return launch_env_tile(p, tile, count, dr, dr, s);
}

// split precisions: FP32 environments, 16-bit matrix cores, FP32 accumulation
hipError_t launch_env_gemm1_split(const EnvParent<float2>* items, int count, const float2* site, int dl,
                                  int dr, int f16, hipStream_t s) {
  EnvG1P<float> p{items, site, dl, dr};
  return f16 ? launch_cgemm_split<_Float16, 64, 64>(p, count, dl, 2 * dr, s)
             : launch_cgemm_split<__bf16, 64, 64>(p, count, dl, 2 * dr, s);
}
hipError_t launch_env_gemm2_split(const EnvChild<float2>* items, int count, const float2* site, int dl,
                                  int dr, int f16, hipStream_t s) {
  EnvG2P<float> p{items, site, dl, dr};
  return f16 ? launch_cgemm_split<_Float16, 64, 64>(p, count, dr, dr, s)
             : launch_cgemm_split<__bf16, 64, 64>(p, count, dr, dr, s);
}

// Site tensor in the environment precision (fwd, may be null) and its
// per-letter transpose tr[s][beta][alpha] = B[s][alpha][beta], which turns the
// right update R' = sum sigma B^{s'} R B^{s+} into the left form on R^T.
template <typename C2>
__global__ void site_prepare_kernel(const double2* site, C2* fwd, C2* tr, int dl, int dr) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int per = dl * dr;
  if (idx >= 2 * per) return;
  const int s = idx / per;
  const int rem = idx - s * per;
  const int a = rem / dr, b = rem - (rem / dr) * dr;
  const double2 v = site[idx];
  C2 o;
  o.x = v.x;
  o.y = v.y;
  if (fwd) fwd[idx] = o;
  tr[(size_t)s * per + (size_t)b * dl + a] = o;
}

hipError_t launch_site_prepare(const double2* site, void* out_fwd, void* out_tr, int dl, int dr,
                               int elem_bytes, hipStream_t s) {
  const int blocks = cdiv(2LL * dl * dr, 256);
  if (elem_bytes == 16)
    hipLaunchKernelGGL(site_prepare_kernel<double2>, dim3(blocks), dim3(256), 0, s, site,
                       (double2*)out_fwd, (double2*)out_tr, dl, dr);
  else
    hipLaunchKernelGGL(site_prepare_kernel<float2>, dim3(blocks), dim3(256), 0, s, site,
                       (float2*)out_fwd, (float2*)out_tr, dl, dr);
  return hipGetLastError();
}

// Roots of the two tries at one bond: diag(lambda^2) (Eq. expec1/expec2) and
// the identity (right boundary in right-canonical form, Eq. rc).
template <typename C2>
__global__ void roots_kernel(const double* lam, C2* lroot, C2* rroot, int d) {
  const int idx = blockIdx.x * 256 + threadIdx.x;
  if (idx >= d * d) return;
  const int i = idx / d, j = idx - (idx / d) * d;
  C2 z;
  z.x = 0;
  z.y = 0;
  C2 lv = z, rv = z;
  if (i == j) {
    lv.x = lam[i] * lam[i];
    rv.x = 1;
  }
  if (lroot) lroot[idx] = lv;
  if (rroot) rroot[idx] = rv;
}

hipError_t launch_roots(const double* lam, void* lroot, void* rroot, int d, int elem_bytes,
                        hipStream_t s) {
  const int blocks = cdiv((long long)d * d, 256);
  if (elem_bytes == 16)
    hipLaunchKernelGGL(roots_kernel<double2>, dim3(blocks), dim3(256), 0, s, lam, (double2*)lroot,
                       (double2*)rroot, d);
  else
    hipLaunchKernelGGL(roots_kernel<float2>, dim3(blocks), dim3(256), 0, s, lam, (float2*)lroot,
                       (float2*)rroot, d);
  return hipGetLastError();
}

// FP64 environment -> a root slot in the environment precision.
template <typename C2>
__global__ void root_copy_kernel(const double2* src, C2* dst, size_t count) {
  const size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i < count) {
    C2 v;
    v.x = src[i].x;
    v.y = src[i].y;
    dst[i] = v;
  }
}

hipError_t launch_root_copy(const double2* src, void* dst, size_t count, int elem_bytes, hipStream_t s) {
  if (count == 0) return hipSuccess;
  const int blocks = cdiv((long long)count, 256);
  if (elem_bytes == 16)
    hipLaunchKernelGGL(root_copy_kernel<double2>, dim3(blocks), dim3(256), 0, s, src, (double2*)dst, count);
  else
    hipLaunchKernelGGL(root_copy_kernel<float2>, dim3(blocks), dim3(256), 0, s, src, (float2*)dst, count);
  return hipGetLastError();
}

// Lists of the two kernels above in one launch each (several states'
// set-up): block row y takes item y, 256 elements per block along x.
template <typename C2>
__global__ void site_prepare_list_kernel(const PrepItem* items) {
  const PrepItem it = items[blockIdx.y];
  const int idx = blockIdx.x * 256 + threadIdx.x;
  const int per = it.dl * it.dr;
  if (idx >= 2 * per) return;
  const int s = idx / per;
  const int rem = idx - s * per;
  const int a = rem / it.dr, b = rem - (rem / it.dr) * it.dr;
  const double2 v = it.site[idx];
  C2 o;
  o.x = v.x;
  o.y = v.y;
  if (it.fwd) ((C2*)it.fwd)[idx] = o;
  ((C2*)it.tr)[(size_t)s * per + (size_t)b * it.dl + a] = o;
}

hipError_t launch_site_prepare_list(const PrepItem* items, int count, int max_elems, int elem_bytes,
                                    hipStream_t s) {
  if (count <= 0 || max_elems <= 0) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  const dim3 grid(cdiv((long long)max_elems, 256), count);
  if (elem_bytes == 16)
    hipLaunchKernelGGL(site_prepare_list_kernel<double2>, grid, dim3(256), 0, s, items);
  else
    hipLaunchKernelGGL(site_prepare_list_kernel<float2>, grid, dim3(256), 0, s, items);
  return hipGetLastError();
}

template <typename C2>
__global__ void root_copy_list_kernel(const CopyItem* items) {
  const CopyItem it = items[blockIdx.y];
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < it.count) {
    C2 v;
    v.x = it.src[i].x;
    v.y = it.src[i].y;
    ((C2*)it.dst)[i] = v;
  }
}

hipError_t launch_root_copy_list(const CopyItem* items, int count, long long max_count, int elem_bytes,
                                 hipStream_t s) {
  if (count <= 0 || max_count <= 0) return hipSuccess;
  if (count > 65535) return hipErrorInvalidValue;
  const dim3 grid(cdiv(max_count, 256), count);
  if (elem_bytes == 16)
    hipLaunchKernelGGL(root_copy_list_kernel<double2>, grid, dim3(256), 0, s, items);
  else
    hipLaunchKernelGGL(root_copy_list_kernel<float2>, grid, dim3(256), 0, s, items);
  return hipGetLastError();
}

// Closing traces: Tr(L_a R_b) = sum_{xy} L_a[x][y] R_b[y][x] = sum_x L_a[x] R^T_b[x]
// with right environments stored transposed; computed in FP64, real part
// only, for the 64x64 tiles of (prefix, suffix) pairs that some string needs.
template <typename C2>
struct GramTileP {
  using T = double;
  struct Ctx {
    const void* const* lptr;
    const void* const* rptr;
    double* g;
    int m, n, k, ldg;
  };
  using RowA = const C2*;
  using ColB = const C2*;
  static constexpr bool A_CONTIG_K = true, B_CONTIG_N = false, REAL_ONLY = true;
  const GramItem* items;
  const GramTile* tiles;
  __device__ Ctx context(int i) const {
    const GramTile t = tiles[i];
    const GramItem b = items[t.item];
    return Ctx{b.lptr + t.r0, b.rptr + t.c0, b.g + (size_t)t.r0 * b.nr + t.c0,
               min(64, b.nl - t.r0), min(64, b.nr - t.c0), b.kdim, b.nr};
  }
  __device__ static void dims(const Ctx& c, int& M, int& N, int& K) {
    M = c.m;
    N = c.n;
    K = c.k;
  }
  __device__ static RowA rowA(const Ctx& c, int i) { return (const C2*)c.lptr[i]; }
  __device__ static ColB colB(const Ctx& c, int j) { return (const C2*)c.rptr[j]; }
  __device__ static double2 loadA(const Ctx&, RowA r, int, int k) {
    const C2 v = r[k];
    return make_double2((double)v.x, (double)v.y);
  }
  __device__ static double2 loadB(const Ctx&, ColB b, int k, int) {
    const C2 v = b[k];
    return make_double2((double)v.x, (double)v.y);
  }
  __device__ static void store(const Ctx& c, int i, int j, double re, double) {
    c.g[(size_t)i * c.ldg + j] = re;
  }
};

// Split-K form: item i = split * n_tiles + tile sums the K range of its split
// (K / splits rounded up to 16) into part[i] (64 x 64, row-major); gram_reduce
// then adds the splits in a fixed order, so the result does not depend on
// scheduling.  Long traces (K = D^2 up to 262144) are split so that a
// launch has enough workgroups to fill the chip.
template <typename C2>
struct GramSplitP {
  using T = double;
  struct Ctx {
    const void* const* lptr;
    const void* const* rptr;
    double* part;
    int m, n, k0, k;
  };
  using RowA = const C2*;
  using ColB = const C2*;
  static constexpr bool A_CONTIG_K = true, B_CONTIG_N = false, REAL_ONLY = true;
  const GramItem* items;
  const GramTile* tiles;
  double* part;
  int n_tiles, splits;
  __device__ Ctx context(int i) const {
    const int tile = i % n_tiles, sp = i / n_tiles;
    const GramTile t = tiles[tile];
    const GramItem b = items[t.item];
    const int chunk = ((b.kdim + splits - 1) / splits + 15) & ~15;
    const int k0 = min(b.kdim, sp * chunk);
    const int k1 = min(b.kdim, k0 + chunk);
    return Ctx{b.lptr + t.r0, b.rptr + t.c0, part + (size_t)i * 4096, min(64, b.nl - t.r0),
               min(64, b.nr - t.c0), k0, k1 - k0};
  }
  __device__ static void dims(const Ctx& c, int& M, int& N, int& K) {
    M = c.m;
    N = c.n;
    K = c.k;
  }
  __device__ static RowA rowA(const Ctx& c, int i) { return (const C2*)c.lptr[i] + c.k0; }
  __device__ static ColB colB(const Ctx& c, int j) { return (const C2*)c.rptr[j] + c.k0; }
  __device__ static double2 loadA(const Ctx&, RowA r, int, int k) {
    const C2 v = r[k];
    return make_double2((double)v.x, (double)v.y);
  }
  __device__ static double2 loadB(const Ctx&, ColB b, int k, int) {
    const C2 v = b[k];
    return make_double2((double)v.x, (double)v.y);
  }
  __device__ static void store(const Ctx& c, int i, int j, double re, double) { c.part[i * 64 + j] = re; }
};

__global__ void gram_reduce_kernel(const GramItem* items, const GramTile* tiles, const double* part,
                                   int n_tiles, int splits) {
  const int tile = blockIdx.x;
  const GramTile t = tiles[tile];
  const GramItem b = items[t.item];
  const int m = min(64, b.nl - t.r0), n = min(64, b.nr - t.c0);
  for (int e = threadIdx.x; e < 4096; e += blockDim.x) {
    const int i = e >> 6, j = e & 63;
    if (i >= m || j >= n) continue;
    double acc = 0.0;
    for (int sp = 0; sp < splits; ++sp) acc += part[((size_t)sp * n_tiles + tile) * 4096 + e];
    b.g[(size_t)(t.r0 + i) * b.nr + t.c0 + j] = acc;
  }
}

int gram_splits(int max_kdim) { return max_kdim >= 32768 ? 8 : (max_kdim >= 8192 ? 4 : 1); }

hipError_t launch_gram(const GramItem* items_dev, const GramTile* tiles_dev, int n_tiles, int elem_bytes,
                       double* part, int splits, hipStream_t s) {
  if (n_tiles <= 0) return hipSuccess;
  if (splits <= 1 || !part) {
    if (elem_bytes == 16) {
      GramTileP<double2> p{items_dev, tiles_dev};
      return launch_cgemm<64, 64, 16>(p, n_tiles, 64, 64, s);
    }
    GramTileP<float2> p{items_dev, tiles_dev};
    return launch_cgemm<64, 64, 16>(p, n_tiles, 64, 64, s);
  }
  hipError_t e;
  if (elem_bytes == 16) {
    GramSplitP<double2> p{items_dev, tiles_dev, part, n_tiles, splits};
    e = launch_cgemm<64, 64, 16>(p, n_tiles * splits, 64, 64, s);
  } else {
    GramSplitP<float2> p{items_dev, tiles_dev, part, n_tiles, splits};
    e = launch_cgemm<64, 64, 16>(p, n_tiles * splits, 64, 64, s);
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(n_tiles), dim3(256), 0, s, items_dev, tiles_dev, part, n_tiles,
                     splits);
  return hipGetLastError();
}

// <P_k> = closing trace / <psi|psi> (nrm null: unit norm)
__global__ void gather_kernel(const double* g, const int64_t* gidx, const double2* nrm, double* per_term,
                              int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (i < n) per_term[i] = nrm ? g[gidx[i]] / nrm->x : g[gidx[i]];
}

hipError_t launch_gather(const double* g, const int64_t* gidx, const double2* nrm, double* per_term,
                         int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(gather_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, gidx, nrm,
                     per_term, n);
  return hipGetLastError();
}

// E = sum_k c_k <P_k>: each thread a contiguous chunk with error-free
// transformations (TwoProduct by fma, TwoSum), then a fixed-shape tree of
// double-double additions -- the result depends only on the string order.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__global__ __launch_bounds__(1024) void energy_kernel(const double* per_term, const double* coeffs,
                                                      int64_t n, double* out) {
  __shared__ double hs[1024], ls[1024];
  const int64_t chunk = (n + 1023) / 1024;
  const int64_t lo = threadIdx.x * chunk;
  const int64_t hi = lo + chunk < n ? lo + chunk : n;
  double s = 0.0, c = 0.0;
  for (int64_t i = lo; i < hi; ++i) {
    const double p = coeffs[i] * per_term[i];
    const double pe = fma(coeffs[i], per_term[i], -p);
    double t, e;
    two_sum(s, p, t, e);
    s = t;
    c += e + pe;
  }
  hs[threadIdx.x] = s;
  ls[threadIdx.x] = c;
  __syncthreads();
  for (int w = 512; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      double t, e;
      two_sum(hs[threadIdx.x], hs[threadIdx.x + w], t, e);
      hs[threadIdx.x] = t;
      ls[threadIdx.x] = ls[threadIdx.x] + ls[threadIdx.x + w] + e;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {  // the compensated pair (sum, error); the value is their sum
    out[0] = hs[0];
    out[1] = ls[0];
  }
}

// Several compensated pairs (hi_i, lo_i), i < n, added in index order with the
// same error-free transformations: out[0] = sum, out[1] = error.
__global__ void pair_sum_kernel(const double* pairs, int n, double* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s = 0.0, c = 0.0;
  for (int i = 0; i < n; ++i) {
    double t, e;
    two_sum(s, pairs[2 * i], t, e);
    s = t;
    c += e + pairs[2 * i + 1];
  }
  out[0] = s;
  out[1] = c;
}

hipError_t launch_pair_sum(const double* pairs, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(pair_sum_kernel, dim3(1), dim3(64), 0, s, pairs, n, out);
  return hipGetLastError();
}

// out[r] = sum_{i in row r} vals[i] <P_{cols[i]}>, one thread per row, with
// the same error-free transformations as the energy (result depends only on
// the order of the row's entries).
__global__ void rows_kernel(const double* per_term, const int64_t* row_ptr, const int64_t* cols,
                           const double* vals, int64_t n_rows, double* out) {
  const int64_t r = blockIdx.x * (int64_t)256 + threadIdx.x;
  if (r >= n_rows) return;
  double s = 0.0, c = 0.0;
  for (int64_t i = row_ptr[r]; i < row_ptr[r + 1]; ++i) {
    const double p = vals[i] * per_term[cols[i]];
    const double pe = fma(vals[i], per_term[cols[i]], -p);
    double t, e;
    two_sum(s, p, t, e);
    s = t;
    c += e + pe;
  }
  out[r] = s + c;
}

hipError_t launch_rows(const double* per_term, const int64_t* row_ptr, const int64_t* cols, const double* vals,
                       int64_t n_rows, double* out, hipStream_t s) {
  if (n_rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(rows_kernel, dim3((unsigned)((n_rows + 255) / 256)), dim3(256), 0, s, per_term, row_ptr,
                     cols, vals, n_rows, out);
  return hipGetLastError();
}

hipError_t launch_energy(const double* per_term, const double* coeffs, int64_t n, double* out,
                         hipStream_t s) {
  hipLaunchKernelGGL(energy_kernel, dim3(1), dim3(1024), 0, s, per_term, coeffs, n, out);
  return hipGetLastError();
}

// One 16x16x4 MFMA of known operands in FP64 (out[0..255]) and FP32
// (out[256..511]), written back through the accumulator layout the GEMMs use.
__global__ void selftest_mfma_kernel(double* out) {
  const int l = threadIdx.x;
  const int r = l & 15, k = l >> 4;
  const double a = 1.0 + r + 0.5 * k;            // A[r][k]
  const double b = 1.0 + 0.25 * k - 0.125 * r;   // B[k][r]
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
  acc = mfma_16x16x4(a, b, acc);
  f4_t facc = {0.f, 0.f, 0.f, 0.f};
  facc = mfma_16x16x4((float)a, (float)b, facc);
  // 16x16x32: A[i][kk] = ((i + 2 kk) mod 7) - 3, B[kk][j] = ((3 kk + j) mod 5) - 2 (exact in 16 bits)
  bf16x8_t ab, bb;
  f16x8_t ah, bh;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int kk = frag32_k(l, j);
    const float av = (float)(((r + 2 * kk) % 7) - 3), bv = (float)(((3 * kk + r) % 5) - 2);
    ab[j] = (__bf16)av;
    bb[j] = (__bf16)bv;
    ah[j] = (_Float16)av;
    bh[j] = (_Float16)bv;
  }
  f4_t c16 = {0.f, 0.f, 0.f, 0.f}, d16 = {0.f, 0.f, 0.f, 0.f};
  c16 = split_traits<__bf16>::mfma(ab, bb, c16);
  d16 = split_traits<_Float16>::mfma(ah, bh, d16);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    out[acc_row<double>(k, v) * 16 + r] = acc[v];
    out[256 + acc_row<float>(k, v) * 16 + r] = (double)facc[v];
    out[512 + acc_row<float>(k, v) * 16 + r] = (double)c16[v];
    out[768 + acc_row<float>(k, v) * 16 + r] = (double)d16[v];
  }
}

hipError_t launch_selftest_mfma(double* out, hipStream_t s) {
  hipLaunchKernelGGL(selftest_mfma_kernel, dim3(1), dim3(64), 0, s, out);
  return hipGetLastError();
}

}  // namespace mps
