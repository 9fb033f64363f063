// Internal interface between the host orchestration (mps_api.cpp) and the
// device kernels (kernels.hip).  Descriptors are plain structs copied to
// device memory; every size in them has been checked on the host against
// the capacity of the buffers the pointers refer to.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mps {

template <typename T> struct cplx_of;
template <> struct cplx_of<double> { using type = double2; };
template <> struct cplx_of<float> { using type = float2; };

// ---------------------------------------------------------------- gates
struct ThetaItem {        // Eq. (C) product B_q (2Dl x Dm) * [B_{q+1}^0 | B_{q+1}^1] (Dm x 2Dr)
  const double2* bl;      // site q, [s][l][m]
  const double2* br;      // site q+1, [s][m][r]
  double2* theta;         // out: (2Dl x 2Dr) row-major, rows (s1,l), cols (s2,r)
  int dl, dm, dr;
};

struct MixItem {          // Q mixing (Eq. C) and lambda row scaling (Eq. C~)
  double2* c;             // in: theta, out: C (in place), (2Dl x 2Dr)
  double2* w;             // out: C~ = lambda_l C, the Jacobi work matrix
  const double* lam;      // lambda of bond q (Dl values)
  const double2* q;       // 4x4 gate, row-major
  double* fro2;           // out: ||C~||_F^2
  int dl, dr;
};

struct JacItem {          // one-sided Jacobi on the n row vectors (length m) of w
  double2* w;
  const double* fro2;     // ||w||_F^2 (invariant under the rotations)
  int* rot;               // rotation count of sweep s at rot[s * rot_stride]
  int* sweeps_done;       // single-launch mode: sweeps executed (negative: no convergence)
  int n, m, wblk, nb;     // vectors, length, vectors per block, number of blocks (even)
  int rot_stride;
};

enum FinalizeMode { FIN_GATE = 0, FIN_LEFT = 1, FIN_RIGHT = 2 };

struct FinItem {          // norms, stable descending sort, truncation, output tensors
  const double2* w;       // converged vectors (n x m)
  double2* vec_out;       // FIN_GATE/FIN_RIGHT: [s][a][r] (k x m split at m/2);
                          // FIN_LEFT: [e][a] (m x k)
  double* lam_out;        // FIN_GATE/FIN_RIGHT: normalised singular values (k)
  int* k_out;             // number kept
  double* scale_out;      // 1 / ||sigma_1..k||
  double* disc_out;       // relative discarded weight
  int* status_out;        // 0 ok, 1 non-finite or zero
  int n, m, cap;          // vectors, length, maximum k
  double cutoff;
  int mode;
};

struct TruncItem {        // Eq. (Bl): out (2Dl x k) = C (2Dl x 2Dr) * conj(V)^T * scale
  const double2* c;
  const double2* v;       // [s][a][r], k rows per s
  double2* out;
  const double* scale;
  const int* k_dev;       // if not null, k is read from here (written by finalize)
  int rows, dr, k;        // rows = 2Dl; k is the upper bound when k_dev is set
};

// ---------------------------------------------------------------- canonical form
struct CanonLeftItem {    // W[beta][(s,alpha)] = sum_g B[s][g][beta] T[alpha][g]
  const double2* b;       // site [s][g][beta], (2, Dg, Db)
  const double2* t;       // carry (r x Dg)
  double2* w;             // out (Db x 2r), row-major
  int r, dg, db, s;
};
struct CanonCarryLeftItem {  // T'[a][beta] = sum_e conj(A[e][a]) W0[beta][e]
  const double2* a;       // left-canonical tensor as (m x k), m = 2r
  const double2* w0;      // M^T (Db x m)
  double2* t;             // out (k x Db)
  int k, m, db;
};
struct CanonRightItem {   // W[alpha][(s,b')] = sum_beta A[s][alpha][beta] T[beta][b']
  const double2* a;       // site (2, Dl, Dm)
  const double2* t;       // carry (Dm x r)
  double2* w;             // out (Dl x 2r)
  int dl, dm, r, s;
};

// ---------------------------------------------------------------- environments
// `site` null: the launch's site tensor and dims (one MPS per launch); set:
// this item's own (launches shared by several MPSs).
template <typename C2>
struct EnvParent {        // X = L [A^0 | A^1]
  const C2* l;            // (Dl x Dl)
  C2* x;                  // (Dl x 2Dr)
  const C2* site;
  int dl, dr;
};
template <typename C2>
struct EnvChild {         // L' = sum_s A^{s+} (ph_s X^{s xor flip})
  const C2* x;
  C2* out;                // (Dr x Dr)
  int letter;             // 0 I, 1 X, 2 Y, 3 Z
  int dl, dr;
  const C2* site;
};

struct GramItem {         // G[a][b] = Re sum_x L_a[x] R_b[x]  (closing traces at one bond)
  const void* const* lptr;
  const void* const* rptr;
  double* g;              // (nl x nr)
  int nl, nr, kdim;
};
struct GramTile {         // one 64x64 block of some bond's G that a string needs
  int item, r0, c0;
};

// ---------------------------------------------------------------- launchers
hipError_t launch_init_product(double2* const* sites, double* const* lam0, const uint8_t* bits,
                               int n, hipStream_t s);
// One fused two-qubit gate (Eqs. C, C~, svd, Bl with Algorithm 1) on one
// workgroup; bond dimensions live in `dims` on the device.  The site and
// lambda buffers are updated in place only when the SVD converged.
struct FusedGate {
  double2* bq;          // site q:   [2][D_l][D_m] in, [2][D_l][k] out
  double2* bq1;         // site q+1: [2][D_m][D_r] in, [2][k][D_r] out
  const double* lam_l;  // lambda at bond q (D_l)
  double* lam_m;        // lambda at bond q+1 (k out)
  const double2* u;     // 4x4 gate, row-major, row index 2 i_q + i_{q+1}
  int* dims;            // bond dimensions (n + 1), dims[q+1] <- k
  double2* c;           // scratch, >= 2 D_l x 2 D_r
  int* status;          // [0]: 0 ok, 1 non-finite, 2 no convergence; [1]: failing gate
  double* disc;         // += relative discarded weight
  int* sweeps;          // += sweeps used
  int q, gate;          // bond index of D_l; gate index reported on failure
  int cap_k;            // capacity of bond q+1
  int max_sweeps;
  double cutoff, eps_scale;
};

// One MPS's gate list for fused_step_kernel (one workgroup per run).  Every
// two-qubit gate must satisfy 2 cap[q] <= 128 and 2 cap[q+2] <= 128.
struct FusedRun {
  double2* const* sites;  // current site buffers (n)
  double* const* lam;     // current lambda buffers (n + 1)
  const int* cap;         // bond capacities (n + 1)
  int* dims;
  double2* c;             // scratch, >= 2 cap x 2 cap
  int* status;
  double* disc;
  int* sweeps;
  const int32_t* q0;      // gate list on the device
  const int32_t* q1;
  const double2* u;       // 16 complex per gate
  int64_t g0, g1;         // gates applied: [g0, g1)
  int max_sweeps;
  double cutoff, eps_scale;
};

hipError_t launch_gate1q(double2* b, const double2* u, int count, hipStream_t s);
hipError_t launch_gate1q_dev(double2* b, const double2* u, const int* dims, const int* status, int q,
                             int max_count, hipStream_t s);
hipError_t launch_gate2q_fused(const FusedGate& g, int max_len, hipStream_t s);
hipError_t configure_fused_lds();
hipError_t launch_jacobi_small(const JacItem* items_dev, int items, int max_sweeps, double eps_scale,
                               hipStream_t s);
hipError_t launch_fused_step(const FusedRun* runs_dev, int n_runs, int64_t step, hipStream_t s);
hipError_t launch_theta(const ThetaItem* items_dev, int items, int max_rows, int max_cols,
                        hipStream_t s);
hipError_t launch_mix(const MixItem* items_dev, int items, int max_dldr, hipStream_t s);
hipError_t configure_jacobi_lds(size_t bytes);
hipError_t launch_jacobi_block(const JacItem* items_dev, int items, int max_pairs, int round,
                               int sweep, double eps_scale, size_t lds_bytes, hipStream_t s);
hipError_t launch_jacobi_wide(const JacItem* items_dev, int items, int max_pairs, int round, int sweep,
                              double eps_scale, hipStream_t s);
hipError_t launch_jacobi_reg(const JacItem* items_dev, int items, int max_pairs, int round,
                             int sweep, double eps_scale, int max_m, hipStream_t s);
hipError_t launch_jacobi_single(const JacItem* items_dev, int items, int max_sweeps,
                                double eps_scale, size_t lds_bytes, hipStream_t s);
hipError_t launch_finalize(const FinItem* items_dev, int items, hipStream_t s);
hipError_t launch_trunc(const TruncItem* items_dev, int items, int max_rows, int max_k,
                        hipStream_t s);
hipError_t launch_canon_left(const CanonLeftItem* items_dev, int items, int max_db, int max_r,
                             hipStream_t s);
hipError_t launch_canon_carry_left(const CanonCarryLeftItem* items_dev, int items, int max_k,
                                   int max_db, hipStream_t s);
hipError_t launch_canon_right(const CanonRightItem* items_dev, int items, int max_dl, int max_r,
                              hipStream_t s);
hipError_t launch_fro2(const double2* w, int count, double* out, hipStream_t s);
hipError_t launch_copy(double2* dst, const double2* src, size_t count, hipStream_t s);
hipError_t launch_fill_ident(double2* dst, int d, hipStream_t s);

// environment products: c128 on FP64 MFMA, c64 on FP32 MFMA, with a choice of
// workgroup tile shapes (BM, BN, BK); index 0 is the default
constexpr int kEnvTiles = 8;
constexpr int kEnvTileShape[kEnvTiles][3] = {{64, 64, 16},  {32, 32, 16},   {128, 64, 16}, {64, 128, 16},
                                             {64, 64, 32},  {32, 64, 16},   {128, 128, 16}, {128, 128, 8}};
hipError_t launch_env_gemm1_c128(const EnvParent<double2>* items, int count, const double2* site,
                                 int dl, int dr, hipStream_t s, int tile = 0);
hipError_t launch_env_gemm2_c128(const EnvChild<double2>* items, int count, const double2* site,
                                 int dl, int dr, hipStream_t s, int tile = 0);
hipError_t launch_env_gemm1_c64(const EnvParent<float2>* items, int count, const float2* site,
                                int dl, int dr, hipStream_t s, int tile = 0);
hipError_t launch_env_gemm2_c64(const EnvChild<float2>* items, int count, const float2* site,
                                int dl, int dr, hipStream_t s, int tile = 0);
hipError_t launch_env_gemm1_split(const EnvParent<float2>* items, int count, const float2* site, int dl,
                                  int dr, int f16, hipStream_t s);
hipError_t launch_env_gemm2_split(const EnvChild<float2>* items, int count, const float2* site, int dl,
                                  int dr, int f16, hipStream_t s);

hipError_t launch_site_prepare(const double2* site, void* out_fwd, void* out_tr, int dl, int dr,
                               int elem_bytes, hipStream_t s);
hipError_t launch_root_copy(const double2* src, void* dst, size_t count, int elem_bytes, hipStream_t s);
struct PrepItem {         // one site tensor to prepare (fwd may be null), as launch_site_prepare
  const double2* site;
  void* fwd;
  void* tr;
  int dl, dr;
};
struct CopyItem {         // one FP64 environment to copy into a root slot, as launch_root_copy
  const double2* src;
  void* dst;
  long long count;
};
hipError_t launch_site_prepare_list(const PrepItem* items, int count, int max_elems, int elem_bytes,
                                    hipStream_t s);
hipError_t launch_root_copy_list(const CopyItem* items, int count, long long max_count, int elem_bytes,
                                 hipStream_t s);
hipError_t launch_roots(const double* lam, void* lroot, void* rroot, int d, int elem_bytes,
                        hipStream_t s);
int gram_splits(int max_kdim);  // K splits of the closing-trace tiles
hipError_t launch_gram(const GramItem* items_dev, const GramTile* tiles_dev, int n_tiles, int elem_bytes,
                       double* part, int splits, hipStream_t s);
hipError_t launch_rows(const double* per_term, const int64_t* row_ptr, const int64_t* cols, const double* vals,
                       int64_t n_rows, double* out, hipStream_t s);
hipError_t launch_gather(const double* g, const int64_t* gidx, const double2* nrm, double* per_term,
                         int64_t n, hipStream_t s);
// out[0], out[1]: compensated (sum, error) pair of sum_k coeffs[k] per_term[k]
hipError_t launch_energy(const double* per_term, const double* coeffs, int64_t n, double* out,
                         hipStream_t s);
hipError_t launch_pair_sum(const double* pairs, int n, double* out, hipStream_t s);

// Fixed device scratch (a static device array, one per device) for the entry
// point that allocates nothing: *out receives the current device's address
// of it (looked up once per device).  Sized for one Jacobi SVD of up to
// kScratchMaxVec vectors of up to kScratchMaxVec elements.
constexpr int kScratchMaxVec = 512;
constexpr size_t kScratchMatBytes = (size_t)kScratchMaxVec * kScratchMaxVec * 16;  // one complex matrix
constexpr size_t kScratchDescBytes = (size_t)64 << 10;                             // launch descriptors
constexpr size_t kScratchMiscBytes = (size_t)64 << 10;                             // norms, counters, sigma
constexpr size_t kScratchBytes = 2 * kScratchMatBytes + kScratchDescBytes + kScratchMiscBytes;
hipError_t scratch_address(void** out);
hipError_t launch_zero(void* dst, size_t bytes, hipStream_t s);
hipError_t launch_sv_site(const double2* in, const double2* b, double2* out, int64_t amps, int dl, int dr,
                          hipStream_t s);
hipError_t launch_selftest_mfma(double* out, hipStream_t s);

}  // namespace mps
