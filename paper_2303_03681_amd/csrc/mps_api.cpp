// Host orchestration and the C ABI of the MPS energy evaluator.
//
// Every numerical step runs in the kernels of kernels.hip; this file owns the
// device memory, builds the per-launch descriptors (checking every size
// against the capacity of the buffer it addresses), sequences the launches on
// the handle's stream and implements the error contract of include/mps.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <utility>
#include <vector>

#include "internal.h"
#include "mps.h"
#include "planner.h"

using namespace mps;

namespace {

thread_local std::string g_err;

mps_status fail(mps_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

constexpr int kMaxStatevectorQubits = 26;
constexpr double kEpsScale = 1.1102230246251565e-16;  // 2^-53: eps = m * 2^-53 (Algorithm 1)
constexpr double kCanonCutoff = 1e-14;                  // round-off singular values only
constexpr int kDefaultSweeps = 60;
constexpr int kMaxBond = 512;                           // finalize handles 2D <= 1024 vectors
constexpr int kMaxJacobiGroups = 3;      // streams of the batched register Jacobi rounds
constexpr int kDefaultJacobiGroups = 2;

int cap_dim(int b, int n, int D) {
  const int e = std::min(b, n - b);
  if (e >= 30) return D;
  return std::min(D, 1 << e);
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

size_t g_lds_budget = 0;  // dynamic LDS the Jacobi kernels may use (set once per process)
std::mutex g_lds_mutex;

}  // namespace

// ----------------------------------------------------------------------------
// plan object

struct mps_psum {
  PauliPlan plan;
  uint64_t serial;
};

static std::atomic<uint64_t> g_plan_serial{1};

// ----------------------------------------------------------------------------
// handle

struct ExpectSetup {
  uint64_t plan_serial = 0;
  int prec = -1;
  std::vector<int> dims;
  // device storage
  void* pool = nullptr;        // environments (left nodes, right nodes, roots)
  size_t pool_bytes = 0;
  void* sites = nullptr;       // prepared site tensors (fwd in env precision, transposed)
  size_t sites_bytes = 0;
  void* xbuf = nullptr;        // GEMM1 outputs for one chunk of parents
  size_t xbuf_bytes = 0;
  void* desc = nullptr;        // all descriptors
  size_t desc_bytes = 0;
  std::vector<char> host_desc; // host copy of the descriptors (environment launches of several MPSs)
  int64_t plan_terms = 0;
  double* gbuf = nullptr;      // closing traces
  size_t gbuf_count = 0;
  double* gpart = nullptr;     // split-K partial tiles of the closing traces
  size_t gpart_count = 0;
  int gram_split = 1;
  double* per_term = nullptr;
  double* coeffs = nullptr;
  int64_t* gidx = nullptr;
  double* energy = nullptr;
  size_t terms_cap = 0;
  // launch lists (host)
  struct EnvLaunch {
    int site, dl, dr;
    size_t parents_off, children_off;  // byte offsets into desc
    int n_parents, n_children;
    bool left;                         // left pass (forward tensor) or right pass (transposed)
    double flops;
  };
  std::vector<EnvLaunch> left_launches, right_launches;
  struct PrepSite {
    int dl, dr;
    void* fwd;
    void* tr;
  };
  std::vector<PrepSite> prep;
  struct RootFill {
    int bond, d;
    void* lroot;
    void* rroot;
  };
  std::vector<RootFill> roots;
  bool fwd128 = false;             // c128 sites copied to fixed buffers (graph replay)
  // captured device sequence (environment launches, closes, gather, energy)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  bool graph_chains = false;       // captured with the boundary-environment norm
  void* rows_buf = nullptr;        // CSR of mps_expect_pauli_rows and its output
  size_t rows_bytes = 0;
  size_t gram_off = 0, tiles_off = 0;
  int gram_items = 0, gram_tiles = 0;
  double gram_flops = 0.0;  // dense tile work of the closing traces
  double pair_flops = 0.0;  // 4 D^2 per distinct (prefix, suffix) pair
  int64_t n_updates = 0;
};

struct mps_state {
  int n = 0, D = 0, max_sweeps = kDefaultSweeps;
  double cutoff = 0.0;
  int device = 0;  // current device at create
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t budget = 0, held = 0;
  bool poisoned = false;
  std::vector<int> dims, cap;
  std::vector<double2*> site[2];
  std::vector<int> site_cur;
  std::vector<size_t> site_cap;  // complex elements
  std::vector<double*> lam[2];
  std::vector<int> lam_cur;
  bool canonical = true;  // exact canonical form: right-orthonormal sites, Schmidt lambdas
  uint64_t version = 0;    // bumped by every change of the state (gates, canonical form, reset, import, copy)
  // identity environments from both boundaries (FP64), the trie roots when the
  // sites are not in exact canonical form: left L_b (slot b), right R_b^T
  double2* d_lchain = nullptr;
  double2* d_rchain = nullptr;
  double2* d_chainx = nullptr;  // GEMM1 output of one chain step
  double2* d_chainxr = nullptr; // ... of the right chain
  double2* d_chaintr = nullptr; // one site tensor, transposed, for the right chain
  void* d_chaindesc = nullptr;
  std::vector<size_t> chain_off;
  uint64_t chain_version = ~0ull;  // state version the boundary environments were computed for
  int chain_rmin = 1 << 30;        // ... and the lowest bond of the right chain
  double norm = 1.0;
  double discarded = 0.0;
  // device helpers
  double2** d_site_ptrs = nullptr;
  double** d_lam_ptrs = nullptr;
  uint8_t* d_bits = nullptr;
  double* d_one = nullptr;
  // gate workspaces
  int ws_items = 0;
  int ctr_items = 0;  // per-item SVD counters allocated (fro2, rot, sweeps, k, scale, disc, status)
  size_t ws_stride = 0;  // complex elements per item
  double2* ws_c = nullptr;
  double2* ws_w = nullptr;
  double* d_fro2 = nullptr;
  int* d_rot = nullptr;
  int* d_sweeps = nullptr;
  int* d_k = nullptr;
  double* d_scale = nullptr;
  double* d_disc = nullptr;
  int* d_status = nullptr;
  // fused single-gate path: bond dimensions on the device while a run of
  // fused gates is queued (host dims are stale until fused_flush)
  bool fused_enabled = true;
  bool fused_active = false;
  int* d_dims = nullptr;
  int* d_fstat = nullptr;   // [0] status, [1] failing gate (chunk-relative)
  double* d_fdisc = nullptr;
  int* d_fsweeps = nullptr;
  int* d_cap = nullptr;       // bond capacities on the device (n + 1)
  int32_t* d_gq = nullptr;    // gate qubits for the multi-MPS path: q0 then q1
  size_t gq_cap = 0;
  double2* d_carry[2] = {nullptr, nullptr};
  void* d_desc = nullptr;
  size_t desc_bytes = 0;
  double2* d_gates = nullptr;
  size_t gates_cap = 0;
  double* d_pairs = nullptr;  // compensated energy pairs of mps_expect_pauli_sums
  size_t pairs_cap = 0;
  std::vector<std::pair<void*, size_t>> allocs;
  ExpectSetup ex;
  // timing
  bool timing = false;
  bool autotune = false;               // choose environment GEMM tiles by measurement
  int forced_tile = -1;                // >= 0: this tile for every environment GEMM
  bool graphs = false;                 // replay the expectation's device work as a HIP graph
  std::vector<hipEvent_t> ev_tune;     // tuning pass events
  size_t ev_tune_used = 0;
  std::vector<hipEvent_t> ev_env, ev_close;
  size_t ev_env_used = 0, ev_close_used = 0;
  hipEvent_t ev_jac[2] = {nullptr, nullptr};
  // second stream (default priority): one-workgroup SVDs of small gates run
  // beside the multi-launch rounds of the large gates of the same batch
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  // streams of the register Jacobi item groups after the first (see run_jacobi)
  hipStream_t jside[kMaxJacobiGroups - 1] = {};
  hipEvent_t ev_jfork = nullptr, ev_jjoin[kMaxJacobiGroups - 1] = {};
  int jacobi_groups = kDefaultJacobiGroups;
  mps_timing tm{};

  double2* cur(int q) { return site[site_cur[q]][q]; }
  double2* spare(int q) { return site[1 - site_cur[q]][q]; }
  double* lcur(int b) { return lam[lam_cur[b]][b]; }
  double* lspare(int b) { return lam[1 - lam_cur[b]][b]; }
};

namespace {

mps_status dev_fail(mps_state* h, const char* what, hipError_t e) {
  if (h) h->poisoned = true;
  return fail(MPS_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(h, expr)                                   \
  do {                                                     \
    hipError_t e_ = (expr);                                \
    if (e_ != hipSuccess) return dev_fail((h), #expr, e_); \
  } while (0)

mps_status dalloc(mps_state* h, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 256;
  if (h->budget && h->held + bytes > h->budget)
    return fail(MPS_ERR_BUDGET, "HBM budget exceeded: need " + std::to_string(h->held + bytes) +
                                    " bytes, budget " + std::to_string(h->budget));
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(MPS_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  h->held += bytes;
  h->allocs.emplace_back(*p, bytes);
  return MPS_OK;
}

void dfree(mps_state* h, void* p) {
  if (!p) return;
  for (size_t i = 0; i < h->allocs.size(); ++i)
    if (h->allocs[i].first == p) {
      h->held -= h->allocs[i].second;
      h->allocs.erase(h->allocs.begin() + i);
      (void)hipFree(p);
      return;
    }
}

template <typename T>
mps_status dalloc_t(mps_state* h, T** p, size_t count) {
  void* v = nullptr;
  mps_status st = dalloc(h, &v, count * sizeof(T));
  *p = (T*)v;
  return st;
}

mps_status check_handle(mps_state* h) {
  if (!h) return fail(MPS_ERR_ARG, "NULL handle");
  if (h->poisoned) return fail(MPS_ERR_DEVICE, "handle poisoned by an earlier device error");
  return MPS_OK;
}

mps_status ensure_lds(mps_state* h) {
  std::lock_guard<std::mutex> lock(g_lds_mutex);
  if (g_lds_budget) return MPS_OK;
  int dev = 0, v = 0;
  HIP_TRY(h, hipGetDevice(&dev));
  HIP_TRY(h, hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  size_t b = (size_t)v;
  if (b > 160 * 1024) b = 160 * 1024;
  b = b > 8 * 1024 ? b - 8 * 1024 : b;  // room for the kernels' static shared arrays
  if (b > 152 * 1024) b = 152 * 1024;
  HIP_TRY(h, configure_jacobi_lds(b));
  HIP_TRY(h, configure_fused_lds());
  g_lds_budget = b;
  return MPS_OK;
}

// Descriptor upload: ordered after the stream's earlier work (which may still
// read the region) and complete before returning, so the host source may be
// a temporary.
mps_status upload(mps_state* h, void* dst, const void* src, size_t bytes) {
  if (bytes == 0) return MPS_OK;
  HIP_TRY(h, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return MPS_OK;
}

mps_status sync(mps_state* h) {
  HIP_TRY(h, hipStreamSynchronize(h->stream));
  return MPS_OK;
}

mps_status ensure_side(mps_state* h) {
  if (h->side) return MPS_OK;
  HIP_TRY(h, hipEventCreateWithFlags(&h->ev_fork, hipEventDisableTiming));
  HIP_TRY(h, hipEventCreateWithFlags(&h->ev_join, hipEventDisableTiming));
  HIP_TRY(h, hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking));
  return MPS_OK;
}

mps_status ensure_jside(mps_state* h, int groups) {
  if (!h->ev_jfork) HIP_TRY(h, hipEventCreateWithFlags(&h->ev_jfork, hipEventDisableTiming));
  for (int g = 0; g + 1 < groups; ++g) {
    if (h->jside[g]) continue;
    HIP_TRY(h, hipEventCreateWithFlags(&h->ev_jjoin[g], hipEventDisableTiming));
    HIP_TRY(h, hipStreamCreateWithFlags(&h->jside[g], hipStreamNonBlocking));
  }
  return MPS_OK;
}

mps_status ensure_desc(mps_state* h, size_t bytes) {
  if (bytes <= h->desc_bytes) return MPS_OK;
  if (h->d_desc) {
    mps_status st = sync(h);
    if (st != MPS_OK) return st;
    dfree(h, h->d_desc);
    h->d_desc = nullptr;
    h->desc_bytes = 0;
  }
  size_t want = std::max(bytes, (size_t)1 << 16);
  mps_status st = dalloc(h, &h->d_desc, want);
  if (st != MPS_OK) return st;
  h->desc_bytes = want;
  return MPS_OK;
}

// Gate workspaces for up to `items` two-qubit gates at the handle's largest size.
// Per-item counters of a batched SVD (the rotation counters laid out
// [sweep][item]) for up to `items` gates.
mps_status ensure_counters(mps_state* h, int items) {
  if (items <= h->ctr_items) return MPS_OK;
  mps_status st = sync(h);
  if (st != MPS_OK) return st;
  for (void* p : {(void*)h->d_fro2, (void*)h->d_rot, (void*)h->d_sweeps, (void*)h->d_k, (void*)h->d_scale,
                  (void*)h->d_disc, (void*)h->d_status})
    dfree(h, p);
  h->d_fro2 = h->d_scale = h->d_disc = nullptr;
  h->d_rot = h->d_sweeps = h->d_k = h->d_status = nullptr;
  h->ctr_items = 0;
  if ((st = dalloc_t(h, &h->d_fro2, items)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &h->d_rot, (size_t)items * h->max_sweeps)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &h->d_sweeps, items)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &h->d_k, items)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &h->d_scale, items)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &h->d_disc, items)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &h->d_status, items)) != MPS_OK) return st;
  h->ctr_items = items;
  return MPS_OK;
}

// Gate workspaces (C and the Jacobi matrix) for up to `items` two-qubit gates
// at the handle's largest size, and their counters.
mps_status ensure_ws(mps_state* h, int items) {
  mps_status st = ensure_counters(h, items);
  if (st != MPS_OK || items <= h->ws_items) return st;
  if ((st = sync(h)) != MPS_OK) return st;
  dfree(h, h->ws_c);
  dfree(h, h->ws_w);
  h->ws_c = h->ws_w = nullptr;
  int dmax = 1;
  for (int b = 0; b <= h->n; ++b) dmax = std::max(dmax, h->cap[b]);
  h->ws_stride = (size_t)(2 * dmax) * (2 * dmax);
  h->ws_items = 0;
  if ((st = dalloc_t(h, &h->ws_c, h->ws_stride * items)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &h->ws_w, h->ws_stride * items)) != MPS_OK) return st;
  if (!h->d_carry[0]) {
    for (int i = 0; i < 2; ++i)
      if ((st = dalloc_t(h, &h->d_carry[i], (size_t)dmax * dmax)) != MPS_OK) return st;
  }
  h->ws_items = items;
  return MPS_OK;
}

// ----------------------------------------------------------------------------
// batched one-sided Jacobi over items already described in host vectors

struct JacobiPlanHost {
  std::vector<JacItem> small;               // register single-launch (n, m <= 128)
  std::vector<JacItem> single, reg, block;  // LDS single-launch, register blocks, LDS blocks
  std::vector<JacItem> wide;                // 513..1024-long rows: partner block in LDS
  size_t single_lds = 0, block_lds = 0;
  int reg_pairs = 0, reg_rounds = 0, reg_max_m = 0;
  int block_pairs = 0, block_rounds = 0;
  int wide_pairs = 0, wide_rounds = 0;
};

constexpr int kRegBlock = 8;     // vectors per block of the register kernels (one per wave)
constexpr int kRegMaxLen = 512;  // longest vector the register kernels hold
constexpr int kSmallMax = 128;   // rows and row length of the one-workgroup register kernel
constexpr size_t kWideLdsBytes = (size_t)kRegBlock * 2 * kRegMaxLen * sizeof(double2);  // one block in LDS
constexpr int64_t kSplitWorkgroups = 256;  // multi-launch rounds split over streams above this size

void plan_jacobi(const std::vector<JacItem>& all, JacobiPlanHost& jp) {
  const size_t budget = g_lds_budget;
  // One workgroup per matrix: for batches of small matrices only, and for
  // tiny ones in any batch (a 128 x 128 item on one CU would otherwise hold
  // up the multi-workgroup rounds of the large items queued after it).
  bool all_small = true;
  for (const JacItem& it : all) all_small = all_small && it.n <= kSmallMax && it.m <= kSmallMax;
  for (JacItem it : all) {
    if (it.n <= kSmallMax && it.m <= kSmallMax && (all_small || it.n * it.m <= 64 * 64)) {
      jp.small.push_back(it);
      continue;
    }
    const size_t per_vec = (size_t)it.m * sizeof(double2);
    const int nloc = (it.n + 1) & ~1;
    if (nloc <= 1024 && (size_t)it.n * per_vec <= budget &&
        (nloc <= 2 * kRegBlock || it.m > kRegMaxLen || (size_t)it.n * it.m <= 64 * 64)) {
      it.wblk = nloc;
      it.nb = 1;
      jp.single.push_back(it);
      jp.single_lds = std::max(jp.single_lds, (size_t)it.n * per_vec);
    } else if (it.m > kRegMaxLen && it.m <= 2 * kRegMaxLen && budget >= kWideLdsBytes) {
      int nb = (it.n + kRegBlock - 1) / kRegBlock;
      if (nb & 1) ++nb;
      it.wblk = kRegBlock;
      it.nb = nb;
      jp.wide.push_back(it);
      jp.wide_pairs = std::max(jp.wide_pairs, nb / 2);
      jp.wide_rounds = std::max(jp.wide_rounds, nb - 1);
    } else if (it.m <= kRegMaxLen) {
      int nb = (it.n + kRegBlock - 1) / kRegBlock;
      if (nb & 1) ++nb;
      it.wblk = kRegBlock;
      it.nb = nb;
      jp.reg.push_back(it);
      jp.reg_pairs = std::max(jp.reg_pairs, nb / 2);
      jp.reg_rounds = std::max(jp.reg_rounds, nb - 1);
      jp.reg_max_m = std::max(jp.reg_max_m, it.m);
    } else {
      const int max_vec = (int)std::max<size_t>(2, budget / per_vec);
      int w = std::min(128, max_vec / 2);
      if (w < 1) w = 1;
      int nb = (it.n + w - 1) / w;
      if (nb & 1) ++nb;
      it.wblk = w;
      it.nb = nb;
      jp.block.push_back(it);
      jp.block_lds = std::max(jp.block_lds, (size_t)(2 * w) * per_vec);
      jp.block_pairs = std::max(jp.block_pairs, nb / 2);
      jp.block_rounds = std::max(jp.block_rounds, nb - 1);
    }
  }
}

// Runs Algorithm 1 on every item (vectors in it.w, ||w||_F^2 in it.fro2 already
// on device).  Item i must use rot = all[0].rot + i with rot_stride =
// all.size(), zeroed for max_sweeps sweeps.  On return (after a stream sync)
// `sweeps_out[i]` holds the sweeps used, or -1 if the sweep limit was hit.
// Items of one multi-launch kind in groups whose rounds are queued on
// separate streams.  One round of a large batch launches more waves than the
// chip holds at once (two per SIMD at the register kernels' register use),
// so a launch runs as a full generation of waves plus a sparse second one;
// with the items dealt (largest first, to the group with the least work so
// far) into groups on separate streams, the waves of one group's round fill
// the slots the others leave idle.  Every item still sees the same rounds in
// the same order as on one stream.  `items` is reordered group by group.
struct ItemGroup {
  int off = 0, count = 0, pairs = 0, rounds = 0, max_m = 0;
  int64_t work = 0;
};

std::vector<ItemGroup> deal_groups(std::vector<JacItem>& items, int want, int pairs, int rounds,
                                   int max_m) {
  std::vector<ItemGroup> groups(1);
  groups[0].count = (int)items.size();
  groups[0].pairs = pairs;
  groups[0].rounds = rounds;
  groups[0].max_m = max_m;
  int64_t wgs = 0;
  for (const JacItem& it : items) wgs += it.nb / 2;
  const int ng = std::min<int>(want, (int)items.size() / 2);
  if (ng < 2 || wgs <= kSplitWorkgroups) return groups;
  std::vector<JacItem> srt = items;
  std::stable_sort(srt.begin(), srt.end(), [](const JacItem& a, const JacItem& b) {
    return (int64_t)a.n * a.m > (int64_t)b.n * b.m;
  });
  groups.assign(ng, ItemGroup{});
  std::vector<std::vector<JacItem>> members(ng);
  for (const JacItem& it : srt) {
    int g = 0;
    for (int k = 1; k < ng; ++k)
      if (groups[k].work < groups[g].work) g = k;
    ItemGroup& G = groups[g];
    G.work += (int64_t)it.n * it.n * it.m;
    G.pairs = std::max(G.pairs, it.nb / 2);
    G.rounds = std::max(G.rounds, it.nb - 1);
    G.max_m = std::max(G.max_m, it.m);
    members[g].push_back(it);
  }
  items.clear();
  for (int g = 0; g < ng; ++g) {
    groups[g].off = (int)items.size();
    groups[g].count = (int)members[g].size();
    items.insert(items.end(), members[g].begin(), members[g].end());
  }
  return groups;
}

mps_status run_jacobi(mps_state* h, const std::vector<JacItem>& all, size_t desc_off,
                      std::vector<int>& sweeps_out) {
  const int count = (int)all.size();
  for (int i = 0; i < count; ++i)
    if (all[i].rot != all[0].rot + i || all[i].rot_stride != count)
      return fail(MPS_ERR_STATE, "internal: Jacobi rotation counters not laid out [sweep][item]");
  JacobiPlanHost jp;
  plan_jacobi(all, jp);
  // Multi-launch items in groups on their own streams (register and wide
  // rounds alike; group g of either kind runs on stream g).
  std::vector<ItemGroup> groups = deal_groups(jp.reg, h->jacobi_groups, jp.reg_pairs, jp.reg_rounds,
                                              jp.reg_max_m);
  std::vector<ItemGroup> wgroups = deal_groups(jp.wide, h->jacobi_groups, jp.wide_pairs,
                                               jp.wide_rounds, 0);
  const int n_groups = (int)std::max(groups.size(), wgroups.size());
  const size_t bytes =
      (jp.small.size() + jp.single.size() + jp.reg.size() + jp.block.size() + jp.wide.size()) *
      sizeof(JacItem);
  mps_status st = ensure_desc(h, desc_off + bytes);
  if (st != MPS_OK) return st;
  char* base = (char*)h->d_desc + desc_off;
  JacItem* d_small = (JacItem*)base;
  JacItem* d_single = d_small + jp.small.size();
  JacItem* d_reg = d_single + jp.single.size();
  JacItem* d_block = d_reg + jp.reg.size();
  JacItem* d_wide = d_block + jp.block.size();
  std::vector<JacItem> packed(jp.small);
  packed.insert(packed.end(), jp.single.begin(), jp.single.end());
  packed.insert(packed.end(), jp.reg.begin(), jp.reg.end());
  packed.insert(packed.end(), jp.block.begin(), jp.block.end());
  packed.insert(packed.end(), jp.wide.begin(), jp.wide.end());
  if ((st = upload(h, base, packed.data(), bytes)) != MPS_OK) return st;
  const int nmulti_items = (int)(jp.reg.size() + jp.block.size() + jp.wide.size());
  const bool overlap = nmulti_items > 0 && (!jp.small.empty() || !jp.single.empty());
  hipStream_t one_stream = h->stream;
  if (overlap) {
    if ((st = ensure_side(h)) != MPS_OK) return st;
    HIP_TRY(h, hipEventRecord(h->ev_fork, h->stream));
    HIP_TRY(h, hipStreamWaitEvent(h->side, h->ev_fork, 0));
    one_stream = h->side;
  }
  if (!jp.small.empty())
    HIP_TRY(h, launch_jacobi_small(d_small, (int)jp.small.size(), h->max_sweeps, kEpsScale, one_stream));
  if (!jp.single.empty())
    HIP_TRY(h, launch_jacobi_single(d_single, (int)jp.single.size(), h->max_sweeps, kEpsScale,
                                    jp.single_lds, one_stream));
  // every later use of the handle's stream (also on an early return) waits for them
  struct Join {
    mps_state* h;
    bool on;
    ~Join() {
      if (on) (void)hipStreamWaitEvent(h->stream, h->ev_join, 0);
    }
  } join{h, false};
  if (overlap) {
    HIP_TRY(h, hipEventRecord(h->ev_join, h->side));
    join.on = true;
  }
  // per item (caller order): first rotation-free sweep, from the counters
  std::vector<int> first_zero(count, -1);
  std::vector<char> is_multi(count, 0);
  for (const JacItem& b : jp.reg) is_multi[b.rot - all[0].rot] = 1;
  for (const JacItem& b : jp.block) is_multi[b.rot - all[0].rot] = 1;
  for (const JacItem& b : jp.wide) is_multi[b.rot - all[0].rot] = 1;
  const int nmulti = nmulti_items;
  const bool timed = h->timing && nmulti > 0;
  h->tm.jacobi_multi_items += nmulti;
  h->tm.jacobi_wide_items += (int64_t)jp.wide.size();
  if (n_groups > 1) h->tm.jacobi_split_batches += 1;
  if (n_groups > 1) {
    if ((st = ensure_jside(h, n_groups)) != MPS_OK) return st;
    HIP_TRY(h, hipEventRecord(h->ev_jfork, h->stream));
    for (int g = 1; g < n_groups; ++g) HIP_TRY(h, hipStreamWaitEvent(h->jside[g - 1], h->ev_jfork, 0));
  }
  // the handle's stream waits for the other groups after every sweep (also
  // on an early return)
  struct JoinGroups {
    mps_state* h;
    int n;
    bool on;
    ~JoinGroups() {
      if (!on) return;
      for (int g = 1; g < n; ++g)
        if (hipEventRecord(h->ev_jjoin[g - 1], h->jside[g - 1]) == hipSuccess)
          (void)hipStreamWaitEvent(h->stream, h->ev_jjoin[g - 1], 0);
    }
  } join_groups{h, n_groups, false};
  if (timed) {
    for (hipEvent_t& ev : h->ev_jac)
      if (!ev) HIP_TRY(h, hipEventCreate(&ev));
    HIP_TRY(h, hipEventRecord(h->ev_jac[0], h->stream));  // after the one-launch items
  }
  if (nmulti > 0) {
    std::vector<int> rot(count);
    int done = 0;
    const int rounds = std::max(std::max(jp.reg_rounds, jp.block_rounds), jp.wide_rounds);
    for (int sw = 0; sw < h->max_sweeps && done < nmulti; ++sw) {
      h->tm.jacobi_batch_sweeps += 1;
      for (int r = 0; r < rounds; ++r) {
        for (int g = 0; g < (int)groups.size(); ++g) {
          const ItemGroup& G = groups[g];
          if (G.count == 0 || r >= G.rounds) continue;
          join_groups.on = join_groups.on || g > 0;
          HIP_TRY(h, launch_jacobi_reg(d_reg + G.off, G.count, G.pairs, r, sw, kEpsScale, G.max_m,
                                       g == 0 ? h->stream : h->jside[g - 1]));
        }
        if (!jp.block.empty() && r < jp.block_rounds)
          HIP_TRY(h, launch_jacobi_block(d_block, (int)jp.block.size(), jp.block_pairs, r, sw,
                                         kEpsScale, jp.block_lds, h->stream));
        for (int g = 0; g < (int)wgroups.size(); ++g) {
          const ItemGroup& G = wgroups[g];
          if (G.count == 0 || r >= G.rounds) continue;
          join_groups.on = join_groups.on || g > 0;
          HIP_TRY(h, launch_jacobi_wide(d_wide + G.off, G.count, G.pairs, r, sw, kEpsScale,
                                        g == 0 ? h->stream : h->jside[g - 1]));
        }
      }
      for (int g = 1; g < n_groups; ++g) {
        HIP_TRY(h, hipEventRecord(h->ev_jjoin[g - 1], h->jside[g - 1]));
        HIP_TRY(h, hipStreamWaitEvent(h->stream, h->ev_jjoin[g - 1], 0));
      }
      join_groups.on = false;
      if (sw >= 3 || sw == h->max_sweeps - 1) {
        HIP_TRY(h, hipMemcpyAsync(rot.data(), all[0].rot + (size_t)sw * count, sizeof(int) * count,
                                  hipMemcpyDeviceToHost, h->stream));
        if ((st = sync(h)) != MPS_OK) return st;
        done = 0;
        for (int i = 0; i < count; ++i)
          if (is_multi[i] && rot[i] == 0) ++done;
      }
    }
    if (timed) HIP_TRY(h, hipEventRecord(h->ev_jac[1], h->stream));
    // exact first rotation-free sweep of every multi-launch item
    std::vector<int> hist((size_t)h->max_sweeps * count);
    HIP_TRY(h, hipMemcpyAsync(hist.data(), all[0].rot, sizeof(int) * hist.size(),
                              hipMemcpyDeviceToHost, h->stream));
    if ((st = sync(h)) != MPS_OK) return st;
    for (int i = 0; i < count; ++i)
      if (is_multi[i])
        for (int sw = 0; sw < h->max_sweeps; ++sw)
          if (hist[(size_t)sw * count + i] == 0) {
            first_zero[i] = sw + 1;
            break;
          }
    if (timed) {
      float ms = 0.f;
      HIP_TRY(h, hipEventElapsedTime(&ms, h->ev_jac[0], h->ev_jac[1]));
      h->tm.jacobi_ms += ms;
      for (int i = 0; i < count; ++i) {
        if (!is_multi[i]) continue;
        const double pairs = 0.5 * (double)all[i].n * (all[i].n - 1), m = all[i].m;
        const int sweeps = first_zero[i] > 0 ? first_zero[i] : h->max_sweeps;
        for (int sw = 0; sw < sweeps; ++sw) {
          const double r = hist[(size_t)sw * count + i];
          h->tm.jacobi_flops += r * 32.0 * m + (pairs - r) * 8.0 * m;
        }
      }
    }
  }
  if (join.on) {
    HIP_TRY(h, hipStreamWaitEvent(h->stream, h->ev_join, 0));
    join.on = false;
  }
  // one-launch items report their sweeps themselves
  std::vector<JacItem> one(jp.small);
  one.insert(one.end(), jp.single.begin(), jp.single.end());
  std::vector<int> one_sweeps(one.size());
  for (size_t j = 0; j < one.size(); ++j)
    HIP_TRY(h, hipMemcpyAsync(&one_sweeps[j], one[j].sweeps_done, sizeof(int),
                              hipMemcpyDeviceToHost, h->stream));
  if ((st = sync(h)) != MPS_OK) return st;
  sweeps_out.assign(count, -1);
  for (int i = 0; i < count; ++i)
    if (is_multi[i]) sweeps_out[i] = first_zero[i];
  for (size_t j = 0; j < one.size(); ++j) {
    const int i = (int)(one[j].rot - all[0].rot);
    sweeps_out[i] = one_sweeps[j] > 0 ? one_sweeps[j] : -1;
  }
  for (int v : sweeps_out)
    if (v > 0) h->tm.jacobi_sweeps += v;
  return MPS_OK;
}

// ----------------------------------------------------------------------------
// two-qubit gates (Eqs. C, C~, svd, Bl), one batch of disjoint bonds

// One two-qubit gate of a batch: the handle whose sites (q, q+1) it updates
// and its 4x4 matrix on the device.
struct GateRef {
  mps_state* h;
  int q;
  const double2* u;
};

// Eqs. (C), (C~), (svd), (Bl) for gates on disjoint bonds, possibly of several
// handles (whose streams are idle): one batched contraction, one batched
// Jacobi SVD and one batched site update.  Counters, descriptors and launches
// are the driver's (on its stream); each gate works in its own handle's
// workspace.  Results go to spare buffers.  all_or_nothing: any failed gate
// fails the call and nothing is committed (the single-handle contract);
// otherwise the gates that succeeded are committed and err[b] / msg[b] report
// the failed ones (their handles unchanged).
mps_status apply_2q_refs(mps_state* drv, const std::vector<GateRef>& g, bool all_or_nothing,
                         std::vector<mps_status>& err, std::vector<std::string>& msg) {
  const int items = (int)g.size();
  err.assign(items, MPS_OK);
  msg.assign(items, std::string());
  mps_status st = ensure_counters(drv, items);
  if (st != MPS_OK) return st;
  std::vector<int> slot(items, 0);
  for (int b = 0; b < items; ++b) {
    for (int c = 0; c < b; ++c)
      if (g[c].h == g[b].h) ++slot[b];
    if ((st = ensure_ws(g[b].h, slot[b] + 1)) != MPS_OK) return st;
  }
  std::vector<ThetaItem> th(items);
  std::vector<MixItem> mx(items);
  std::vector<JacItem> jc(items);
  std::vector<FinItem> fn(items);
  std::vector<TruncItem> tr(items);
  int max_rows = 0, max_cols = 0, max_dldr = 0, max_k = 0;
  for (int b = 0; b < items; ++b) {
    mps_state* h = g[b].h;
    const int q = g[b].q;
    const int dl = h->dims[q], dm = h->dims[q + 1], dr = h->dims[q + 2];
    if ((size_t)(2 * dl) * (2 * dr) > h->ws_stride)
      return fail(MPS_ERR_STATE, "internal: workspace too small");
    double2* c = h->ws_c + (size_t)slot[b] * h->ws_stride;
    double2* w = h->ws_w + (size_t)slot[b] * h->ws_stride;
    const int capk = std::min(h->cap[q + 1], std::min(2 * dl, 2 * dr));
    th[b] = ThetaItem{h->cur(q), h->cur(q + 1), c, dl, dm, dr};
    mx[b] = MixItem{c, w, h->lcur(q), g[b].u, drv->d_fro2 + b, dl, dr};
    jc[b] = JacItem{w, drv->d_fro2 + b, drv->d_rot + b, drv->d_sweeps + b, 2 * dl, 2 * dr, 0, 0, items};
    fn[b] = FinItem{w, h->spare(q + 1), h->lspare(q + 1), drv->d_k + b, drv->d_scale + b,
                    drv->d_disc + b, drv->d_status + b, 2 * dl, 2 * dr, capk, h->cutoff, FIN_GATE};
    // Eq. (Bl) with k read on the device: it is enqueued before the host
    // learns k; the result stays in the spare buffers until committed.
    tr[b] = TruncItem{c, h->spare(q + 1), h->spare(q), drv->d_scale + b, drv->d_k + b, 2 * dl, dr, capk};
    max_rows = std::max(max_rows, 2 * dl);
    max_cols = std::max(max_cols, 2 * dr);
    max_dldr = std::max(max_dldr, dl * dr);
    max_k = std::max(max_k, capk);
  }
  // one upload for all descriptors of the batch
  std::vector<char> blob;
  auto place = [&](const void* src, size_t bytes) {
    const size_t o = blob.size();
    blob.resize(o + ((bytes + 255) & ~(size_t)255));
    std::memcpy(blob.data() + o, src, bytes);
    return o;
  };
  const size_t o_th = place(th.data(), sizeof(ThetaItem) * items);
  const size_t o_mx = place(mx.data(), sizeof(MixItem) * items);
  const size_t o_fn = place(fn.data(), sizeof(FinItem) * items);
  const size_t o_tr = place(tr.data(), sizeof(TruncItem) * items);
  const size_t o_jac = blob.size();
  if ((st = ensure_desc(drv, o_jac + 3 * sizeof(JacItem) * items + 512)) != MPS_OK) return st;
  char* d = (char*)drv->d_desc;
  if ((st = upload(drv, d, blob.data(), blob.size())) != MPS_OK) return st;
  HIP_TRY(drv, hipMemsetAsync(drv->d_fro2, 0, sizeof(double) * items, drv->stream));
  HIP_TRY(drv, hipMemsetAsync(drv->d_rot, 0, sizeof(int) * items * drv->max_sweeps, drv->stream));
  HIP_TRY(drv, launch_theta((const ThetaItem*)(d + o_th), items, max_rows, max_cols, drv->stream));
  HIP_TRY(drv, launch_mix((const MixItem*)(d + o_mx), items, max_dldr, drv->stream));
  std::vector<int> sweeps;
  if ((st = run_jacobi(drv, jc, o_jac, sweeps)) != MPS_OK) return st;
  HIP_TRY(drv, launch_finalize((const FinItem*)(d + o_fn), items, drv->stream));
  HIP_TRY(drv, launch_trunc((const TruncItem*)(d + o_tr), items, max_rows, max_k, drv->stream));
  std::vector<int> k(items), status(items);
  std::vector<double> disc(items);
  HIP_TRY(drv, hipMemcpyAsync(k.data(), drv->d_k, sizeof(int) * items, hipMemcpyDeviceToHost, drv->stream));
  HIP_TRY(drv, hipMemcpyAsync(status.data(), drv->d_status, sizeof(int) * items, hipMemcpyDeviceToHost,
                              drv->stream));
  HIP_TRY(drv, hipMemcpyAsync(disc.data(), drv->d_disc, sizeof(double) * items, hipMemcpyDeviceToHost,
                              drv->stream));
  if ((st = sync(drv)) != MPS_OK) return st;
  bool any_bad = false;
  for (int b = 0; b < items; ++b) {
    const std::string where = " (gate on qubit " + std::to_string(g[b].q) + ")";
    if (sweeps[b] < 0 || sweeps[b] > g[b].h->max_sweeps) {
      err[b] = MPS_ERR_NOCONV;
      msg[b] = "Jacobi SVD did not converge within " + std::to_string(g[b].h->max_sweeps) + " sweeps" + where;
    } else if (status[b] != 0) {
      err[b] = MPS_ERR_NONFINITE;
      msg[b] = "non-finite or zero singular values" + where;
    } else if (k[b] < 1 || k[b] > tr[b].k) {
      return fail(MPS_ERR_STATE, "internal: kept rank out of range");
    }
    any_bad = any_bad || err[b] != MPS_OK;
  }
  if (any_bad && all_or_nothing) {
    for (int b = 0; b < items; ++b)
      if (err[b] != MPS_OK) return fail(err[b], msg[b]);
  }
  for (int b = 0; b < items; ++b) {
    if (err[b] != MPS_OK) continue;
    mps_state* h = g[b].h;
    const int q = g[b].q;
    h->site_cur[q] ^= 1;
    h->site_cur[q + 1] ^= 1;
    h->lam_cur[q + 1] ^= 1;
    h->dims[q + 1] = k[b];
    h->discarded += disc[b];
    h->canonical = false;
    ++h->version;
  }
  return MPS_OK;
}

mps_status apply_2q_batch(mps_state* h, const std::vector<int>& qs, const std::vector<int>& gidx) {
  std::vector<GateRef> g(qs.size());
  for (size_t b = 0; b < qs.size(); ++b) g[b] = GateRef{h, qs[b], h->d_gates + (size_t)gidx[b] * 16};
  std::vector<mps_status> err;
  std::vector<std::string> msg;
  return apply_2q_refs(h, g, true, err, msg);
}

// ----------------------------------------------------------------------------
// canonical form: left-to-right orthonormalisation, right-to-left SVD sweep

mps_status canonicalize_impl(mps_state* h) {
  const double t0 = now_ms();
  mps_status st = ensure_ws(h, 1);
  if (st != MPS_OK) return st;
  const int n = h->n;
  const double2 one = make_double2(1.0, 0.0);
  double2* T = h->d_carry[0];
  double2* Tn = h->d_carry[1];
  if ((st = upload(h, T, &one, sizeof(double2))) != MPS_OK) return st;
  if ((st = ensure_desc(h, 4096)) != MPS_OK) return st;  // descriptors of both sweeps
  double2* W0 = h->ws_c;
  double2* W = h->ws_w;
  char* d = nullptr;
  std::vector<int> sweeps;
  int r = 1;  // rows of the carry
  // ---- left to right: M = T B_q (2r x Db); U of its SVD becomes A_q, carry U^+ M
  const std::vector<int> od = h->dims;  // shapes of the B tensors before the sweep
  for (int q = 0; q < n; ++q) {
    const int dg = od[q], db = od[q + 1];
    const int m = 2 * r;
    if ((size_t)db * m > h->ws_stride) return fail(MPS_ERR_STATE, "internal: canon workspace");
    CanonLeftItem cl[2] = {{h->cur(q), T, W0, r, dg, db, 0}, {h->cur(q), T, W0, r, dg, db, 1}};
    FinItem fi{W, h->spare(q), nullptr, h->d_k, h->d_scale, h->d_disc, h->d_status,
               db, m, h->cap[q + 1], kCanonCutoff, FIN_LEFT};
    d = (char*)h->d_desc;
    if ((st = upload(h, d, cl, sizeof(cl))) != MPS_OK) return st;
    if ((st = upload(h, d + 512, &fi, sizeof(fi))) != MPS_OK) return st;
    HIP_TRY(h, launch_canon_left((const CanonLeftItem*)d, 2, db, r, h->stream));
    HIP_TRY(h, launch_copy(W, W0, (size_t)db * m, h->stream));
    HIP_TRY(h, hipMemsetAsync(h->d_fro2, 0, sizeof(double), h->stream));
    HIP_TRY(h, hipMemsetAsync(h->d_rot, 0, sizeof(int) * h->max_sweeps, h->stream));
    HIP_TRY(h, launch_fro2(W, db * m, h->d_fro2, h->stream));
    std::vector<JacItem> jc{JacItem{W, h->d_fro2, h->d_rot, h->d_sweeps, db, m, 0, 0, 1}};
    if ((st = run_jacobi(h, jc, 1024, sweeps)) != MPS_OK) return st;
    if (sweeps[0] < 0) return fail(MPS_ERR_NOCONV, "Jacobi did not converge in canonicalisation");
    HIP_TRY(h, launch_finalize((const FinItem*)(d + 512), 1, h->stream));
    int k = 0, status = 0;
    HIP_TRY(h, hipMemcpyAsync(&k, h->d_k, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipMemcpyAsync(&status, h->d_status, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    if ((st = sync(h)) != MPS_OK) return st;
    if (status != 0) return fail(MPS_ERR_NONFINITE, "non-finite state in canonicalisation");
    CanonCarryLeftItem cc{h->spare(q), W0, Tn, k, m, db};
    if ((st = upload(h, d + 2048, &cc, sizeof(cc))) != MPS_OK) return st;
    HIP_TRY(h, launch_canon_carry_left((const CanonCarryLeftItem*)(d + 2048), 1, k, db, h->stream));
    h->site_cur[q] ^= 1;  // A_q (2, r, k) is now the site tensor
    h->dims[q + 1] = k;
    std::swap(T, Tn);
    r = k;
  }
  // T is the 1x1 carry (norm and phase); A_{n-1} has right bond 1.
  // ---- right to left: M = A_q T (Dl x 2r'); B_q = normalised rows of V^+, lambda_q = sigma
  int rr = 1;
  const std::vector<int> od2 = h->dims;  // shapes of the A tensors after the first sweep
  for (int q = n - 1; q >= 0; --q) {
    const int dl = od2[q], dm = od2[q + 1];
    const int m = 2 * rr;
    if ((size_t)dl * m > h->ws_stride) return fail(MPS_ERR_STATE, "internal: canon workspace");
    CanonRightItem cr[2] = {{h->cur(q), T, W0, dl, dm, rr, 0}, {h->cur(q), T, W0, dl, dm, rr, 1}};
    FinItem fi{W, h->spare(q), h->lspare(q), h->d_k, h->d_scale, h->d_disc, h->d_status,
               dl, m, h->cap[q], kCanonCutoff, FIN_RIGHT};
    d = (char*)h->d_desc;
    if ((st = upload(h, d, cr, sizeof(cr))) != MPS_OK) return st;
    if ((st = upload(h, d + 512, &fi, sizeof(fi))) != MPS_OK) return st;
    HIP_TRY(h, launch_canon_right((const CanonRightItem*)d, 2, dl, rr, h->stream));
    HIP_TRY(h, launch_copy(W, W0, (size_t)dl * m, h->stream));
    HIP_TRY(h, hipMemsetAsync(h->d_fro2, 0, sizeof(double), h->stream));
    HIP_TRY(h, hipMemsetAsync(h->d_rot, 0, sizeof(int) * h->max_sweeps, h->stream));
    HIP_TRY(h, launch_fro2(W, dl * m, h->d_fro2, h->stream));
    std::vector<JacItem> jc{JacItem{W, h->d_fro2, h->d_rot, h->d_sweeps, dl, m, 0, 0, 1}};
    if ((st = run_jacobi(h, jc, 1024, sweeps)) != MPS_OK) return st;
    if (sweeps[0] < 0) return fail(MPS_ERR_NOCONV, "Jacobi did not converge in canonicalisation");
    HIP_TRY(h, launch_finalize((const FinItem*)(d + 512), 1, h->stream));
    int k = 0, status = 0;
    double scale = 0.0;
    HIP_TRY(h, hipMemcpyAsync(&k, h->d_k, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipMemcpyAsync(&status, h->d_status, sizeof(int), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(h, hipMemcpyAsync(&scale, h->d_scale, sizeof(double), hipMemcpyDeviceToHost, h->stream));
    if ((st = sync(h)) != MPS_OK) return st;
    if (status != 0) return fail(MPS_ERR_NONFINITE, "non-finite state in canonicalisation");
    if (q > 0) {
      TruncItem ti{W0, h->spare(q), Tn, h->d_one, nullptr, dl, rr, k};
      if ((st = upload(h, d + 2048, &ti, sizeof(ti))) != MPS_OK) return st;
      HIP_TRY(h, launch_trunc((const TruncItem*)(d + 2048), 1, dl, k, h->stream));
    } else {
      h->norm = scale > 0.0 ? 1.0 / scale : 0.0;
    }
    h->site_cur[q] ^= 1;
    h->lam_cur[q] ^= 1;
    h->dims[q] = k;
    std::swap(T, Tn);
    rr = k;
  }
  if ((st = sync(h)) != MPS_OK) return st;
  h->canonical = true;
  ++h->version;
  h->tm.canon_ms += now_ms() - t0;
  return MPS_OK;
}

// Identity environments from both boundaries (Eq. expec2 with identity
// letters), FP64:  L_0 = [1], L_{b+1} = sum_s B_b^{s+} L_b B_b^s for b < N, so
// that L_N = <psi|psi>;  R_N = [1] and, in the transposed form of the right
// pass, R_b^T = sum_s (B_b^{sT})^+ R_{b+1}^T B_b^{sT} for b >= rmin.  They
// replace diag(lambda^2) and the identity (Eqs. expec1, rc) as trie roots
// when the sites are not in exact canonical form.  Slots and descriptors are
// laid out once by bond capacity; the chains are recomputed only after the
// state changed (e.g. several Pauli sums, or chunks of one, on one state).
mps_status ensure_chain_buffers(mps_state* h) {
  const int n = h->n;
  mps_status st;
  using P = EnvParent<double2>;
  using Ch = EnvChild<double2>;
  if (!h->d_lchain) {
    std::vector<size_t> off(n + 1, 0);
    size_t tot = 0, xmax = 1;
    for (int b = 0; b <= n; ++b) {
      off[b] = tot;
      tot += (size_t)h->cap[b] * h->cap[b];
      if (b < n) xmax = std::max(xmax, (size_t)h->cap[b] * 2 * h->cap[b + 1]);
    }
    // cx: GEMM1 output of the left chain, cxr: of the right chain (the chains
    // may run concurrently), ctr: the transposed site of the right chain
    double2 *lc = nullptr, *rc = nullptr, *cx = nullptr, *cxr = nullptr, *ctr = nullptr;
    void* desc = nullptr;
    auto undo = [&]() {
      dfree(h, lc);
      dfree(h, rc);
      dfree(h, cx);
      dfree(h, cxr);
      dfree(h, ctr);
      dfree(h, desc);
    };
    if ((st = dalloc_t(h, &lc, tot)) != MPS_OK || (st = dalloc_t(h, &rc, tot)) != MPS_OK ||
        (st = dalloc_t(h, &cx, xmax)) != MPS_OK || (st = dalloc_t(h, &cxr, xmax)) != MPS_OK ||
        (st = dalloc_t(h, &ctr, xmax)) != MPS_OK ||
        (st = dalloc(h, &desc, 2 * (sizeof(P) + sizeof(Ch)) * n)) != MPS_OK) {
      undo();
      return st;
    }
    // [left parents | left children | right parents | right children], indexed by site
    std::vector<char> host(2 * (sizeof(P) + sizeof(Ch)) * n);
    P* lp = (P*)host.data();
    Ch* lch = (Ch*)(lp + n);
    P* rp = (P*)(lch + n);
    Ch* rch = (Ch*)(rp + n);
    for (int q = 0; q < n; ++q) {
      lp[q] = P{lc + off[q], cx};
      lch[q] = Ch{cx, lc + off[q + 1], 0};
      rp[q] = P{rc + off[q + 1], cxr};
      rch[q] = Ch{cxr, rc + off[q], 0};
    }
    const double2 one = make_double2(1.0, 0.0);
    hipError_t e = hipMemcpy(desc, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(lc, &one, sizeof(one), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(rc + off[n], &one, sizeof(one), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      undo();
      return dev_fail(h, "identity environment set-up", e);
    }
    h->d_lchain = lc;
    h->d_rchain = rc;
    h->d_chainx = cx;
    h->d_chainxr = cxr;
    h->d_chaintr = ctr;
    h->d_chaindesc = desc;
    h->chain_off = off;
  }
  return MPS_OK;
}

mps_status identity_chains(mps_state* h, int rmin) {
  const int n = h->n;
  mps_status st;
  using P = EnvParent<double2>;
  using Ch = EnvChild<double2>;
  if ((st = ensure_chain_buffers(h)) != MPS_OK) return st;
  if (h->chain_version == h->version && h->chain_rmin <= rmin) return MPS_OK;  // still current
  const P* lp = (const P*)h->d_chaindesc;
  const Ch* lch = (const Ch*)(lp + n);
  const P* rp = (const P*)(lch + n);
  const Ch* rch = (const Ch*)(rp + n);
  // the two chains are independent: the right one runs on the second stream;
  // one item per launch, so the small 32 x 32 tile (four times the
  // workgroups of the default) once the bonds are large
  const bool split = n >= 8;
  hipStream_t rs = h->stream;
  if (split) {
    if ((st = ensure_side(h)) != MPS_OK) return st;
    HIP_TRY(h, hipEventRecord(h->ev_fork, h->stream));
    HIP_TRY(h, hipStreamWaitEvent(h->side, h->ev_fork, 0));
    rs = h->side;
  }
  auto tile = [&](int a, int b) { return std::max(a, b) >= 128 ? 1 : 0; };
  for (int q = 0; q < n; ++q) {
    const int t = tile(h->dims[q], h->dims[q + 1]);
    HIP_TRY(h, launch_env_gemm1_c128(lp + q, 1, h->cur(q), h->dims[q], h->dims[q + 1], h->stream, t));
    HIP_TRY(h, launch_env_gemm2_c128(lch + q, 1, h->cur(q), h->dims[q], h->dims[q + 1], h->stream, t));
  }
  for (int q = n - 1; q >= rmin; --q) {
    const int t = tile(h->dims[q], h->dims[q + 1]);
    HIP_TRY(h, launch_site_prepare(h->cur(q), nullptr, h->d_chaintr, h->dims[q], h->dims[q + 1], 16, rs));
    HIP_TRY(h, launch_env_gemm1_c128(rp + q, 1, h->d_chaintr, h->dims[q + 1], h->dims[q], rs, t));
    HIP_TRY(h, launch_env_gemm2_c128(rch + q, 1, h->d_chaintr, h->dims[q + 1], h->dims[q], rs, t));
  }
  if (split) {
    HIP_TRY(h, hipEventRecord(h->ev_join, h->side));
    HIP_TRY(h, hipStreamWaitEvent(h->stream, h->ev_join, 0));
  }
  h->chain_version = h->version;
  h->chain_rmin = rmin;
  return MPS_OK;
}

// ----------------------------------------------------------------------------
// expectation values

mps_status timed_begin(mps_state* h, std::vector<hipEvent_t>& pool, size_t& used, hipEvent_t& b,
                       hipEvent_t& e) {
  if (used + 2 > pool.size()) {
    const size_t grow = std::max<size_t>(64, pool.size());
    for (size_t i = 0; i < grow; ++i) {
      hipEvent_t ev;
      HIP_TRY(h, hipEventCreate(&ev));
      pool.push_back(ev);
    }
  }
  b = pool[used];
  e = pool[used + 1];
  used += 2;
  HIP_TRY(h, hipEventRecord(b, h->stream));
  return MPS_OK;
}

mps_status flush_timing(mps_state* h) {
  if (!h->timing) return MPS_OK;
  mps_status st = sync(h);
  if (st != MPS_OK) return st;
  for (size_t i = 0; i + 1 < h->ev_env_used; i += 2) {
    float ms = 0.f;
    HIP_TRY(h, hipEventElapsedTime(&ms, h->ev_env[i], h->ev_env[i + 1]));
    h->tm.env_ms += ms;
  }
  for (size_t i = 0; i + 1 < h->ev_close_used; i += 2) {
    float ms = 0.f;
    HIP_TRY(h, hipEventElapsedTime(&ms, h->ev_close[i], h->ev_close[i + 1]));
    h->tm.close_ms += ms;
  }
  h->ev_env_used = h->ev_close_used = 0;
  return MPS_OK;
}

void drop_graph(ExpectSetup& ex) {
  if (ex.gexec) (void)hipGraphExecDestroy(ex.gexec);
  if (ex.graph) (void)hipGraphDestroy(ex.graph);
  ex.gexec = nullptr;
  ex.graph = nullptr;
}

mps_status build_expect(mps_state* h, const mps_psum* ps, int prec) {
  ExpectSetup& ex = h->ex;
  const PauliPlan& P = ps->plan;
  const int n = h->n;
  const bool fwd128 = prec == MPS_PREC_C128 && h->graphs;
  if (ex.plan_serial == ps->serial && ex.prec == prec && ex.dims == h->dims &&
      (prec != MPS_PREC_C128 || ex.fwd128 == fwd128))
    return MPS_OK;
  mps_status st = sync(h);
  if (st != MPS_OK) return st;
  drop_graph(ex);
  const size_t el = prec == MPS_PREC_C128 ? sizeof(double2) : sizeof(float2);
  const std::vector<int>& D = h->dims;
  // ---- environment pool layout
  std::vector<size_t> loff(P.left.size()), roff(P.right.size());
  size_t pool = 0;
  for (size_t i = 0; i < P.left.size(); ++i) {
    loff[i] = pool;
    const size_t d = D[P.left[i].site + 1];
    pool += d * d;
  }
  for (size_t i = 0; i < P.right.size(); ++i) {
    roff[i] = pool;
    const size_t d = D[P.right[i].site];
    pool += d * d;
  }
  std::vector<char> need_l(n + 1, 0), need_r(n + 1, 0);
  for (const TrieNode& nd : P.left)
    if (is_root(nd.parent)) need_l[root_bond(nd.parent)] = 1;
  for (const TrieNode& nd : P.right)
    if (is_root(nd.parent)) need_r[root_bond(nd.parent)] = 1;
  for (int64_t k = 0; k < P.n_terms; ++k) {
    if (is_root(P.close_left[k])) need_l[root_bond(P.close_left[k])] = 1;
    if (is_root(P.close_right[k])) need_r[root_bond(P.close_right[k])] = 1;
  }
  std::vector<size_t> lroot(n + 1, SIZE_MAX), rroot(n + 1, SIZE_MAX);
  for (int b = 0; b <= n; ++b) {
    const size_t d = D[b];
    if (need_l[b]) { lroot[b] = pool; pool += d * d; }
    if (need_r[b]) { rroot[b] = pool; pool += d * d; }
  }
  // ---- prepared sites
  size_t site_elems = 0;
  std::vector<size_t> sfwd(n), str(n);
  for (int q = 0; q < n; ++q) {
    const size_t cnt = 2 * (size_t)D[q] * D[q + 1];
    sfwd[q] = site_elems;
    if (el != sizeof(double2) || fwd128) site_elems += cnt;
    str[q] = site_elems;
    site_elems += cnt;
  }
  // ---- X chunking
  size_t xmax_per = 1;
  for (int q = 0; q < n; ++q) {
    xmax_per = std::max(xmax_per, (size_t)D[q] * 2 * D[q + 1]);
    xmax_per = std::max(xmax_per, (size_t)D[q + 1] * 2 * D[q]);
  }
  const size_t x_budget_elems = std::max(xmax_per, ((size_t)1 << 30) / el);  // ~1 GiB
  const int chunk_cap = (int)std::max<size_t>(1, x_budget_elems / xmax_per);
  // ---- allocate (re-use when large enough)
  auto grow = [&](void** p, size_t& have, size_t want) -> mps_status {
    if (want <= have && *p) return MPS_OK;
    dfree(h, *p);
    *p = nullptr;
    have = 0;
    mps_status s2 = dalloc(h, p, want);
    if (s2 == MPS_OK) have = want;
    return s2;
  };
  if ((st = grow(&ex.pool, ex.pool_bytes, pool * el)) != MPS_OK) return st;
  if ((st = grow(&ex.sites, ex.sites_bytes, site_elems * el)) != MPS_OK) return st;
  // X space actually needed: the largest chunk of distinct parents times its
  // per-parent size, over every site of both passes.
  auto x_need = [&](const std::vector<TrieNode>& nodes) {
    size_t need = 0;
    size_t i = 0;
    while (i < nodes.size()) {
      const int site = nodes[i].site;
      const size_t xper = (size_t)D[site] * 2 * D[site + 1];
      size_t distinct = 0;
      int32_t last = INT32_MIN;
      for (; i < nodes.size() && nodes[i].site == site; ++i)
        if (nodes[i].parent != last) {
          last = nodes[i].parent;
          ++distinct;
        }
      need = std::max(need, std::min<size_t>(distinct, (size_t)chunk_cap) * xper);
    }
    return need;
  };
  const size_t x_elems = std::max<size_t>(1, std::max(x_need(P.left), x_need(P.right)));
  if ((st = grow(&ex.xbuf, ex.xbuf_bytes, x_elems * el)) != MPS_OK) return st;
  char* poolp = (char*)ex.pool;
  char* sitep = (char*)ex.sites;
  auto lref_ptr = [&](int32_t ref) -> char* {
    return is_root(ref) ? poolp + lroot[root_bond(ref)] * el : poolp + loff[ref] * el;
  };
  auto rref_ptr = [&](int32_t ref) -> char* {
    return is_root(ref) ? poolp + rroot[root_bond(ref)] * el : poolp + roff[ref] * el;
  };
  // ---- descriptors
  std::vector<char> host;
  auto put = [&](const void* src, size_t bytes) {
    const size_t o = host.size();
    host.resize(o + ((bytes + 255) & ~(size_t)255));
    if (bytes && src) std::memcpy(host.data() + o, src, bytes);
    return o;
  };
  ex.prep.clear();
  for (int q = 0; q < n; ++q)
    ex.prep.push_back({D[q], D[q + 1], el == sizeof(double2) && !fwd128 ? nullptr : (void*)(sitep + sfwd[q] * el),
                       (void*)(sitep + str[q] * el)});
  ex.roots.clear();
  for (int b = 0; b <= n; ++b)
    if (need_l[b] || need_r[b])
      ex.roots.push_back({b, D[b], need_l[b] ? (void*)(poolp + lroot[b] * el) : nullptr,
                          need_r[b] ? (void*)(poolp + rroot[b] * el) : nullptr});
  ex.n_updates = (int64_t)(P.left.size() + P.right.size());
  auto build_pass = [&](const std::vector<TrieNode>& nodes, const std::vector<size_t>& off,
                        bool left, std::vector<ExpectSetup::EnvLaunch>& out) {
    out.clear();
    size_t i = 0;
    while (i < nodes.size()) {
      const int site = nodes[i].site;
      size_t j = i;
      while (j < nodes.size() && nodes[j].site == site) ++j;
      // left: parent at bond site (Dl = D[site]) -> child at bond site+1
      // right (transposed form): parent at bond site+1 -> child at bond site
      const int dl = left ? D[site] : D[site + 1];
      const int dr = left ? D[site + 1] : D[site];
      const size_t xper = (size_t)dl * 2 * dr;
      size_t a = i;
      while (a < j) {
        // one chunk: up to chunk_cap distinct parents
        std::vector<EnvParent<double2>> par;   // pointers only, reinterpreted per precision
        std::vector<EnvChild<double2>> chi;
        size_t b = a;
        int32_t last_parent = INT32_MIN;
        while (b < j) {
          if (nodes[b].parent != last_parent) {
            if ((int)par.size() == chunk_cap) break;
            last_parent = nodes[b].parent;
            char* pp = left ? lref_ptr(last_parent) : rref_ptr(last_parent);
            par.push_back({(const double2*)pp, (double2*)((char*)ex.xbuf + par.size() * xper * el)});
          }
          chi.push_back({(const double2*)par.back().x, (double2*)(poolp + off[b] * el),
                         (int)nodes[b].letter});
          ++b;
        }
        ExpectSetup::EnvLaunch L;
        L.site = site;
        L.dl = dl;
        L.dr = dr;
        L.n_parents = (int)par.size();
        L.n_children = (int)chi.size();
        L.parents_off = put(par.data(), par.size() * sizeof(par[0]));
        L.children_off = put(chi.data(), chi.size() * sizeof(chi[0]));
        L.left = left;
        L.flops = 8.0 * dl * dl * 2.0 * dr * par.size() + 8.0 * dr * dr * 2.0 * dl * chi.size();
        out.push_back(L);
        a = b;
      }
      i = j;
    }
  };
  build_pass(P.left, loff, true, ex.left_launches);
  build_pass(P.right, roff, false, ex.right_launches);
  // ---- closes: per bond, unique left and right references, reordered so that
  // the pairs strings need cluster into few 64x64 tiles of G (alternating
  // barycentric sorts of the bipartite pair graph), and the list of tiles that
  // hold at least one needed pair.
  std::vector<std::vector<int64_t>> by_bond(n + 1);
  for (int64_t k = 0; k < P.n_terms; ++k) by_bond[P.close_bond[k]].push_back(k);
  std::vector<GramItem> gram;
  std::vector<GramTile> tiles;
  std::vector<int64_t> gidx((size_t)P.n_terms);
  size_t gtot = 0;
  std::vector<std::vector<const void*>> lptrs, rptrs;
  ex.gram_flops = 0.0;
  ex.pair_flops = 0.0;
  for (int c = 0; c <= n; ++c) {
    if (by_bond[c].empty()) continue;
    std::unordered_map<int32_t, int> li, ri;
    std::vector<int32_t> lref, rref;
    std::vector<int> pa, pb;  // pair endpoints (first-appearance indices)
    for (int64_t k : by_bond[c]) {
      auto a = li.emplace(P.close_left[k], (int)lref.size());
      if (a.second) lref.push_back(P.close_left[k]);
      auto b = ri.emplace(P.close_right[k], (int)rref.size());
      if (b.second) rref.push_back(P.close_right[k]);
      pa.push_back(a.first->second);
      pb.push_back(b.first->second);
    }
    const int nl = (int)lref.size(), nr = (int)rref.size();
    {  // the method's own work: Re Tr(L R) = 4 D^2 FLOPs per distinct pair
      std::unordered_set<int64_t> distinct;
      for (size_t q = 0; q < pa.size(); ++q) distinct.insert((int64_t)pa[q] * nr + pb[q]);
      ex.pair_flops += 4.0 * (double)distinct.size() * D[c] * D[c];
    }
    std::vector<int> lpos(nl), rpos(nr);
    for (int i = 0; i < nl; ++i) lpos[i] = i;
    for (int i = 0; i < nr; ++i) rpos[i] = i;
    if (nl > 64 && nr > 64) {
      std::vector<double> key;
      std::vector<int> cnt, order;
      for (int it = 0; it < 8; ++it) {
        for (int side = 0; side < 2; ++side) {
          const int cnt_n = side == 0 ? nl : nr;
          key.assign(cnt_n, 0.0);
          cnt.assign(cnt_n, 0);
          for (size_t q = 0; q < pa.size(); ++q) {
            const int self = side == 0 ? pa[q] : pb[q];
            const int other = side == 0 ? rpos[pb[q]] : lpos[pa[q]];
            key[self] += other;
            cnt[self] += 1;
          }
          order.resize(cnt_n);
          for (int i = 0; i < cnt_n; ++i) order[i] = i;
          std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
            return key[x] * cnt[y] < key[y] * cnt[x];
          });
          std::vector<int>& pos = side == 0 ? lpos : rpos;
          for (int i = 0; i < cnt_n; ++i) pos[order[i]] = i;
        }
      }
    }
    std::vector<const void*> lp(nl), rp(nr);
    for (int i = 0; i < nl; ++i) lp[lpos[i]] = lref_ptr(lref[i]);
    for (int i = 0; i < nr; ++i) rp[rpos[i]] = rref_ptr(rref[i]);
    const int item = (int)gram.size();
    std::vector<char> used((size_t)((nl + 63) / 64) * ((nr + 63) / 64), 0);
    const int tcols = (nr + 63) / 64;
    for (size_t q = 0; q < pa.size(); ++q) {
      const int a = lpos[pa[q]], b = rpos[pb[q]];
      gidx[by_bond[c][q]] = (int64_t)gtot + (int64_t)a * nr + b;
      char& u = used[(size_t)(a / 64) * tcols + b / 64];
      if (!u) {
        u = 1;
        tiles.push_back(GramTile{item, (a / 64) * 64, (b / 64) * 64});
      }
    }
    GramItem gi{nullptr, nullptr, (double*)(uintptr_t)gtot, nl, nr, D[c] * D[c]};
    gram.push_back(gi);
    lptrs.push_back(std::move(lp));
    rptrs.push_back(std::move(rp));
    gtot += (size_t)nl * nr;
  }
  for (const GramTile& t : tiles) {
    const GramItem& b = gram[t.item];
    ex.gram_flops += 4.0 * std::min(64, b.nl - t.r0) * std::min(64, b.nr - t.c0) * (double)b.kdim;
  }
  if (gtot > ex.gbuf_count || !ex.gbuf) {
    dfree(h, ex.gbuf);
    ex.gbuf = nullptr;
    if ((st = dalloc_t(h, &ex.gbuf, std::max<size_t>(gtot, 1))) != MPS_OK) return st;
    ex.gbuf_count = gtot;
  }
  // pointer lists go into the descriptor blob; patch addresses after upload placement
  std::vector<size_t> lp_off(gram.size()), rp_off(gram.size());
  for (size_t g = 0; g < gram.size(); ++g) {
    lp_off[g] = put(lptrs[g].data(), lptrs[g].size() * sizeof(void*));
    rp_off[g] = put(rptrs[g].data(), rptrs[g].size() * sizeof(void*));
  }
  ex.gram_items = (int)gram.size();
  int max_kdim = 0;
  for (const GramItem& gi : gram) max_kdim = std::max(max_kdim, gi.kdim);
  ex.gram_split = gram_splits(max_kdim);
  if (ex.gram_split > 1) {
    const size_t need = (size_t)ex.gram_split * tiles.size() * 4096;
    if (need > ex.gpart_count || !ex.gpart) {
      dfree(h, ex.gpart);
      ex.gpart = nullptr;
      ex.gpart_count = 0;
      if ((st = dalloc_t(h, &ex.gpart, std::max<size_t>(need, 1))) != MPS_OK) return st;
      ex.gpart_count = need;
    }
  }
  ex.gram_off = put(nullptr, gram.size() * sizeof(GramItem));
  ex.gram_tiles = (int)tiles.size();
  ex.tiles_off = put(tiles.data(), tiles.size() * sizeof(GramTile));
  // terms
  const size_t T = (size_t)P.n_terms;
  if (T > ex.terms_cap || !ex.per_term) {
    for (void* p : {(void*)ex.per_term, (void*)ex.coeffs, (void*)ex.gidx, (void*)ex.energy})
      dfree(h, p);
    ex.per_term = ex.coeffs = ex.energy = nullptr;
    ex.gidx = nullptr;
    const size_t tc = std::max<size_t>(T, 1);
    if ((st = dalloc_t(h, &ex.per_term, tc)) != MPS_OK) return st;
    if ((st = dalloc_t(h, &ex.coeffs, tc)) != MPS_OK) return st;
    if ((st = dalloc_t(h, &ex.gidx, tc)) != MPS_OK) return st;
    if ((st = dalloc_t(h, &ex.energy, 2)) != MPS_OK) return st;  // compensated (sum, error)
    ex.terms_cap = tc;
  }
  // ---- upload the blob
  if (host.size() > ex.desc_bytes || !ex.desc) {
    dfree(h, ex.desc);
    ex.desc = nullptr;
    ex.desc_bytes = 0;
    if ((st = dalloc(h, &ex.desc, host.size() + 256)) != MPS_OK) return st;
    ex.desc_bytes = host.size() + 256;
  }
  char* db = (char*)ex.desc;
  for (size_t g = 0; g < gram.size(); ++g) {
    gram[g].lptr = (const void* const*)(db + lp_off[g]);
    gram[g].rptr = (const void* const*)(db + rp_off[g]);
    gram[g].g = ex.gbuf + (size_t)(uintptr_t)gram[g].g;
  }
  if (!gram.empty()) std::memcpy(host.data() + ex.gram_off, gram.data(), gram.size() * sizeof(GramItem));
  HIP_TRY(h, hipMemcpy(ex.desc, host.data(), host.size(), hipMemcpyHostToDevice));
  ex.host_desc = host;
  ex.plan_terms = T;
  if (T) {
    HIP_TRY(h, hipMemcpy(ex.gidx, gidx.data(), T * sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(ex.coeffs, P.coeffs.data(), T * sizeof(double), hipMemcpyHostToDevice));
  }
  ex.plan_serial = ps->serial;
  ex.prec = prec;
  ex.dims = D;
  ex.fwd128 = fwd128;
  return MPS_OK;
}

// ----------------------------------------------------------------------------
// tile autotuner for the environment GEMMs (c128, c64)
//
// A launch class is (device, precision, GEMM half, D_l, D_r, ceil(log2 items)).
// The first expectation that meets a class it has no entry for times every
// tile shape on that launch, twice, and keeps the fastest; the table is
// process-wide per device.  All shapes give bitwise-identical results, so
// tuning changes speed only.

struct TuneKey {
  int dev, prec, half, dl, dr, bucket;
  bool operator<(const TuneKey& o) const {
    const int a[6] = {dev, prec, half, dl, dr, bucket}, b[6] = {o.dev, o.prec, o.half, o.dl, o.dr, o.bucket};
    return std::lexicographical_compare(a, a + 6, b, b + 6);
  }
};
struct TuneEntry {
  int tile = 0;
  float ms[kEnvTiles] = {};
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;

struct TunePending {
  TuneKey key;
  size_t ev0;  // first event of 2 reps x kEnvTiles x (begin, end)
};

int tune_bucket(int items) {
  int b = 0;
  while ((1 << b) < items) ++b;
  return b;
}

TuneKey tune_key(const mps_state* h, int prec, int half, const ExpectSetup::EnvLaunch& L) {
  return TuneKey{h->device, prec, half, L.dl, L.dr, tune_bucket(half == 1 ? L.n_parents : L.n_children)};
}

// 0: no entry yet (default tile), else the tuned tile.
int tuned_tile(const TuneKey& k, bool* known) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  auto it = g_tune.find(k);
  *known = it != g_tune.end();
  return *known ? it->second.tile : 0;
}

hipError_t env_half(mps_state* h, const ExpectSetup::EnvLaunch& L, int prec, int half, const void* site,
                    int tile) {
  const char* db = (const char*)h->ex.desc;
  if (prec == MPS_PREC_C128)
    return half == 1 ? launch_env_gemm1_c128((const EnvParent<double2>*)(db + L.parents_off), L.n_parents,
                                             (const double2*)site, L.dl, L.dr, h->stream, tile)
                     : launch_env_gemm2_c128((const EnvChild<double2>*)(db + L.children_off), L.n_children,
                                             (const double2*)site, L.dl, L.dr, h->stream, tile);
  if (prec == MPS_PREC_C64)
    return half == 1 ? launch_env_gemm1_c64((const EnvParent<float2>*)(db + L.parents_off), L.n_parents,
                                            (const float2*)site, L.dl, L.dr, h->stream, tile)
                     : launch_env_gemm2_c64((const EnvChild<float2>*)(db + L.children_off), L.n_children,
                                            (const float2*)site, L.dl, L.dr, h->stream, tile);
  const int f16 = prec == MPS_PREC_SPLIT_F16;
  return half == 1 ? launch_env_gemm1_split((const EnvParent<float2>*)(db + L.parents_off), L.n_parents,
                                            (const float2*)site, L.dl, L.dr, f16, h->stream)
                   : launch_env_gemm2_split((const EnvChild<float2>*)(db + L.children_off), L.n_children,
                                            (const float2*)site, L.dl, L.dr, f16, h->stream);
}

mps_status run_env_launch(mps_state* h, const ExpectSetup::EnvLaunch& L, int prec,
                          std::vector<TunePending>* pending, bool capturing) {
  // c128 without a fixed copy reads the live site buffer (it flips with every gate)
  const void* site_ptr = L.left ? (h->ex.prep[L.site].fwd ? h->ex.prep[L.site].fwd
                                                          : (const void*)h->cur(L.site))
                                : h->ex.prep[L.site].tr;
  const bool tunable = h->autotune && (prec == MPS_PREC_C128 || prec == MPS_PREC_C64);
  int tile[3] = {0, 0, 0};
  bool tune[3] = {false, false, false};
  if (tunable)
    for (int half = 1; half <= 2; ++half) {
      bool known = false;
      const TuneKey k = tune_key(h, prec, half, L);
      tile[half] = tuned_tile(k, &known);
      if (!known && pending) {
        bool queued = false;
        for (const TunePending& p : *pending)
          if (!(p.key < k) && !(k < p.key)) queued = true;
        tune[half] = !queued;
      }
    }
  if (h->forced_tile >= 0 && (prec == MPS_PREC_C128 || prec == MPS_PREC_C64)) {
    tile[1] = tile[2] = h->forced_tile;
    tune[1] = tune[2] = false;
  }
  mps_status st;
  if (tune[1] || tune[2]) {
    // a tuning launch: every tile shape twice, bracketed by events; not counted
    // in the environment timing
    for (int half = 1; half <= 2; ++half) {
      if (!tune[half]) {
        HIP_TRY(h, env_half(h, L, prec, half, site_ptr, tile[half]));
        continue;
      }
      const size_t need = h->ev_tune_used + 4 * kEnvTiles;
      while (h->ev_tune.size() < need) {
        hipEvent_t ev;
        HIP_TRY(h, hipEventCreate(&ev));
        h->ev_tune.push_back(ev);
      }
      pending->push_back(TunePending{tune_key(h, prec, half, L), h->ev_tune_used});
      for (int rep = 0; rep < 2; ++rep)
        for (int t = 0; t < kEnvTiles; ++t) {
          HIP_TRY(h, hipEventRecord(h->ev_tune[h->ev_tune_used++], h->stream));
          HIP_TRY(h, env_half(h, L, prec, half, site_ptr, t));
          HIP_TRY(h, hipEventRecord(h->ev_tune[h->ev_tune_used++], h->stream));
        }
    }
    return MPS_OK;
  }
  hipEvent_t b = nullptr, e = nullptr;
  const bool timed = h->timing && !capturing;
  if (timed && (st = timed_begin(h, h->ev_env, h->ev_env_used, b, e)) != MPS_OK) return st;
  HIP_TRY(h, env_half(h, L, prec, 1, site_ptr, tile[1]));
  HIP_TRY(h, env_half(h, L, prec, 2, site_ptr, tile[2]));
  if (timed) {
    HIP_TRY(h, hipEventRecord(e, h->stream));
    h->tm.env_launches += 2;
    h->tm.env_flops += L.flops;
  }
  return MPS_OK;
}

// After the stream has drained: the fastest tile of every class tuned in this pass.
mps_status finish_tuning(mps_state* h, const std::vector<TunePending>& pending) {
  for (const TunePending& p : pending) {
    TuneEntry en;
    float best = 0.f;
    for (int t = 0; t < kEnvTiles; ++t) {
      float m = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        const size_t i = p.ev0 + 2 * ((size_t)rep * kEnvTiles + t);
        float ms = 0.f;
        HIP_TRY(h, hipEventElapsedTime(&ms, h->ev_tune[i], h->ev_tune[i + 1]));
        m = rep == 0 ? ms : std::min(m, ms);
      }
      en.ms[t] = m;
      if (t == 0 || m < best) {
        best = m;
        en.tile = t;
      }
    }
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[p.key] = en;
  }
  h->ev_tune_used = 0;
  return MPS_OK;
}

// Linear combinations of the string expectations (CSR, host arrays).
struct RowsSpec {
  int64_t n_rows, nnz;
  const int64_t* row_ptr;
  const int64_t* cols;
  const double* vals;
  double* out;
};

// pair_out (device, may be null) receives the energy's compensated (sum,
// error) pair, for sums over several plans added on the device.
// The expectation's set-up on h's stream: the plan's device layout, the site
// tensors in environment precision (and transposed), the trie roots.  *nrm:
// the device value <psi|psi> to divide by (boundary environments), or null in
// exact canonical form.
mps_status expect_open(mps_state* h, const mps_psum* ps, int prec, const double2** nrm_out) {
  mps_status st;
  if ((st = build_expect(h, ps, prec)) != MPS_OK) return st;
  ExpectSetup& ex = h->ex;
  const int el = prec == MPS_PREC_C128 ? 16 : 8;
  // layer 0: site tensors in environment precision and transposed; trie roots
  for (int q = 0; q < h->n; ++q)
    HIP_TRY(h, launch_site_prepare(h->cur(q), ex.prep[q].fwd, ex.prep[q].tr, ex.prep[q].dl,
                                   ex.prep[q].dr, el, h->stream));
  // Exact canonical form: diag(lambda^2) and identity roots, unit norm.  After
  // gates (truncated Hastings updates leave the sites only nearly
  // right-orthonormal and the norm near 1): identity environments from both
  // boundaries and division by <psi|psi>, the same values without a sweep.
  const bool chains = !h->canonical;
  const double2* nrm = nullptr;
  if (chains) {
    int rmin = h->n;
    for (const auto& r : ex.roots)
      if (r.rroot) rmin = std::min(rmin, r.bond);
    if ((st = identity_chains(h, rmin)) != MPS_OK) return st;
    nrm = h->d_lchain + h->chain_off[h->n];
    for (const auto& r : ex.roots) {
      const size_t cnt = (size_t)r.d * r.d;
      if (r.lroot)
        HIP_TRY(h, launch_root_copy(h->d_lchain + h->chain_off[r.bond], r.lroot, cnt, el, h->stream));
      if (r.rroot)
        HIP_TRY(h, launch_root_copy(h->d_rchain + h->chain_off[r.bond], r.rroot, cnt, el, h->stream));
    }
  } else {
    for (const auto& r : ex.roots)
      HIP_TRY(h, launch_roots(h->lcur(r.bond), r.lroot, r.rroot, r.d, el, h->stream));
  }
  *nrm_out = nrm;
  return MPS_OK;
}

// The closing traces (a11), per-string values normalised by *nrm (a9) and the
// compensated energy (a12) of h's current plan, on stream s.
mps_status expect_close(mps_state* h, int el, const double2* nrm, hipStream_t s) {
  const ExpectSetup& ex = h->ex;
  const int64_t T = ex.plan_terms;
  HIP_TRY(h, launch_gram((const GramItem*)((char*)ex.desc + ex.gram_off),
                         (const GramTile*)((char*)ex.desc + ex.tiles_off), ex.gram_tiles, el, ex.gpart,
                         ex.gram_split, s));
  HIP_TRY(h, launch_gather(ex.gbuf, ex.gidx, nrm, ex.per_term, T, s));
  HIP_TRY(h, launch_energy(ex.per_term, ex.coeffs, T, ex.energy, s));
  return MPS_OK;
}

mps_status expect_impl(mps_state* h, const mps_psum* ps, int prec, double* energy,
                       double* per_term, const RowsSpec* rows = nullptr, double* pair_out = nullptr) {
  mps_status st;
  const double t0 = now_ms();
  const double2* nrm = nullptr;
  if ((st = expect_open(h, ps, prec, &nrm)) != MPS_OK) return st;
  ExpectSetup& ex = h->ex;
  const int el = prec == MPS_PREC_C128 ? 16 : 8;
  const bool chains = nrm != nullptr;
  std::vector<TunePending> pending;
  h->ev_tune_used = 0;
  const int64_t T = ps->plan.n_terms;
  // Environment launches, closes, gather and energy: from fixed buffers only
  // (prepared sites, roots, pool, descriptors), so with graphs enabled they
  // are captured once per (plan, precision, bond dims, root kind) and replayed.
  auto device_sequence = [&](bool capturing) -> mps_status {
    mps_status s2;
    for (const auto& L : ex.left_launches)
      if ((s2 = run_env_launch(h, L, prec, capturing ? nullptr : &pending, capturing)) != MPS_OK) return s2;
    for (const auto& L : ex.right_launches)
      if ((s2 = run_env_launch(h, L, prec, capturing ? nullptr : &pending, capturing)) != MPS_OK) return s2;
    hipEvent_t b = nullptr, e = nullptr;
    const bool timed = h->timing && !capturing;
    if (timed && (s2 = timed_begin(h, h->ev_close, h->ev_close_used, b, e)) != MPS_OK) return s2;
    HIP_TRY(h, launch_gram((const GramItem*)((char*)ex.desc + ex.gram_off),
                           (const GramTile*)((char*)ex.desc + ex.tiles_off), ex.gram_tiles, el, ex.gpart,
                           ex.gram_split,
                           h->stream));
    if (timed) {
      HIP_TRY(h, hipEventRecord(e, h->stream));
      h->tm.close_flops += ex.pair_flops;
      h->tm.close_tile_flops += ex.gram_flops;
    }
    if (!capturing && h->timing) h->tm.env_updates += ex.n_updates;
    HIP_TRY(h, launch_gather(ex.gbuf, ex.gidx, nrm, ex.per_term, T, h->stream));
    HIP_TRY(h, launch_energy(ex.per_term, ex.coeffs, T, ex.energy, h->stream));
    return MPS_OK;
  };
  // a graph only once every tile of this sequence is known (tuning runs eagerly)
  bool use_graph = h->graphs;
  if (use_graph && h->autotune && h->forced_tile < 0 && (prec == MPS_PREC_C128 || prec == MPS_PREC_C64))
    for (int pass = 0; pass < 2 && use_graph; ++pass)
      for (const auto& L : pass == 0 ? ex.left_launches : ex.right_launches) {
        bool k1 = false, k2 = false;
        tuned_tile(tune_key(h, prec, 1, L), &k1);
        tuned_tile(tune_key(h, prec, 2, L), &k2);
        if (!k1 || !k2) {
          use_graph = false;
          break;
        }
      }
  if (use_graph) {
    if (ex.gexec && ex.graph_chains != chains) drop_graph(ex);
    if (!ex.gexec) {
      HIP_TRY(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
      const mps_status s_seq = device_sequence(true);
      hipGraph_t g = nullptr;
      const hipError_t e_end = hipStreamEndCapture(h->stream, &g);
      if (s_seq != MPS_OK) {
        if (g) (void)hipGraphDestroy(g);
        return s_seq;
      }
      if (e_end != hipSuccess) return dev_fail(h, "hipStreamEndCapture", e_end);
      ex.graph = g;
      const hipError_t e_inst = hipGraphInstantiate(&ex.gexec, g, nullptr, nullptr, 0);
      if (e_inst != hipSuccess) {
        ex.gexec = nullptr;
        drop_graph(ex);
        return dev_fail(h, "hipGraphInstantiate", e_inst);
      }
      ex.graph_chains = chains;
    }
    HIP_TRY(h, hipGraphLaunch(ex.gexec, h->stream));
    if (h->timing) h->tm.graph_launches += 1;
  } else if ((st = device_sequence(false)) != MPS_OK) {
    return st;
  }
  double E2[2] = {0.0, 0.0};
  double2 nn = make_double2(1.0, 0.0);
  if (pair_out)
    HIP_TRY(h, hipMemcpyAsync(pair_out, ex.energy, 2 * sizeof(double), hipMemcpyDeviceToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(E2, ex.energy, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if (nrm) HIP_TRY(h, hipMemcpyAsync(&nn, nrm, sizeof(double2), hipMemcpyDeviceToHost, h->stream));
  if (per_term && T)
    HIP_TRY(h, hipMemcpyAsync(per_term, ex.per_term, sizeof(double) * T, hipMemcpyDeviceToHost,
                              h->stream));
  if (rows && rows->n_rows > 0) {
    const size_t need = sizeof(int64_t) * (rows->n_rows + 1 + rows->nnz) + sizeof(double) * (rows->nnz + rows->n_rows);
    if (need > ex.rows_bytes) {
      if ((st = sync(h)) != MPS_OK) return st;
      dfree(h, ex.rows_buf);
      ex.rows_buf = nullptr;
      ex.rows_bytes = 0;
      if ((st = dalloc(h, &ex.rows_buf, need)) != MPS_OK) return st;
      ex.rows_bytes = need;
    }
    int64_t* d_ptr = (int64_t*)ex.rows_buf;
    int64_t* d_cols = d_ptr + rows->n_rows + 1;
    double* d_vals = (double*)(d_cols + rows->nnz);
    double* d_out = d_vals + rows->nnz;
    HIP_TRY(h, hipMemcpyAsync(d_ptr, rows->row_ptr, sizeof(int64_t) * (rows->n_rows + 1), hipMemcpyHostToDevice,
                              h->stream));
    if (rows->nnz) {
      HIP_TRY(h, hipMemcpyAsync(d_cols, rows->cols, sizeof(int64_t) * rows->nnz, hipMemcpyHostToDevice, h->stream));
      HIP_TRY(h, hipMemcpyAsync(d_vals, rows->vals, sizeof(double) * rows->nnz, hipMemcpyHostToDevice, h->stream));
    }
    HIP_TRY(h, launch_rows(ex.per_term, d_ptr, d_cols, d_vals, rows->n_rows, d_out, h->stream));
    HIP_TRY(h, hipMemcpyAsync(rows->out, d_out, sizeof(double) * rows->n_rows, hipMemcpyDeviceToHost, h->stream));
  }
  if ((st = sync(h)) != MPS_OK) return st;
  if ((st = flush_timing(h)) != MPS_OK) return st;
  if (!pending.empty() && (st = finish_tuning(h, pending)) != MPS_OK) return st;
  if (!(nn.x > 0.0) || !std::isfinite(nn.x)) return fail(MPS_ERR_NONFINITE, "state norm is zero or not finite");
  if (nrm) h->norm = std::sqrt(nn.x);
  *energy = E2[0] + E2[1];
  h->tm.expect_ms += now_ms() - t0;
  return MPS_OK;
}

// Several MPSs, each with its own plan, evaluated together, every step that
// launches per site or per trie node merged over the states: one launch
// prepares all states' site tensors, each depth of the boundary-environment
// chains (FP64, Eq. expec2 with identity letters) is one launch per GEMM half
// for all states whose chains are stale, one launch fills all roots, and the
// environment updates of equal depth in the states' trie sequences are one
// launch per GEMM half (every item carries its own site tensor and dims);
// then each state's closes, gather and energy.  All on the first state's
// stream.  Per-element accumulation order is that of the single-state path
// (every tile shape takes K in the same 16x16x4 steps), so the values equal
// those of one expectation per state bit for bit.
mps_status expect_multi_impl(mps_state* const* hs, const mps_psum* const* ps, int count, int prec,
                             double* energies, double* const* per_term) {
  mps_state* drv = hs[0];
  const int el = prec == MPS_PREC_C128 ? 16 : 8;
  const double t0 = now_ms();
  mps_status st;
  std::vector<const double2*> nrm(count, nullptr);
  std::vector<int> rmin(count, 0), stale(count, 0);
  int max_n = 0;
  for (int i = 0; i < count; ++i) {
    mps_state* h = hs[i];
    if ((st = build_expect(h, ps[i], prec)) != MPS_OK) return st;
    if (h->stream != drv->stream && (st = sync(h)) != MPS_OK) return st;  // h's earlier work done
    max_n = std::max(max_n, h->n);
    if (h->canonical) continue;
    if ((st = ensure_chain_buffers(h)) != MPS_OK) return st;
    rmin[i] = h->n;
    for (const auto& r : h->ex.roots)
      if (r.rroot) rmin[i] = std::min(rmin[i], r.bond);
    stale[i] = !(h->chain_version == h->version && h->chain_rmin <= rmin[i]);
    nrm[i] = h->d_lchain + h->chain_off[h->n];
  }
  using P = EnvParent<double2>;  // pointer layout shared by every precision
  using Ch = EnvChild<double2>;
  std::vector<char> blob;
  auto put = [&](const void* src, size_t bytes) {
    const size_t o = blob.size();
    blob.resize(o + ((bytes + 255) & ~(size_t)255));
    if (src && bytes) std::memcpy(blob.data() + o, src, bytes);
    return o;
  };
  struct Gemms {  // one merged launch per GEMM half
    size_t par_off = 0, chi_off = 0;
    int n_par = 0, n_chi = 0, max_dl = 0, max_dr = 0;
  };
  struct Preps {
    size_t off = 0;
    int n = 0, max_elems = 0;
  };
  auto put_preps = [&](const std::vector<PrepItem>& v) {
    Preps r;
    r.n = (int)v.size();
    for (const PrepItem& it : v) r.max_elems = std::max(r.max_elems, 2 * it.dl * it.dr);
    r.off = put(v.data(), v.size() * sizeof(PrepItem));
    return r;
  };
  auto put_gemms = [&](const std::vector<P>& par, const std::vector<Ch>& chi) {
    Gemms g;
    g.n_par = (int)par.size();
    g.n_chi = (int)chi.size();
    for (const P& x : par) {
      g.max_dl = std::max(g.max_dl, x.dl);
      g.max_dr = std::max(g.max_dr, x.dr);
    }
    g.par_off = put(par.data(), par.size() * sizeof(P));
    g.chi_off = put(chi.data(), chi.size() * sizeof(Ch));
    return g;
  };
  // (1) every state's sites in environment precision (and transposed)
  std::vector<PrepItem> pv;
  for (int i = 0; i < count; ++i)
    for (int q = 0; q < hs[i]->n; ++q) {
      const auto& pr = hs[i]->ex.prep[q];
      pv.push_back(PrepItem{hs[i]->cur(q), pr.fwd, pr.tr, pr.dl, pr.dr});
    }
  const Preps site_preps = put_preps(pv);
  // (2) boundary-environment chains of the stale states, depth by depth
  std::vector<Gemms> left_chain;
  for (int q = 0; q < max_n; ++q) {
    std::vector<P> par;
    std::vector<Ch> chi;
    for (int i = 0; i < count; ++i) {
      mps_state* h = hs[i];
      if (!stale[i] || q >= h->n) continue;
      const int dl = h->dims[q], dr = h->dims[q + 1];
      double2* lc = h->d_lchain;
      par.push_back(P{lc + h->chain_off[q], h->d_chainx, h->cur(q), dl, dr});
      chi.push_back(Ch{h->d_chainx, lc + h->chain_off[q + 1], 0, dl, dr, h->cur(q)});
    }
    if (!par.empty()) left_chain.push_back(put_gemms(par, chi));
  }
  std::vector<std::pair<Preps, Gemms>> right_chain;
  for (int t = 0; t < max_n; ++t) {
    std::vector<PrepItem> tv;
    std::vector<P> par;
    std::vector<Ch> chi;
    for (int i = 0; i < count; ++i) {
      mps_state* h = hs[i];
      const int q = h->n - 1 - t;
      if (!stale[i] || q < rmin[i] || q < 0) continue;
      const int dl = h->dims[q + 1], dr = h->dims[q];  // transposed form
      double2* rc = h->d_rchain;
      tv.push_back(PrepItem{h->cur(q), nullptr, h->d_chaintr, h->dims[q], h->dims[q + 1]});
      par.push_back(P{rc + h->chain_off[q + 1], h->d_chainxr, h->d_chaintr, dl, dr});
      chi.push_back(Ch{h->d_chainxr, rc + h->chain_off[q], 0, dl, dr, h->d_chaintr});
    }
    if (!par.empty()) right_chain.push_back({put_preps(tv), put_gemms(par, chi)});
  }
  // (3) roots from the chains
  std::vector<CopyItem> cv;
  long long copy_max = 0;
  for (int i = 0; i < count; ++i) {
    mps_state* h = hs[i];
    if (h->canonical) continue;
    for (const auto& r : h->ex.roots) {
      const long long cnt = (long long)r.d * r.d;
      if (r.lroot) cv.push_back(CopyItem{h->d_lchain + h->chain_off[r.bond], r.lroot, cnt});
      if (r.rroot) cv.push_back(CopyItem{h->d_rchain + h->chain_off[r.bond], r.rroot, cnt});
      copy_max = std::max(copy_max, cnt);
    }
  }
  const size_t copy_off = put(cv.data(), cv.size() * sizeof(CopyItem));
  // (4) environment updates of equal trie depth: [left depth 0, 1, ...][right depth 0, 1, ...]
  std::vector<Gemms> env;
  for (int pass = 0; pass < 2; ++pass) {
    size_t depth = 0;
    for (int i = 0; i < count; ++i) {
      const auto& ls = pass == 0 ? hs[i]->ex.left_launches : hs[i]->ex.right_launches;
      depth = std::max(depth, ls.size());
    }
    for (size_t t = 0; t < depth; ++t) {
      std::vector<P> par;
      std::vector<Ch> chi;
      for (int i = 0; i < count; ++i) {
        mps_state* h = hs[i];
        const auto& ls = pass == 0 ? h->ex.left_launches : h->ex.right_launches;
        if (t >= ls.size()) continue;
        const ExpectSetup::EnvLaunch& L = ls[t];
        // the site tensor the single-state launch would take (run_env_launch)
        const void* site = L.left ? (h->ex.prep[L.site].fwd ? h->ex.prep[L.site].fwd
                                                            : (const void*)h->cur(L.site))
                                  : h->ex.prep[L.site].tr;
        const P* sp = (const P*)(h->ex.host_desc.data() + L.parents_off);
        const Ch* sc = (const Ch*)(h->ex.host_desc.data() + L.children_off);
        for (int k = 0; k < L.n_parents; ++k) {
          P x = sp[k];
          x.site = (const double2*)site;
          x.dl = L.dl;
          x.dr = L.dr;
          par.push_back(x);
        }
        for (int k = 0; k < L.n_children; ++k) {
          Ch x = sc[k];
          x.site = (const double2*)site;
          x.dl = L.dl;
          x.dr = L.dr;
          chi.push_back(x);
        }
      }
      env.push_back(put_gemms(par, chi));
    }
  }
  if ((st = ensure_desc(drv, blob.size() + 256)) != MPS_OK) return st;
  char* d = (char*)drv->d_desc;
  if ((st = upload(drv, d, blob.data(), blob.size())) != MPS_OK) return st;
  hipStream_t s = drv->stream;
  auto run_preps = [&](const Preps& p, int elem) -> hipError_t {
    return launch_site_prepare_list((const PrepItem*)(d + p.off), p.n, p.max_elems, elem, s);
  };
  // launch-level site null: every item names its own; the dims size the grid
  auto run_gemms = [&](const Gemms& g, int pr) -> hipError_t {
    const P* dp = (const P*)(d + g.par_off);
    const Ch* dc = (const Ch*)(d + g.chi_off);
    hipError_t e;
    if (pr == MPS_PREC_C128) {
      e = launch_env_gemm1_c128(dp, g.n_par, nullptr, g.max_dl, g.max_dr, s, 0);
      return e != hipSuccess ? e : launch_env_gemm2_c128(dc, g.n_chi, nullptr, g.max_dl, g.max_dr, s, 0);
    }
    if (pr == MPS_PREC_C64) {
      e = launch_env_gemm1_c64((const EnvParent<float2>*)dp, g.n_par, nullptr, g.max_dl, g.max_dr, s, 0);
      return e != hipSuccess ? e
                             : launch_env_gemm2_c64((const EnvChild<float2>*)dc, g.n_chi, nullptr, g.max_dl,
                                                    g.max_dr, s, 0);
    }
    const int f16 = pr == MPS_PREC_SPLIT_F16;
    e = launch_env_gemm1_split((const EnvParent<float2>*)dp, g.n_par, nullptr, g.max_dl, g.max_dr, f16, s);
    return e != hipSuccess ? e
                           : launch_env_gemm2_split((const EnvChild<float2>*)dc, g.n_chi, nullptr, g.max_dl,
                                                    g.max_dr, f16, s);
  };
  HIP_TRY(drv, run_preps(site_preps, el));
  for (const Gemms& g : left_chain) HIP_TRY(drv, run_gemms(g, MPS_PREC_C128));
  for (const auto& rl : right_chain) {
    HIP_TRY(drv, run_preps(rl.first, 16));
    HIP_TRY(drv, run_gemms(rl.second, MPS_PREC_C128));
  }
  HIP_TRY(drv, launch_root_copy_list((const CopyItem*)(d + copy_off), (int)cv.size(), copy_max, el, s));
  for (int i = 0; i < count; ++i)
    if (hs[i]->canonical)
      for (const auto& r : hs[i]->ex.roots)
        HIP_TRY(drv, launch_roots(hs[i]->lcur(r.bond), r.lroot, r.rroot, r.d, el, s));
  for (const Gemms& g : env) HIP_TRY(drv, run_gemms(g, prec));
  for (int i = 0; i < count; ++i)
    if (stale[i]) {
      hs[i]->chain_version = hs[i]->version;
      hs[i]->chain_rmin = rmin[i];
    }
  if (drv->timing) drv->tm.env_launches += 2 * (int64_t)env.size();
  std::vector<double> e2(2 * (size_t)count, 0.0);
  std::vector<double2> nn(count, make_double2(1.0, 0.0));
  for (int i = 0; i < count; ++i) {
    mps_state* h = hs[i];
    if ((st = expect_close(h, el, nrm[i], s)) != MPS_OK) return st;
    HIP_TRY(drv, hipMemcpyAsync(e2.data() + 2 * i, h->ex.energy, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    if (nrm[i]) HIP_TRY(drv, hipMemcpyAsync(&nn[i], nrm[i], sizeof(double2), hipMemcpyDeviceToHost, s));
    if (per_term && per_term[i] && h->ex.plan_terms)
      HIP_TRY(drv, hipMemcpyAsync(per_term[i], h->ex.per_term, sizeof(double) * h->ex.plan_terms,
                                  hipMemcpyDeviceToHost, s));
  }
  if ((st = sync(drv)) != MPS_OK) return st;
  for (int i = 0; i < count; ++i) {
    if (!(nn[i].x > 0.0) || !std::isfinite(nn[i].x))
      return fail(MPS_ERR_NONFINITE, "state " + std::to_string(i) + ": norm is zero or not finite");
    if (nrm[i]) hs[i]->norm = std::sqrt(nn[i].x);
    energies[i] = e2[2 * i] + e2[2 * i + 1];
  }
  drv->tm.expect_ms += now_ms() - t0;
  return MPS_OK;
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// ----------------------------------------------------------------------------
// fused single-gate path (one workgroup per gate, ranks kept on the device)

constexpr int kFusedMaxLen = 128;  // 2 D_l and 2 D_r limit of the fused kernel
constexpr int kFusedMaxBatch = 4;  // larger disjoint batches use the batched path

bool fused_eligible(const mps_state* h, int q) {
  return 2 * h->cap[q] <= kFusedMaxLen && 2 * h->cap[q + 2] <= kFusedMaxLen;
}

mps_status fused_begin(mps_state* h) {
  if (h->fused_active) return MPS_OK;
  mps_status st = ensure_ws(h, 1);
  if (st != MPS_OK) return st;
  if ((st = upload(h, h->d_dims, h->dims.data(), sizeof(int) * (h->n + 1))) != MPS_OK) return st;
  HIP_TRY(h, hipMemsetAsync(h->d_fstat, 0, 2 * sizeof(int), h->stream));
  HIP_TRY(h, hipMemsetAsync(h->d_fdisc, 0, sizeof(double), h->stream));
  HIP_TRY(h, hipMemsetAsync(h->d_fsweeps, 0, sizeof(int), h->stream));
  h->fused_active = true;
  return MPS_OK;
}

// Ends a run of fused gates: reads back ranks, status and accumulators.  On a
// failed gate, *failed_at = its chunk-relative index and *code its status
// (the gates before it were applied, it and the later ones were not).
mps_status fused_flush(mps_state* h, int64_t* failed_at, int* code) {
  *failed_at = -1;
  *code = 0;
  if (!h->fused_active) return MPS_OK;
  std::vector<int> dims(h->n + 1);
  int stat[2] = {0, 0}, sweeps = 0;
  double disc = 0.0;
  HIP_TRY(h, hipMemcpyAsync(dims.data(), h->d_dims, sizeof(int) * (h->n + 1), hipMemcpyDeviceToHost,
                            h->stream));
  HIP_TRY(h, hipMemcpyAsync(stat, h->d_fstat, sizeof(stat), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipMemcpyAsync(&disc, h->d_fdisc, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipMemcpyAsync(&sweeps, h->d_fsweeps, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  mps_status st = sync(h);
  if (st != MPS_OK) return st;
  h->fused_active = false;
  for (int b = 0; b <= h->n; ++b)
    if (dims[b] < 1 || dims[b] > h->cap[b]) {
      h->poisoned = true;
      return fail(MPS_ERR_DEVICE, "fused gates: bond dimension out of range");
    }
  h->dims = dims;
  h->discarded += disc;
  h->tm.jacobi_sweeps += sweeps;
  if (stat[0] != 0) {
    *failed_at = stat[1];
    *code = stat[0];
  }
  return MPS_OK;
}

mps_status fused_launch(mps_state* h, int q, const double2* u, int gate) {
  FusedGate g{h->cur(q), h->cur(q + 1), h->lcur(q), h->lcur(q + 1), u, h->d_dims, h->ws_c,
              h->d_fstat, h->d_fdisc, h->d_fsweeps, q, gate, h->cap[q + 1], h->max_sweeps,
              h->cutoff, kEpsScale};
  HIP_TRY(h, launch_gate2q_fused(g, 2 * h->cap[q + 2], h->stream));
  return MPS_OK;
}

}  // namespace

// ============================================================================ C ABI

extern "C" {

const char* mps_last_error(void) { return g_err.c_str(); }

mps_status mps_create(const mps_config* cfg, mps_handle* out) {
  if (!cfg || !out) return fail(MPS_ERR_ARG, "NULL config or output");
  if (cfg->n_qubits < 1 || cfg->n_qubits > 30000) return fail(MPS_ERR_ARG, "n_qubits out of range");
  if (cfg->max_bond < 1 || cfg->max_bond > kMaxBond)
    return fail(MPS_ERR_ARG, "max_bond must be in [1, 512]");
  if (!(cfg->svd_cutoff >= 0.0) || !std::isfinite(cfg->svd_cutoff))
    return fail(MPS_ERR_ARG, "svd_cutoff must be finite and >= 0");
  if (cfg->max_jacobi_sweeps < 0 || cfg->max_jacobi_sweeps > 1000)
    return fail(MPS_ERR_ARG, "max_jacobi_sweeps must be in [0, 1000]");
  if (cfg->init_bits)
    for (int q = 0; q < cfg->n_qubits; ++q)
      if (cfg->init_bits[q] > 1) return fail(MPS_ERR_ARG, "init_bits must be 0 or 1");
  struct Owner {
    mps_state* p;
    ~Owner() {
      if (p) mps_destroy(p);
    }
    mps_state* get() const { return p; }
    mps_state* operator->() const { return p; }
    mps_state* release() {
      mps_state* q = p;
      p = nullptr;
      return q;
    }
  } h{new mps_state()};
  h->n = cfg->n_qubits;
  h->D = cfg->max_bond;
  h->cutoff = cfg->svd_cutoff;
  h->max_sweeps = cfg->max_jacobi_sweeps ? cfg->max_jacobi_sweeps : kDefaultSweeps;
  h->budget = cfg->hbm_budget_bytes;
  if (hipGetDevice(&h->device) != hipSuccess) return fail(MPS_ERR_DEVICE, "hipGetDevice failed");
  if (cfg->stream) {
    h->stream = (hipStream_t)cfg->stream;
  } else {
    HIP_TRY(nullptr, hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
    h->own_stream = true;
  }
  mps_status st = ensure_lds(h.get());
  if (st != MPS_OK) return st;
  const int n = h->n;
  h->dims.assign(n + 1, 1);
  h->cap.resize(n + 1);
  for (int b = 0; b <= n; ++b) h->cap[b] = cap_dim(b, n, h->D);
  for (int i = 0; i < 2; ++i) {
    h->site[i].assign(n, nullptr);
    h->lam[i].assign(n + 1, nullptr);
  }
  h->site_cur.assign(n, 0);
  h->lam_cur.assign(n + 1, 0);
  h->site_cap.resize(n);
  for (int q = 0; q < n; ++q) {
    h->site_cap[q] = 2 * (size_t)h->cap[q] * h->cap[q + 1];
    for (int i = 0; i < 2; ++i)
      if ((st = dalloc_t(h.get(), &h->site[i][q], h->site_cap[q])) != MPS_OK) return st;
  }
  for (int b = 0; b <= n; ++b)
    for (int i = 0; i < 2; ++i)
      if ((st = dalloc_t(h.get(), &h->lam[i][b], h->cap[b])) != MPS_OK) return st;
  if ((st = dalloc_t(h.get(), &h->d_site_ptrs, n)) != MPS_OK) return st;
  if ((st = dalloc_t(h.get(), &h->d_lam_ptrs, n + 1)) != MPS_OK) return st;
  if ((st = dalloc_t(h.get(), &h->d_bits, n)) != MPS_OK) return st;
  if ((st = dalloc_t(h.get(), &h->d_one, 1)) != MPS_OK) return st;
  if ((st = dalloc_t(h.get(), &h->d_dims, n + 1)) != MPS_OK) return st;
  if ((st = dalloc_t(h.get(), &h->d_fstat, 2)) != MPS_OK) return st;
  if ((st = dalloc_t(h.get(), &h->d_fdisc, 1)) != MPS_OK) return st;
  if ((st = dalloc_t(h.get(), &h->d_fsweeps, 1)) != MPS_OK) return st;
  if ((st = dalloc_t(h.get(), &h->d_cap, n + 1)) != MPS_OK) return st;
  HIP_TRY(h.get(), hipMemcpy(h->d_cap, h->cap.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice));
  const double one = 1.0;
  HIP_TRY(h.get(), hipMemcpy(h->d_one, &one, sizeof(double), hipMemcpyHostToDevice));
  if ((st = mps_reset(h.get(), cfg->init_bits)) != MPS_OK) return st;
  *out = h.release();
  return MPS_OK;
}

mps_status mps_destroy(mps_handle h) {
  if (!h) return MPS_OK;
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  if (h->side) (void)hipStreamSynchronize(h->side);
  for (hipStream_t js : h->jside)
    if (js) (void)hipStreamSynchronize(js);
  drop_graph(h->ex);
  for (auto& a : h->allocs) (void)hipFree(a.first);
  for (hipEvent_t e : h->ev_env) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->ev_tune) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->ev_close) (void)hipEventDestroy(e);
  for (hipEvent_t e : h->ev_jac)
    if (e) (void)hipEventDestroy(e);
  if (h->side) (void)hipStreamDestroy(h->side);
  for (hipStream_t js : h->jside)
    if (js) (void)hipStreamDestroy(js);
  for (hipEvent_t ev : h->ev_jjoin)
    if (ev) (void)hipEventDestroy(ev);
  if (h->ev_jfork) (void)hipEventDestroy(h->ev_jfork);
  if (h->ev_fork) (void)hipEventDestroy(h->ev_fork);
  if (h->ev_join) (void)hipEventDestroy(h->ev_join);
  if (h->own_stream && h->stream) (void)hipStreamDestroy(h->stream);
  delete h;
  return MPS_OK;
}

mps_status mps_reset(mps_handle h, const uint8_t* bits) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  const int n = h->n;
  std::vector<uint8_t> b(n, 0);
  if (bits)
    for (int q = 0; q < n; ++q) {
      if (bits[q] > 1) return fail(MPS_ERR_ARG, "bits must be 0 or 1");
      b[q] = bits[q];
    }
  std::fill(h->site_cur.begin(), h->site_cur.end(), 0);
  std::fill(h->lam_cur.begin(), h->lam_cur.end(), 0);
  std::fill(h->dims.begin(), h->dims.end(), 1);
  std::vector<double2*> sp(h->site[0]);
  std::vector<double*> lp(h->lam[0]);
  HIP_TRY(h, hipMemcpyAsync(h->d_site_ptrs, sp.data(), sizeof(double2*) * n, hipMemcpyHostToDevice,
                            h->stream));
  HIP_TRY(h, hipMemcpyAsync(h->d_lam_ptrs, lp.data(), sizeof(double*) * (n + 1),
                            hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, hipMemcpyAsync(h->d_bits, b.data(), n, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, launch_init_product(h->d_site_ptrs, h->d_lam_ptrs, h->d_bits, n, h->stream));
  if ((st = sync(h)) != MPS_OK) return st;
  h->canonical = true;
  ++h->version;
  h->norm = 1.0;
  h->discarded = 0.0;
  return MPS_OK;
}

mps_status mps_apply_gates(mps_handle h, int64_t ng, const int32_t* q0, const int32_t* q1,
                           const double* u, int64_t* n_done) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if (n_done) *n_done = 0;
  if (ng < 0 || (ng > 0 && (!q0 || !q1 || !u))) return fail(MPS_ERR_ARG, "bad gate arrays");
  for (int64_t i = 0; i < ng; ++i) {
    if (q0[i] < 0 || q0[i] >= h->n) return fail(MPS_ERR_ARG, "gate " + std::to_string(i) + ": q0 out of range");
    if (q1[i] >= 0 && (q1[i] != q0[i] + 1 || q1[i] >= h->n))
      return fail(MPS_ERR_ARG, "gate " + std::to_string(i) + ": two-qubit gates must act on (q, q+1)");
    if (!finite_all(u + 32 * i, q1[i] >= 0 ? 32 : 8))
      return fail(MPS_ERR_NONFINITE, "gate " + std::to_string(i) + ": non-finite matrix entry");
  }
  const double t0 = now_ms();
  const int64_t chunk = 1 << 16;
  int64_t done = 0;
  for (int64_t c0 = 0; c0 < ng; c0 += chunk) {
    const int64_t c1 = std::min(ng, c0 + chunk);
    const size_t need = (size_t)(c1 - c0) * 16;
    if (need > h->gates_cap) {
      if ((st = sync(h)) != MPS_OK) return st;
      dfree(h, h->d_gates);
      h->d_gates = nullptr;
      h->gates_cap = 0;
      if ((st = dalloc_t(h, &h->d_gates, need)) != MPS_OK) return st;
      h->gates_cap = need;
    }
    if ((st = sync(h)) != MPS_OK) return st;
    HIP_TRY(h, hipMemcpy(h->d_gates, u + 32 * c0, sizeof(double) * 32 * (c1 - c0),
                         hipMemcpyHostToDevice));
    int64_t i = c0;
    // ends a fused run; on a failed gate reports it and how many were applied
    auto flush = [&]() -> mps_status {
      int64_t bad = -1;
      int code = 0;
      mps_status s2 = fused_flush(h, &bad, &code);
      if (s2 != MPS_OK) return s2;
      if (bad >= 0) {
        done = c0 + bad;
        const std::string where = " (gate " + std::to_string(done) + " on qubit " +
                                  std::to_string(q0[done]) + ")";
        if (code == 2)
          return fail(MPS_ERR_NOCONV, "Jacobi SVD did not converge within " +
                                          std::to_string(h->max_sweeps) + " sweeps" + where);
        return fail(MPS_ERR_NONFINITE, "non-finite or zero singular values" + where);
      }
      return MPS_OK;
    };
    auto finish = [&](mps_status s2) {
      if (n_done) *n_done = done;
      h->tm.gates_ms += now_ms() - t0;
      return s2;
    };
    while (i < c1) {
      const double2* ug = h->d_gates + (size_t)(i - c0) * 16;
      if (q1[i] < 0) {
        const int q = q0[i];
        if (h->fused_active)
          HIP_TRY(h, launch_gate1q_dev(h->cur(q), ug, h->d_dims, h->d_fstat, q,
                                       h->cap[q] * h->cap[q + 1], h->stream));
        else
          HIP_TRY(h, launch_gate1q(h->cur(q), ug, h->dims[q] * h->dims[q + 1], h->stream));
        h->canonical = false;
        ++h->version;
        ++i;
        if (!h->fused_active) done = i;
        continue;
      }
      std::vector<int> qs, gi;
      std::vector<char> used(h->n, 0);
      int64_t j = i;
      bool all_small = true;
      while (j < c1 && q1[j] >= 0 && !used[q0[j]] && !used[q0[j] + 1] && (int)qs.size() < h->n) {
        used[q0[j]] = used[q0[j] + 1] = 1;
        qs.push_back(q0[j]);
        gi.push_back((int)(j - c0));
        all_small = all_small && fused_eligible(h, q0[j]);
        ++j;
      }
      if (h->fused_enabled && all_small && (int)qs.size() <= kFusedMaxBatch) {
        if ((st = fused_begin(h)) != MPS_OK) return finish(st);
        for (size_t b = 0; b < qs.size(); ++b)
          if ((st = fused_launch(h, qs[b], h->d_gates + (size_t)gi[b] * 16, gi[b])) != MPS_OK)
            return finish(st);
        h->canonical = false;
        ++h->version;
        i = j;
        continue;
      }
      if ((st = flush()) != MPS_OK) return finish(st);
      done = i;
      if ((st = apply_2q_batch(h, qs, gi)) != MPS_OK) return finish(st);
      i = j;
      done = i;
    }
    if ((st = flush()) != MPS_OK) return finish(st);
    done = c1;
  }
  if ((st = sync(h)) != MPS_OK) return st;
  if (n_done) *n_done = done;
  h->tm.gates_ms += now_ms() - t0;
  return MPS_OK;
}

// mps_apply_gates_multi for lists with bonds above the fused limit: step k
// applies gate k of every list that has one; its one-qubit gates first, then
// its two-qubit gates -- on distinct handles, hence disjoint -- as one batch
// of the multi-workgroup path (one batched contraction, Jacobi SVD and site
// update), driven by the first handle on its stream.  A failed gate stops
// only its own list.  Arguments were validated by the caller.
mps_status apply_gates_multi_batched(int32_t n_handles, const mps_handle* hs, const int64_t* n_gates,
                                     const int32_t* const* q0, const int32_t* const* q1,
                                     const double* const* u, int64_t* n_done) {
  const double t0 = now_ms();
  mps_state* drv = hs[0];
  mps_status st;
  int64_t steps = 0;
  for (int i = 0; i < n_handles; ++i) {
    mps_state* h = hs[i];
    const int64_t ng = n_gates[i];
    steps = std::max(steps, ng);
    if ((st = sync(h)) != MPS_OK) return st;
    const size_t need = (size_t)std::max<int64_t>(ng, 1) * 16;
    if (need > h->gates_cap) {
      dfree(h, h->d_gates);
      h->d_gates = nullptr;
      h->gates_cap = 0;
      if ((st = dalloc_t(h, &h->d_gates, need)) != MPS_OK) return st;
      h->gates_cap = need;
    }
    if (ng > 0) HIP_TRY(h, hipMemcpy(h->d_gates, u[i], sizeof(double) * 32 * ng, hipMemcpyHostToDevice));
  }
  std::vector<char> alive(n_handles, 1);
  std::vector<int64_t> done(n_handles, 0);
  mps_status first = MPS_OK;
  int first_handle = n_handles;
  std::string first_msg;
  std::vector<GateRef> refs;
  std::vector<int> owner;
  std::vector<mps_status> err;
  std::vector<std::string> msg;
  for (int64_t k = 0; k < steps; ++k) {
    refs.clear();
    owner.clear();
    for (int i = 0; i < n_handles; ++i) {
      if (!alive[i] || k >= n_gates[i]) continue;
      mps_state* h = hs[i];
      const int q = q0[i][k];
      const double2* ug = h->d_gates + (size_t)k * 16;
      if (q1[i][k] < 0) {
        HIP_TRY(drv, launch_gate1q(h->cur(q), ug, h->dims[q] * h->dims[q + 1], drv->stream));
        h->canonical = false;
        ++h->version;
        done[i] = k + 1;
      } else {
        refs.push_back(GateRef{h, q, ug});
        owner.push_back(i);
      }
    }
    if (refs.empty()) continue;
    if ((st = apply_2q_refs(drv, refs, false, err, msg)) != MPS_OK) return st;
    for (size_t b = 0; b < refs.size(); ++b) {
      const int i = owner[b];
      if (err[b] == MPS_OK) {
        done[i] = k + 1;
        continue;
      }
      alive[i] = 0;
      if (i < first_handle) {
        first_handle = i;
        first = err[b];
        first_msg = msg[b] + " (handle " + std::to_string(i) + ", gate " + std::to_string(k) + ")";
      }
    }
  }
  if ((st = sync(drv)) != MPS_OK) return st;
  const double dt = now_ms() - t0;
  for (int i = 0; i < n_handles; ++i) {
    if (n_done) n_done[i] = done[i];
    hs[i]->tm.gates_ms += dt;
  }
  if (first != MPS_OK) return fail(first, first_msg);
  return MPS_OK;
}

mps_status mps_apply_gates_multi(int32_t n_handles, const mps_handle* hs, const int64_t* n_gates,
                                 const int32_t* const* q0, const int32_t* const* q1,
                                 const double* const* u, void* stream, int64_t* n_done) {
  if (n_handles < 0) return fail(MPS_ERR_ARG, "n_handles < 0");
  if (n_handles == 0) return MPS_OK;
  if (!hs || !n_gates || !q0 || !q1 || !u) return fail(MPS_ERR_ARG, "NULL array");
  if (n_handles > 65535) return fail(MPS_ERR_ARG, "at most 65535 handles per call");
  bool fused_mode = true;  // every two-qubit gate within the fused limit
  for (int i = 0; i < n_handles; ++i) {
    if (n_done) n_done[i] = 0;
    mps_status st = check_handle(hs[i]);
    if (st != MPS_OK) return st;
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(MPS_ERR_ARG, "handles must be distinct");
    mps_state* h = hs[i];
    const int64_t ng = n_gates[i];
    if (ng < 0 || (ng > 0 && (!q0[i] || !q1[i] || !u[i])))
      return fail(MPS_ERR_ARG, "handle " + std::to_string(i) + ": bad gate arrays");
    for (int64_t g = 0; g < ng; ++g) {
      const int32_t a = q0[i][g], b = q1[i][g];
      const std::string where = "handle " + std::to_string(i) + ", gate " + std::to_string(g);
      if (a < 0 || a >= h->n) return fail(MPS_ERR_ARG, where + ": q0 out of range");
      if (b >= 0 && (b != a + 1 || b >= h->n))
        return fail(MPS_ERR_ARG, where + ": two-qubit gates must act on (q, q+1)");
      if (b >= 0 && !fused_eligible(h, a)) fused_mode = false;
      if (!finite_all(u[i] + 32 * g, b >= 0 ? 32 : 8))
        return fail(MPS_ERR_NONFINITE, where + ": non-finite matrix entry");
    }
  }
  const double t0 = now_ms();
  if (!fused_mode) return apply_gates_multi_batched(n_handles, hs, n_gates, q0, q1, u, n_done);
  hipStream_t s = stream ? (hipStream_t)stream : hs[0]->stream;
  std::vector<FusedRun> runs(n_handles);
  int64_t steps = 0;
  for (int i = 0; i < n_handles; ++i) {
    mps_state* h = hs[i];
    const int64_t ng = n_gates[i];
    steps = std::max(steps, ng);
    mps_status st = ensure_ws(h, 1);
    if (st != MPS_OK) return st;
    if ((st = sync(h)) != MPS_OK) return st;
    const size_t need = (size_t)std::max<int64_t>(ng, 1);
    if (need * 16 > h->gates_cap) {
      dfree(h, h->d_gates);
      h->d_gates = nullptr;
      h->gates_cap = 0;
      if ((st = dalloc_t(h, &h->d_gates, need * 16)) != MPS_OK) return st;
      h->gates_cap = need * 16;
    }
    if (need * 2 > h->gq_cap) {
      dfree(h, h->d_gq);
      h->d_gq = nullptr;
      h->gq_cap = 0;
      if ((st = dalloc_t(h, &h->d_gq, need * 2)) != MPS_OK) return st;
      h->gq_cap = need * 2;
    }
    if (ng > 0) {
      HIP_TRY(h, hipMemcpy(h->d_gates, u[i], sizeof(double) * 32 * ng, hipMemcpyHostToDevice));
      HIP_TRY(h, hipMemcpy(h->d_gq, q0[i], sizeof(int32_t) * ng, hipMemcpyHostToDevice));
      HIP_TRY(h, hipMemcpy(h->d_gq + ng, q1[i], sizeof(int32_t) * ng, hipMemcpyHostToDevice));
    }
    std::vector<double2*> sp(h->n);
    std::vector<double*> lp(h->n + 1);
    for (int q = 0; q < h->n; ++q) sp[q] = h->cur(q);
    for (int b = 0; b <= h->n; ++b) lp[b] = h->lcur(b);
    HIP_TRY(h, hipMemcpy(h->d_site_ptrs, sp.data(), sizeof(double2*) * h->n, hipMemcpyHostToDevice));
    HIP_TRY(h, hipMemcpy(h->d_lam_ptrs, lp.data(), sizeof(double*) * (h->n + 1), hipMemcpyHostToDevice));
    if ((st = fused_begin(h)) != MPS_OK) return st;
    if ((st = sync(h)) != MPS_OK) return st;
    runs[i] = FusedRun{h->d_site_ptrs, h->d_lam_ptrs, h->d_cap, h->d_dims, h->ws_c, h->d_fstat,
                       h->d_fdisc, h->d_fsweeps, h->d_gq, h->d_gq + ng, (const double2*)h->d_gates,
                       0, ng, h->max_sweeps, h->cutoff, kEpsScale};
  }
  mps_state* h0 = hs[0];
  mps_status st = ensure_desc(h0, sizeof(FusedRun) * n_handles);
  if (st != MPS_OK) return st;
  HIP_TRY(h0, hipMemcpy(h0->d_desc, runs.data(), sizeof(FusedRun) * n_handles, hipMemcpyHostToDevice));
  for (int64_t k = 0; k < steps; ++k)
    HIP_TRY(h0, launch_fused_step((const FusedRun*)h0->d_desc, n_handles, k, s));
  HIP_TRY(h0, hipStreamSynchronize(s));
  const double dt = now_ms() - t0;
  mps_status first = MPS_OK;
  std::string first_msg;
  for (int i = 0; i < n_handles; ++i) {
    mps_state* h = hs[i];
    int64_t bad = -1;
    int code = 0;
    if ((st = fused_flush(h, &bad, &code)) != MPS_OK) return st;
    const int64_t done = bad >= 0 ? bad : n_gates[i];
    if (n_done) n_done[i] = done;
    if (done > 0) {
      h->canonical = false;
      ++h->version;
    }
    h->tm.gates_ms += dt;
    if (bad >= 0 && first == MPS_OK) {
      first = code == 2 ? MPS_ERR_NOCONV : MPS_ERR_NONFINITE;
      first_msg = std::string(code == 2 ? "Jacobi SVD did not converge within " +
                                              std::to_string(h->max_sweeps) + " sweeps"
                                        : "non-finite or zero singular values") +
                  " (handle " + std::to_string(i) + ", gate " + std::to_string(bad) + ")";
    }
  }
  if (first != MPS_OK) return fail(first, first_msg);
  return MPS_OK;
}

mps_status mps_apply_gate(mps_handle h, int32_t q0, int32_t q1, const double* u) {
  if (!u) return fail(MPS_ERR_ARG, "NULL gate matrix");
  double buf[32] = {0};
  std::memcpy(buf, u, sizeof(double) * (q1 >= 0 ? 32 : 8));
  return mps_apply_gates(h, 1, &q0, &q1, buf, nullptr);
}

mps_status mps_canonicalize(mps_handle h) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  return canonicalize_impl(h);
}

mps_status mps_norm(mps_handle h, double* norm) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if (!norm) return fail(MPS_ERR_ARG, "NULL output");
  *norm = h->norm;
  return MPS_OK;
}

mps_status mps_discarded_weight(mps_handle h, double* w) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if (!w) return fail(MPS_ERR_ARG, "NULL output");
  *w = h->discarded;
  return MPS_OK;
}

mps_status mps_bond_dims(mps_handle h, int32_t* dims) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if (!dims) return fail(MPS_ERR_ARG, "NULL output");
  for (int b = 0; b <= h->n; ++b) dims[b] = h->dims[b];
  return MPS_OK;
}

mps_status mps_pauli_sum_create(int32_t n_qubits, int64_t n_terms, const uint8_t* codes,
                                const double* coeffs, mps_pauli_sum* out) {
  if (!out) return fail(MPS_ERR_ARG, "NULL output");
  std::unique_ptr<mps_psum> p(new mps_psum());
  std::string err;
  if (!build_pauli_plan(n_qubits, n_terms, codes, coeffs, p->plan, err))
    return fail(MPS_ERR_ARG, err);
  p->serial = g_plan_serial.fetch_add(1);
  *out = p.release();
  return MPS_OK;
}

mps_status mps_pauli_sum_destroy(mps_pauli_sum p) {
  delete p;
  return MPS_OK;
}

mps_status mps_pauli_sum_stats(mps_pauli_sum p, int64_t* nl, int64_t* nr, int64_t* nc,
                               int32_t* meet) {
  if (!p) return fail(MPS_ERR_ARG, "NULL plan");
  if (nl) *nl = (int64_t)p->plan.left.size();
  if (nr) *nr = (int64_t)p->plan.right.size();
  if (nc) *nc = p->plan.n_terms;
  if (meet) *meet = p->plan.meet;
  return MPS_OK;
}

mps_status mps_pauli_sum_export(mps_pauli_sum p, int32_t* lp, int32_t* ls, int32_t* ll,
                                int32_t* rp, int32_t* rs, int32_t* rl, int32_t* cb, int32_t* cl,
                                int32_t* cr) {
  if (!p) return fail(MPS_ERR_ARG, "NULL plan");
  const PauliPlan& P = p->plan;
  for (size_t i = 0; i < P.left.size(); ++i) {
    if (lp) lp[i] = P.left[i].parent;
    if (ls) ls[i] = P.left[i].site;
    if (ll) ll[i] = P.left[i].letter;
  }
  for (size_t i = 0; i < P.right.size(); ++i) {
    if (rp) rp[i] = P.right[i].parent;
    if (rs) rs[i] = P.right[i].site;
    if (rl) rl[i] = P.right[i].letter;
  }
  for (int64_t k = 0; k < P.n_terms; ++k) {
    if (cb) cb[k] = P.close_bond[k];
    if (cl) cl[k] = P.close_left[k];
    if (cr) cr[k] = P.close_right[k];
  }
  return MPS_OK;
}

mps_status mps_expect_pauli_sum(mps_handle h, mps_pauli_sum p, mps_precision prec, double* energy,
                                double* per_term) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if (!p || !energy) return fail(MPS_ERR_ARG, "NULL plan or output");
  if (p->plan.n_qubits != h->n) return fail(MPS_ERR_ARG, "plan and MPS qubit counts differ");
  if (prec != MPS_PREC_C128 && prec != MPS_PREC_C64 && prec != MPS_PREC_SPLIT_BF16 &&
      prec != MPS_PREC_SPLIT_F16)
    return fail(MPS_ERR_ARG, "unknown precision");
  return expect_impl(h, p, (int)prec, energy, per_term);
}

mps_status mps_expect_pauli_sum_multi(int32_t count, const mps_handle* states, const mps_pauli_sum* plans,
                                      mps_precision prec, double* energies, double* const* per_term) {
  if (count < 0) return fail(MPS_ERR_ARG, "count < 0");
  if (count == 0) return MPS_OK;
  if (!states || !plans || !energies) return fail(MPS_ERR_ARG, "NULL array");
  if (prec != MPS_PREC_C128 && prec != MPS_PREC_C64 && prec != MPS_PREC_SPLIT_BF16 &&
      prec != MPS_PREC_SPLIT_F16)
    return fail(MPS_ERR_ARG, "unknown precision");
  int64_t sites = 0;
  for (int32_t i = 0; i < count; ++i) {
    mps_status st = check_handle(states[i]);
    if (st != MPS_OK) return st;
    for (int32_t j = 0; j < i; ++j)
      if (states[j] == states[i]) return fail(MPS_ERR_ARG, "states must be distinct");
    sites += states[i]->n + 1;
    if (!plans[i]) return fail(MPS_ERR_ARG, "NULL plan");
    if (plans[i]->plan.n_qubits != states[i]->n)
      return fail(MPS_ERR_ARG, "state " + std::to_string(i) + ": plan and MPS qubit counts differ");
  }
  // one launch row per site (and two per bond for the roots)
  if (2 * sites > 65535) return fail(MPS_ERR_ARG, "at most 32767 sites (qubits + 1 per state) per call");
  return expect_multi_impl(states, plans, count, (int)prec, energies, per_term);
}

mps_status mps_expect_pauli_rows(mps_handle h, mps_pauli_sum p, mps_precision prec, int64_t n_rows,
                                 const int64_t* row_ptr, const int64_t* cols, const double* vals,
                                 double* out) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if (!p) return fail(MPS_ERR_ARG, "NULL plan");
  if (p->plan.n_qubits != h->n) return fail(MPS_ERR_ARG, "plan and MPS qubit counts differ");
  if (prec != MPS_PREC_C128 && prec != MPS_PREC_C64 && prec != MPS_PREC_SPLIT_BF16 &&
      prec != MPS_PREC_SPLIT_F16)
    return fail(MPS_ERR_ARG, "unknown precision");
  if (n_rows < 0 || (n_rows > 0 && (!row_ptr || !out))) return fail(MPS_ERR_ARG, "bad row arrays");
  const int64_t T = p->plan.n_terms;
  int64_t nnz = 0;
  if (n_rows > 0) {
    if (row_ptr[0] != 0) return fail(MPS_ERR_ARG, "row_ptr[0] must be 0");
    for (int64_t r = 0; r < n_rows; ++r)
      if (row_ptr[r + 1] < row_ptr[r]) return fail(MPS_ERR_ARG, "row_ptr must be non-decreasing");
    nnz = row_ptr[n_rows];
    if (nnz > 0 && (!cols || !vals)) return fail(MPS_ERR_ARG, "NULL cols or vals");
    for (int64_t i = 0; i < nnz; ++i)
      if (cols[i] < 0 || cols[i] >= T) return fail(MPS_ERR_ARG, "column index out of range");
  }
  RowsSpec rs{n_rows, nnz, row_ptr, cols, vals, out};
  double energy = 0.0;
  return expect_impl(h, p, (int)prec, &energy, nullptr, &rs);
}

mps_status mps_expect_pauli_sums(mps_handle h, int32_t n_plans, const mps_pauli_sum* plans,
                                 mps_precision prec, double* energy, double* per_term) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if (n_plans < 1 || !plans || !energy) return fail(MPS_ERR_ARG, "need n_plans >= 1, plans and energy");
  for (int32_t i = 0; i < n_plans; ++i) {
    if (!plans[i]) return fail(MPS_ERR_ARG, "NULL plan");
    if (plans[i]->plan.n_qubits != h->n) return fail(MPS_ERR_ARG, "plan and MPS qubit counts differ");
  }
  if (prec != MPS_PREC_C128 && prec != MPS_PREC_C64 && prec != MPS_PREC_SPLIT_BF16 &&
      prec != MPS_PREC_SPLIT_F16)
    return fail(MPS_ERR_ARG, "unknown precision");
  const size_t need = 2 * (size_t)n_plans + 2;
  if (need > h->pairs_cap || !h->d_pairs) {
    if ((st = sync(h)) != MPS_OK) return st;
    dfree(h, h->d_pairs);
    h->d_pairs = nullptr;
    h->pairs_cap = 0;
    if ((st = dalloc_t(h, &h->d_pairs, need)) != MPS_OK) return st;
    h->pairs_cap = need;
  }
  size_t off = 0;
  for (int32_t i = 0; i < n_plans; ++i) {
    double e = 0.0;
    if ((st = expect_impl(h, plans[i], (int)prec, &e, per_term ? per_term + off : nullptr, nullptr,
                          h->d_pairs + 2 * (size_t)i)) != MPS_OK)
      return st;
    off += (size_t)plans[i]->plan.n_terms;
  }
  double* out = h->d_pairs + 2 * (size_t)n_plans;
  HIP_TRY(h, launch_pair_sum(h->d_pairs, n_plans, out, h->stream));
  double E2[2] = {0.0, 0.0};
  HIP_TRY(h, hipMemcpyAsync(E2, out, 2 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if ((st = sync(h)) != MPS_OK) return st;
  *energy = E2[0] + E2[1];
  return MPS_OK;
}

mps_status mps_to_statevector(mps_handle h, double* psi) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if (!psi) return fail(MPS_ERR_ARG, "NULL output");
  if (h->n > kMaxStatevectorQubits)
    return fail(MPS_ERR_ARG, "statevector limited to " + std::to_string(kMaxStatevectorQubits) + " qubits");
  // Every partial contraction holds 2^q D_q <= 2^N amplitudes (D_q <= 2^(N-q)).
  const size_t amps = (size_t)1 << h->n;
  if ((st = sync(h)) != MPS_OK) return st;
  double2* buf[2] = {nullptr, nullptr};
  struct Free {
    mps_state* h;
    double2** b;
    ~Free() {
      (void)hipStreamSynchronize(h->stream);
      dfree(h, b[0]);
      dfree(h, b[1]);
    }
  } release{h, buf};
  if ((st = dalloc_t(h, &buf[0], amps)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &buf[1], amps)) != MPS_OK) return st;
  const double2 one = make_double2(1.0, 0.0);
  HIP_TRY(h, hipMemcpyAsync(buf[0], &one, sizeof(double2), hipMemcpyHostToDevice, h->stream));
  int cur = 0;
  int64_t rows = 1;
  for (int q = 0; q < h->n; ++q) {
    const int dl = h->dims[q], dr = h->dims[q + 1];
    if (rows * 2 * dr > (int64_t)amps) return fail(MPS_ERR_STATE, "internal: bond dimension above 2^(N-q)");
    HIP_TRY(h, launch_sv_site(buf[cur], h->cur(q), buf[1 - cur], rows, dl, dr, h->stream));
    cur = 1 - cur;
    rows *= 2;
  }
  HIP_TRY(h, hipMemcpyAsync(psi, buf[cur], sizeof(double2) * amps, hipMemcpyDeviceToHost, h->stream));
  return sync(h);
}

mps_status mps_export(mps_handle h, int32_t q, int32_t* dl, int32_t* dr, double* b,
                      double* lambda_left) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if (q < 0 || q >= h->n || !dl || !dr) return fail(MPS_ERR_ARG, "bad site or NULL outputs");
  if ((st = sync(h)) != MPS_OK) return st;
  const int a = h->dims[q], c = h->dims[q + 1];
  if (b) HIP_TRY(h, hipMemcpy(b, h->cur(q), sizeof(double2) * 2 * a * c, hipMemcpyDeviceToHost));
  if (lambda_left) HIP_TRY(h, hipMemcpy(lambda_left, h->lcur(q), sizeof(double) * a, hipMemcpyDeviceToHost));
  *dl = a;
  *dr = c;
  return MPS_OK;
}

mps_status mps_import(mps_handle h, int32_t q, int32_t dl, int32_t dr, const double* b,
                      const double* lambda_left) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if (q < 0 || q >= h->n || !b || !lambda_left) return fail(MPS_ERR_ARG, "bad site or NULL inputs");
  if (dl < 1 || dr < 1 || dl > h->cap[q] || dr > h->cap[q + 1])
    return fail(MPS_ERR_ARG, "site dimensions exceed the bond capacity");
  if ((q == 0 && dl != 1) || (q == h->n - 1 && dr != 1))
    return fail(MPS_ERR_ARG, "boundary bonds must have dimension 1");
  if (!finite_all(b, 4 * (size_t)dl * dr) || !finite_all(lambda_left, dl))
    return fail(MPS_ERR_NONFINITE, "non-finite import");
  if ((st = sync(h)) != MPS_OK) return st;
  HIP_TRY(h, hipMemcpy(h->cur(q), b, sizeof(double2) * 2 * dl * dr, hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(h->lcur(q), lambda_left, sizeof(double) * dl, hipMemcpyHostToDevice));
  h->dims[q] = dl;
  h->dims[q + 1] = dr;
  h->canonical = true;
  ++h->version;
  return MPS_OK;
}

mps_status mps_jacobi_svd(int32_t n_vec, int32_t vec_len, const double* vectors, double* sigma,
                          double* out_vectors, int32_t* sweeps) {
  if (n_vec < 1 || n_vec > 1024 || vec_len < 1 || vec_len > 4096 || !vectors || !sigma)
    return fail(MPS_ERR_ARG, "need 1 <= n_vec <= 1024, 1 <= vec_len <= 4096 and non-NULL arrays");
  if (!finite_all(vectors, 2 * (size_t)n_vec * vec_len))
    return fail(MPS_ERR_NONFINITE, "non-finite input");
  mps_state tmp;
  tmp.n = 1;
  HIP_TRY(nullptr, hipStreamCreateWithFlags(&tmp.stream, hipStreamNonBlocking));
  tmp.own_stream = true;
  struct Guard {
    mps_state* s;
    ~Guard() {
      if (s->stream) (void)hipStreamSynchronize(s->stream);
      for (auto& a : s->allocs) (void)hipFree(a.first);
      if (s->stream) (void)hipStreamDestroy(s->stream);
      s->allocs.clear();
      s->stream = nullptr;
    }
  } guard{&tmp};
  mps_state* h = &tmp;
  mps_status st = ensure_lds(h);
  if (st != MPS_OK) return st;
  const size_t cnt = (size_t)n_vec * vec_len;
  double2 *w = nullptr, *out = nullptr;
  double *fro2 = nullptr, *lam = nullptr, *scale = nullptr, *disc = nullptr;
  int *rot = nullptr, *sw = nullptr, *k = nullptr, *status = nullptr;
  // FIN_GATE writes vec_out as [s][a][r] with m split in halves; with an odd
  // length use FIN_LEFT-free path: pad the length to even.
  const int m = vec_len + (vec_len & 1);
  if ((st = dalloc_t(h, &w, (size_t)n_vec * m)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &out, (size_t)n_vec * m)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &fro2, 1)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &lam, n_vec)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &scale, 1)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &disc, 1)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &rot, kDefaultSweeps * 2)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &sw, 1)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &k, 1)) != MPS_OK) return st;
  if ((st = dalloc_t(h, &status, 1)) != MPS_OK) return st;
  h->max_sweeps = kDefaultSweeps * 2;
  std::vector<double2> padded((size_t)n_vec * m, make_double2(0.0, 0.0));
  for (int v = 0; v < n_vec; ++v)
    for (int e = 0; e < vec_len; ++e)
      padded[(size_t)v * m + e] = make_double2(vectors[2 * ((size_t)v * vec_len + e)],
                                               vectors[2 * ((size_t)v * vec_len + e) + 1]);
  HIP_TRY(h, hipMemcpy(w, padded.data(), sizeof(double2) * padded.size(), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemset(fro2, 0, sizeof(double)));
  HIP_TRY(h, hipMemset(rot, 0, sizeof(int) * h->max_sweeps));
  HIP_TRY(h, launch_fro2(w, n_vec * m, fro2, h->stream));
  std::vector<int> swp;
  std::vector<JacItem> jc{JacItem{w, fro2, rot, sw, n_vec, m, 0, 0, 1}};
  if ((st = run_jacobi(h, jc, 0, swp)) != MPS_OK) return st;
  if (swp[0] < 0) return fail(MPS_ERR_NOCONV, "Jacobi SVD did not converge");
  FinItem fi{w, out, lam, k, scale, disc, status, n_vec, m, n_vec, 0.0, FIN_GATE};
  if ((st = ensure_desc(h, 4096)) != MPS_OK) return st;
  if ((st = upload(h, h->d_desc, &fi, sizeof(fi))) != MPS_OK) return st;
  HIP_TRY(h, launch_finalize((const FinItem*)h->d_desc, 1, h->stream));
  if ((st = sync(h)) != MPS_OK) return st;
  int kk = 0, stt = 0;
  double sc = 0.0;
  HIP_TRY(h, hipMemcpy(&kk, k, sizeof(int), hipMemcpyDeviceToHost));
  HIP_TRY(h, hipMemcpy(&stt, status, sizeof(int), hipMemcpyDeviceToHost));
  HIP_TRY(h, hipMemcpy(&sc, scale, sizeof(double), hipMemcpyDeviceToHost));
  // sigma: lam holds sigma / ||sigma|| for the kept (= all, cutoff 0) values
  std::vector<double> lv(n_vec, 0.0);
  HIP_TRY(h, hipMemcpy(lv.data(), lam, sizeof(double) * kk, hipMemcpyDeviceToHost));
  for (int a = 0; a < n_vec; ++a) sigma[a] = (a < kk && sc > 0.0) ? lv[a] / sc : 0.0;
  if (out_vectors) {
    std::vector<double2> o((size_t)kk * m);
    HIP_TRY(h, hipMemcpy(o.data(), out, sizeof(double2) * o.size(), hipMemcpyDeviceToHost));
    const int half = m / 2;
    std::memset(out_vectors, 0, sizeof(double) * 2 * cnt);
    for (int a = 0; a < kk; ++a)
      for (int e = 0; e < vec_len; ++e) {
        const int s = e / half, r = e - s * half;
        const double2 x = o[((size_t)s * kk + a) * half + r];
        out_vectors[2 * ((size_t)a * vec_len + e)] = x.x;
        out_vectors[2 * ((size_t)a * vec_len + e) + 1] = x.y;
      }
  }
  if (sweeps) *sweeps = swp[0];
  return MPS_OK;
}

mps_status mps_jacobi_svd_noalloc(int32_t n_vec, int32_t vec_len, const double* vectors, double* sigma,
                                  double* out_vectors, int32_t* sweeps, void* stream) {
  if (n_vec < 1 || n_vec > kScratchMaxVec || vec_len < 1 || vec_len > kScratchMaxVec || !vectors || !sigma)
    return fail(MPS_ERR_ARG, "need 1 <= n_vec <= " + std::to_string(kScratchMaxVec) + ", 1 <= vec_len <= " +
                                 std::to_string(kScratchMaxVec) + " and non-NULL arrays");
  if (!finite_all(vectors, 2 * (size_t)n_vec * vec_len))
    return fail(MPS_ERR_NONFINITE, "non-finite input");
  void* base = nullptr;
  HIP_TRY(nullptr, scratch_address(&base));
  mps_state tmp;  // host-side bookkeeping only: no device allocation below
  tmp.n = 1;
  tmp.stream = (hipStream_t)stream;
  tmp.own_stream = false;
  tmp.max_sweeps = kDefaultSweeps * 2;
  mps_state* h = &tmp;
  mps_status st = ensure_lds(h);
  if (st != MPS_OK) return st;
  // scratch layout: the work matrix, the output vectors, descriptors, then
  // small values (all offsets multiples of 256 bytes)
  char* p = (char*)base;
  const int m = vec_len + (vec_len & 1);  // even length: finalize splits rows in halves
  double2* w = (double2*)p;
  double2* out = (double2*)(p + kScratchMatBytes);
  h->d_desc = p + 2 * kScratchMatBytes;
  h->desc_bytes = kScratchDescBytes;
  char* misc = p + 2 * kScratchMatBytes + kScratchDescBytes;
  double* fro2 = (double*)misc;
  double* scale = (double*)(misc + 256);
  double* disc = (double*)(misc + 512);
  int* k = (int*)(misc + 768);
  int* status = (int*)(misc + 1024);
  int* sw = (int*)(misc + 1280);
  int* rot = (int*)(misc + 1536);  // max_sweeps counters
  double* lam = (double*)(misc + 2048);
  static_assert(2048 + sizeof(double) * kScratchMaxVec <= kScratchMiscBytes, "misc scratch too small");
  static_assert(1536 + sizeof(int) * kDefaultSweeps * 2 <= 2048, "rotation counters overlap sigma");
  // the previous call's contents stay: clear what accumulates or is padded
  HIP_TRY(h, launch_zero(w, sizeof(double2) * (size_t)n_vec * m, h->stream));
  HIP_TRY(h, launch_zero(misc, 2048, h->stream));
  HIP_TRY(h, hipMemcpy2DAsync(w, sizeof(double2) * m, vectors, sizeof(double2) * vec_len,
                              sizeof(double2) * vec_len, n_vec, hipMemcpyHostToDevice, h->stream));
  HIP_TRY(h, launch_fro2(w, n_vec * m, fro2, h->stream));
  std::vector<int> swp;
  std::vector<JacItem> jc{JacItem{w, fro2, rot, sw, n_vec, m, 0, 0, 1}};
  if ((st = run_jacobi(h, jc, 0, swp)) != MPS_OK) return st;
  if (swp[0] < 0) return fail(MPS_ERR_NOCONV, "Jacobi SVD did not converge");
  FinItem fi{w, out, lam, k, scale, disc, status, n_vec, m, n_vec, 0.0, FIN_GATE};
  if ((st = upload(h, h->d_desc, &fi, sizeof(fi))) != MPS_OK) return st;
  HIP_TRY(h, launch_finalize((const FinItem*)h->d_desc, 1, h->stream));
  int kk = 0, stt = 0;
  double sc = 0.0;
  HIP_TRY(h, hipMemcpyAsync(&kk, k, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipMemcpyAsync(&stt, status, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(h, hipMemcpyAsync(&sc, scale, sizeof(double), hipMemcpyDeviceToHost, h->stream));
  if ((st = sync(h)) != MPS_OK) return st;
  if (kk < 0 || kk > n_vec) return fail(MPS_ERR_STATE, "internal: kept rank out of range");
  // sigma: lam holds sigma / ||sigma|| for the kept (= all nonzero) values
  HIP_TRY(h, hipMemcpyAsync(sigma, lam, sizeof(double) * kk, hipMemcpyDeviceToHost, h->stream));
  if (out_vectors) {
    // finalize writes the vectors as [s][a][r], each row split at m / 2
    const int half = m / 2;
    for (int s2 = 0; s2 < 2; ++s2) {
      const int width = s2 == 0 ? std::min(half, vec_len) : vec_len - half;
      if (width <= 0 || kk == 0) continue;
      HIP_TRY(h, hipMemcpy2DAsync(out_vectors + 2 * (size_t)s2 * half, sizeof(double2) * vec_len,
                                  out + (size_t)s2 * kk * half, sizeof(double2) * half,
                                  sizeof(double2) * width, kk, hipMemcpyDeviceToHost, h->stream));
    }
  }
  if ((st = sync(h)) != MPS_OK) return st;
  for (int a = 0; a < n_vec; ++a) sigma[a] = (a < kk && sc > 0.0) ? sigma[a] / sc : 0.0;
  if (out_vectors && kk < n_vec)
    std::memset(out_vectors + 2 * (size_t)kk * vec_len, 0, sizeof(double) * 2 * (size_t)(n_vec - kk) * vec_len);
  if (sweeps) *sweeps = swp[0];
  return MPS_OK;
}

mps_status mps_set_jacobi_groups(mps_handle h, int32_t groups) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if (groups < 1 || groups > kMaxJacobiGroups)
    return fail(MPS_ERR_ARG, "jacobi groups must be 1.." + std::to_string(kMaxJacobiGroups));
  h->jacobi_groups = groups;
  return MPS_OK;
}

mps_status mps_set_fused_gates(mps_handle h, int32_t enabled) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  h->fused_enabled = enabled != 0;
  return MPS_OK;
}

mps_status mps_copy(mps_handle dst, mps_handle src) {
  mps_status st = check_handle(dst);
  if (st != MPS_OK) return st;
  if ((st = check_handle(src)) != MPS_OK) return st;
  if (dst == src) return MPS_OK;
  if (dst->n != src->n || dst->cap != src->cap)
    return fail(MPS_ERR_ARG, "mps_copy needs equal qubit counts and bond capacities");
  if ((st = sync(src)) != MPS_OK) return st;  // src's last gates have landed
  const int n = src->n;
  for (int q = 0; q < n; ++q)
    HIP_TRY(dst, hipMemcpyAsync(dst->cur(q), src->cur(q),
                                sizeof(double2) * 2 * (size_t)src->dims[q] * src->dims[q + 1],
                                hipMemcpyDeviceToDevice, dst->stream));
  for (int b = 0; b <= n; ++b)
    HIP_TRY(dst, hipMemcpyAsync(dst->lcur(b), src->lcur(b), sizeof(double) * (size_t)src->dims[b],
                                hipMemcpyDeviceToDevice, dst->stream));
  // complete before returning: src's next gates may overwrite its buffers in place
  if ((st = sync(dst)) != MPS_OK) return st;
  dst->dims = src->dims;
  dst->canonical = src->canonical;
  ++dst->version;
  dst->norm = src->norm;
  dst->discarded = src->discarded;
  return MPS_OK;
}

mps_status mps_set_autotune(mps_handle h, int32_t enabled) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  h->autotune = enabled != 0;
  return MPS_OK;
}

mps_status mps_set_graphs(mps_handle h, int32_t enabled) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if ((st = sync(h)) != MPS_OK) return st;
  h->graphs = enabled != 0;
  if (!h->graphs) drop_graph(h->ex);
  return MPS_OK;
}

mps_status mps_set_env_tile(mps_handle h, int32_t tile) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if (tile < -1 || tile >= kEnvTiles) return fail(MPS_ERR_ARG, "tile index out of range");
  if ((st = sync(h)) != MPS_OK) return st;
  if (tile != h->forced_tile) drop_graph(h->ex);  // captured with the old tiles
  h->forced_tile = tile;
  return MPS_OK;
}

mps_status mps_autotune_table(char* buf, int64_t cap, int64_t* len) {
  static const char* prec_name[] = {"c128", "c64", "split_bf16", "split_f16"};
  std::string out;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    for (const auto& kv : g_tune) {
      const TuneKey& k = kv.first;
      const TuneEntry& e = kv.second;
      const int* sh = kEnvTileShape[e.tile];
      out += std::to_string(k.dev) + " " + (k.prec >= 0 && k.prec < 4 ? prec_name[k.prec] : "?") + " " +
             std::to_string(k.half) + " " + std::to_string(k.dl) + " " + std::to_string(k.dr) + " " +
             std::to_string(k.bucket) + " " + std::to_string(e.tile) + " " + std::to_string(sh[0]) + "x" +
             std::to_string(sh[1]) + "x" + std::to_string(sh[2]);
      for (int t = 0; t < kEnvTiles; ++t) {
        char tmp[32];
        std::snprintf(tmp, sizeof(tmp), " %.6g", e.ms[t]);
        out += tmp;
      }
      out += "\n";
    }
  }
  if (len) *len = (int64_t)out.size() + 1;
  if (!buf) return MPS_OK;
  if (cap < (int64_t)out.size() + 1) return fail(MPS_ERR_ARG, "autotune table buffer too small");
  std::memcpy(buf, out.c_str(), out.size() + 1);
  return MPS_OK;
}

mps_status mps_autotune_reset(void) {
  std::lock_guard<std::mutex> g(g_tune_mu);
  g_tune.clear();
  return MPS_OK;
}

mps_status mps_set_timing(mps_handle h, int32_t enabled) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if ((st = sync(h)) != MPS_OK) return st;
  h->timing = enabled != 0;
  h->tm = mps_timing{};
  h->ev_env_used = h->ev_close_used = 0;
  return MPS_OK;
}

mps_status mps_get_timing(mps_handle h, mps_timing* out) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if (!out) return fail(MPS_ERR_ARG, "NULL output");
  if ((st = flush_timing(h)) != MPS_OK) return st;
  *out = h->tm;
  return MPS_OK;
}

mps_status mps_device_bytes(mps_handle h, size_t* bytes) {
  mps_status st = check_handle(h);
  if (st != MPS_OK) return st;
  if (!bytes) return fail(MPS_ERR_ARG, "NULL output");
  *bytes = h->held;
  return MPS_OK;
}

mps_status mps_selftest_mfma(double* out) {
  if (!out) return fail(MPS_ERR_ARG, "NULL output");
  double* d = nullptr;
  hipError_t e = hipMalloc((void**)&d, 1024 * sizeof(double));
  if (e != hipSuccess) return fail(MPS_ERR_DEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
  e = launch_selftest_mfma(d, nullptr);
  if (e == hipSuccess) e = hipMemcpy(out, d, 1024 * sizeof(double), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return fail(MPS_ERR_DEVICE, std::string("selftest: ") + hipGetErrorString(e));
  return MPS_OK;
}

}  // extern "C"
