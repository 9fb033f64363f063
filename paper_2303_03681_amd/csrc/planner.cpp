// Pauli-sum planner (host C++).  See planner.h.
#include "planner.h"

#include <algorithm>
#include <cmath>
#include <unordered_map>

namespace mps {

namespace {

struct TermShape {
  int lo, hi;  // admissible cut bonds [lo, hi]
  int m, n;    // support (m > n: identity string)
};

TermShape shape_of(const uint8_t* code, int nq) {
  TermShape t{0, 0, nq, -1};
  for (int q = 0; q < nq; ++q)
    if (code[q]) {
      t.m = q;
      break;
    }
  for (int q = nq - 1; q >= 0; --q)
    if (code[q]) {
      t.n = q;
      break;
    }
  if (t.n < 0) {  // identity: close the bond-0 roots (lambda_0^2 = 1 against the identity)
    t.lo = t.hi = 0;
    return t;
  }
  if (t.m == t.n) {  // one letter: lambda^2 root against the single right update
    t.lo = t.hi = t.m;
    return t;
  }
  int best_len = 0, best_g0 = -1;
  int run = 0;
  for (int q = t.m + 1; q < t.n; ++q) {
    if (code[q] == 0) {
      ++run;
      if (run > best_len) {
        best_len = run;
        best_g0 = q - run + 1;
      }
    } else {
      run = 0;
    }
  }
  if (best_len > 0) {
    t.lo = best_g0;                 // left part ends just before the run
    t.hi = best_g0 + best_len;      // left part swallows the whole run
  } else {
    // No identity inside the support: split before the middle X/Y letter, so
    // that e.g. P Z..Z P P Z..Z P becomes two shared Z-chain halves; with at
    // most one X/Y letter, cut before the last letter.
    int pos[64];
    int r = 0;
    for (int q = t.m; q <= t.n && r < 64; ++q)
      if (code[q] == 1 || code[q] == 2) pos[r++] = q;
    t.lo = t.hi = (r >= 2) ? pos[r / 2] : t.n;
  }
  return t;
}

struct Trie {
  std::unordered_map<uint64_t, int32_t> map;
  std::vector<TrieNode> nodes;
  int32_t child(int32_t parent, int site, uint8_t letter) {
    const uint64_t key = ((uint64_t)(uint32_t)parent << 2) | letter;
    auto it = map.find(key);
    if (it != map.end()) return it->second;
    const int32_t id = (int32_t)nodes.size();
    nodes.push_back(TrieNode{parent, (int16_t)site, letter});
    map.emplace(key, id);
    return id;
  }
};

inline int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Walks every term for meeting bond `meet`; fills the tries and closes.
void walk(int nq, int64_t T, const uint8_t* codes, const std::vector<TermShape>& shp, int meet,
          Trie& L, Trie& R, std::vector<int16_t>* cb, std::vector<int32_t>* cl,
          std::vector<int32_t>* cr) {
  for (int64_t k = 0; k < T; ++k) {
    const uint8_t* code = codes + k * (int64_t)nq;
    const TermShape& s = shp[k];
    if (s.n < 0) {
      if (cb) {
        (*cb)[k] = 0;
        (*cl)[k] = root_ref(0);
        (*cr)[k] = root_ref(0);
      }
      continue;
    }
    const int c = clampi(meet, s.lo, s.hi);
    int32_t lref = root_ref(s.m);
    for (int q = s.m; q < c; ++q) lref = L.child(lref, q, code[q]);
    int32_t rref = root_ref(s.n + 1);
    for (int q = s.n; q >= c; --q) rref = R.child(rref, q, code[q]);
    if (cb) {
      (*cb)[k] = (int16_t)c;
      (*cl)[k] = lref;
      (*cr)[k] = rref;
    }
  }
}

// Renumber so that nodes are grouped by site (ascending for the left trie,
// descending for the right) and, within a site, by parent.
std::vector<int32_t> regroup(std::vector<TrieNode>& nodes, bool ascending) {
  const size_t n = nodes.size();
  std::vector<int32_t> newid(n, -1);
  std::vector<int32_t> order(n);
  for (size_t i = 0; i < n; ++i) order[i] = (int32_t)i;
  // parents are always at an earlier site in processing order, so sorting by
  // (processing position of site, new parent id) is well defined if done site
  // by site; a stable sort on site first, then per-site sort by parent id.
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return ascending ? nodes[a].site < nodes[b].site : nodes[a].site > nodes[b].site;
  });
  size_t i = 0;
  int32_t next = 0;
  std::vector<TrieNode> out(n);
  while (i < n) {
    size_t j = i;
    while (j < n && nodes[order[j]].site == nodes[order[i]].site) ++j;
    auto pkey = [&](int32_t idx) -> int64_t {
      const int32_t p = nodes[idx].parent;
      return is_root(p) ? (int64_t)p : (int64_t)newid[p] + (1LL << 40);
    };
    std::stable_sort(order.begin() + i, order.begin() + j,
                     [&](int32_t a, int32_t b) { return pkey(a) < pkey(b); });
    for (size_t t = i; t < j; ++t) newid[order[t]] = next++;
    i = j;
  }
  for (size_t t = 0; t < n; ++t) {
    TrieNode nd = nodes[t];
    if (!is_root(nd.parent)) nd.parent = newid[nd.parent];
    out[newid[t]] = nd;
  }
  nodes.swap(out);
  return newid;
}

}  // namespace

bool build_pauli_plan(int nq, int64_t T, const uint8_t* codes, const double* coeffs,
                      PauliPlan& plan, std::string& err) {
  if (nq < 1 || nq > 30000) {
    err = "n_qubits must be in [1, 30000]";
    return false;
  }
  if (T < 0 || T > (1LL << 30)) {
    err = "n_terms must be in [0, 2^30]";
    return false;
  }
  if (T > 0 && (!codes || !coeffs)) {
    err = "codes and coeffs must not be NULL";
    return false;
  }
  for (int64_t i = 0; i < T * (int64_t)nq; ++i)
    if (codes[i] > 3) {
      err = "Pauli codes must be 0..3";
      return false;
    }
  for (int64_t k = 0; k < T; ++k)
    if (!std::isfinite(coeffs[k])) {
      err = "non-finite coefficient";
      return false;
    }
  std::vector<TermShape> shp((size_t)T);
  for (int64_t k = 0; k < T; ++k) shp[k] = shape_of(codes + k * (int64_t)nq, nq);

  // meeting bond: coarse scan then local refinement on the trie node count
  auto cost = [&](int meet) {
    Trie L, R;
    L.map.reserve((size_t)std::min<int64_t>(T * 4, 1 << 24));
    R.map.reserve((size_t)std::min<int64_t>(T * 4, 1 << 24));
    walk(nq, T, codes, shp, meet, L, R, nullptr, nullptr, nullptr);
    return (int64_t)(L.nodes.size() + R.nodes.size());
  };
  int best = nq / 2;
  if (nq > 2 && T > 0) {
    int64_t best_cost = cost(best);
    const int step = std::max(1, nq / 12);
    for (int c = std::max(1, nq / 4); c <= (3 * nq) / 4; c += step) {
      if (c == best) continue;
      const int64_t v = cost(c);
      if (v < best_cost) {
        best_cost = v;
        best = c;
      }
    }
    for (int d = -step + 1; d < step; ++d) {
      const int c = best + d;
      if (c < 1 || c >= nq || d == 0) continue;
      const int64_t v = cost(c);
      if (v < best_cost) {
        best_cost = v;
        best = c;
      }
    }
  }

  Trie L, R;
  plan = PauliPlan();
  plan.n_qubits = nq;
  plan.n_terms = T;
  plan.meet = best;
  plan.coeffs.assign(coeffs, coeffs + T);
  plan.close_bond.resize((size_t)T);
  plan.close_left.resize((size_t)T);
  plan.close_right.resize((size_t)T);
  walk(nq, T, codes, shp, best, L, R, &plan.close_bond, &plan.close_left, &plan.close_right);
  plan.left.swap(L.nodes);
  plan.right.swap(R.nodes);
  const std::vector<int32_t> lmap = regroup(plan.left, true);
  const std::vector<int32_t> rmap = regroup(plan.right, false);
  for (int64_t k = 0; k < T; ++k) {
    if (!is_root(plan.close_left[k])) plan.close_left[k] = lmap[plan.close_left[k]];
    if (!is_root(plan.close_right[k])) plan.close_right[k] = rmap[plan.close_right[k]];
  }
  return true;
}

}  // namespace mps
