// Pauli-sum planner: turns every string of sum_k c_k P_k into one closing
// trace Tr(L_c R_c) at a bond c, where L_c is the transfer-matrix product of
// the string's letters left of c started from diag(lambda^2) at its first
// non-identity site (Eqs. expec1, expec2) and R_c the product of the letters
// right of c started from the identity at its last one (the right boundary
// of a right-canonical MPS).  Products are shared through two tries: strings
// with the same prefix (first site and letters) share L nodes, strings with
// the same suffix share R nodes.
//
// Cut rule: inside the longest interior run of identity letters, clamped to a
// meeting bond chosen to minimise the number of trie nodes; strings without
// such a run are cut before their middle X/Y letter (before the last site if
// they have fewer than two); single-site strings after the lambda^2 root.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace mps {

// A reference to an environment at some bond: a trie node (>= 0) or the
// root at bond b (-(b + 1)): diag(lambda_b^2) on the left, identity on the right.
inline int32_t root_ref(int bond) { return -(bond + 1); }
inline bool is_root(int32_t ref) { return ref < 0; }
inline int root_bond(int32_t ref) { return -ref - 1; }

struct TrieNode {
  int32_t parent;   // reference of the environment the letter is applied to
  int16_t site;     // the site whose tensor and letter are applied
  uint8_t letter;   // 1 X, 2 Y, 3 Z (0 I for identity crossings)
};

struct PauliPlan {
  int n_qubits = 0;
  int64_t n_terms = 0;
  int meet = 0;
  std::vector<double> coeffs;
  // left trie: node bond = site + 1; grouped by site, parents before children
  std::vector<TrieNode> left;
  // right trie: node bond = site; grouped by descending site
  std::vector<TrieNode> right;
  // per term: bond and the two references closed there
  std::vector<int16_t> close_bond;
  std::vector<int32_t> close_left, close_right;
};

// Builds the plan; returns false and sets err on invalid input.
bool build_pauli_plan(int n_qubits, int64_t n_terms, const uint8_t* codes, const double* coeffs,
                      PauliPlan& plan, std::string& err);

}  // namespace mps
