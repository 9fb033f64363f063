/*
 * mps.h -- C ABI of the MI355X matrix-product-state energy evaluator.
 *
 * The library evaluates E(theta) = sum_k c_k <psi(theta)|P_k|psi(theta)> for a
 * state held as a right-canonical matrix product state (MPS) of bond
 * dimension D, following the paper's Methods:
 *   - "MPS algorithm for quantum circuit simulation": right-canonical gauge
 *     (Eq. rc), one-qubit gates (Eq. 1q), two-qubit gates by the Hastings
 *     scheme: two-site contraction (Eq. C), lambda scaling (Eq. C~),
 *     truncated SVD (Eq. svd) by the one-sided Jacobi method of Algorithm 1,
 *     site update (Eq. Bl);
 *   - "The implementation of UCCSD with matrix product states": Pauli-string
 *     expectations from lambda^2 and transfer matrices (Eqs. expec1,
 *     expec2), the energy as the coefficient-weighted sum of them.
 *
 * Conventions shared by every entry point
 *   - Sites 0..N-1 are qubits 0..N-1; bond b sits left of site b; bond 0 and
 *     bond N have dimension 1.  Site tensor B_q has shape (2, D_q, D_{q+1}),
 *     row-major, complex numbers as (re, im) double pairs.
 *   - Two-qubit gate matrices are 4x4 with row/column index 2*i_q0 + i_q1,
 *     one-qubit gates 2x2; row-major (re, im) pairs.
 *   - Pauli codes: 0 = I, 1 = X, 2 = Y, 3 = Z, one byte per qubit.
 *   - Ownership: the caller owns every host array and may reuse it when the
 *     call returns (the library copies).  The library owns all device memory
 *     it allocates until the matching *_destroy.
 *   - Streams: work is enqueued on the handle's stream (mps_config.stream, a
 *     hipStream_t, or a stream the library creates when NULL).  Calls that
 *     return host values synchronise that stream.
 *   - Errors: every call returns an mps_status; on failure, output arguments
 *     are left untouched and mps_last_error() (thread-local) describes the
 *     failure.  MPS_ERR_ARG, MPS_ERR_BUDGET, MPS_ERR_NOCONV and
 *     MPS_ERR_NONFINITE leave the MPS as it was before the call.
 *     MPS_ERR_DEVICE poisons the handle: later calls on it return
 *     MPS_ERR_DEVICE until mps_destroy.
 *   - Threading: one handle is used by one thread at a time.
 */
#ifndef MPS_H_
#define MPS_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mps_state* mps_handle;
typedef struct mps_psum* mps_pauli_sum;

typedef enum {
  MPS_OK = 0,
  MPS_ERR_ARG = -1,       /* invalid argument or shape                          */
  MPS_ERR_OOM = -2,       /* device allocation failed                           */
  MPS_ERR_BUDGET = -3,    /* the handle's HBM budget would be exceeded          */
  MPS_ERR_NOCONV = -4,    /* Jacobi SVD did not converge within the sweep limit */
  MPS_ERR_NONFINITE = -5, /* NaN/Inf in an input or an SVD                      */
  MPS_ERR_DEVICE = -6,    /* HIP runtime error (handle poisoned)                */
  MPS_ERR_STATE = -7      /* call not valid in the current state                */
} mps_status;

/* Arithmetic of the environment (transfer-matrix) products of Eq. (expec2).
 * Gates, SVDs, canonicalisation and the final energy sum are always FP64.
 * The split variants store environments in FP32 like C64 and evaluate the
 * transfer-matrix products on 16-bit matrix cores: each FP32 operand x is
 * split into a leading 16-bit part h and a trailing part l (x ~ h + l / S)
 * and each real product is h h' + (h l' + l h') / S with FP32 accumulation
 * (about 16 significant bits for bf16, S = 1; about 22 for f16, S = 2^11,
 * which needs operands bounded by 1, as site tensors and environments are).
 * For every precision the closing traces Re Tr(L R) accumulate in FP64 (from
 * FP32 environments for C64 and the split variants). */
typedef enum {
  MPS_PREC_C128 = 0,       /* complex128 on FP64 MFMA                              */
  MPS_PREC_C64 = 1,        /* complex64 on FP32 MFMA                               */
  MPS_PREC_SPLIT_BF16 = 2, /* FP32 split into bf16 h + l, bf16 MFMA, FP32 accumulate */
  MPS_PREC_SPLIT_F16 = 3   /* FP32 split into f16 h + l/2^11, f16 MFMA, FP32 accum.  */
} mps_precision;

typedef struct {
  int32_t n_qubits;          /* N >= 1                                             */
  int32_t max_bond;          /* D >= 1: bond dimensions are capped at D            */
  double svd_cutoff;         /* keep sigma_j > svd_cutoff * ||sigma||_2 (Methods,
                                two-qubit gate: "truncate the small singular
                                values below a certain threshold or simply
                                reserve the largest few"); >= 0                   */
  int32_t max_jacobi_sweeps; /* 0 = default (60)                                   */
  const uint8_t* init_bits;  /* N bytes in {0,1}: initial product state; NULL = 0s */
  void* stream;              /* hipStream_t to enqueue on; NULL = library-owned    */
  size_t hbm_budget_bytes;   /* 0 = unlimited; otherwise device bytes the handle
                                may hold (MPS, workspaces, environments)           */
} mps_config;

/* Create an MPS holding the product state |init_bits> (Methods, Hartree-Fock
 * reference of the UCC ansatz: B^s = delta_{s,b}, all bonds of dimension 1,
 * lambda = 1).  Allocates the site tensors at their maximal size
 * min(D, 2^min(b, N-b)) per bond.  *out receives the handle. */
mps_status mps_create(const mps_config* cfg, mps_handle* out);

/* Release all device memory of the handle.  NULL is a no-op. */
mps_status mps_destroy(mps_handle h);

/* Return to the product state |bits> (NULL = |0..0>) keeping allocations. */
mps_status mps_reset(mps_handle h, const uint8_t* bits);

/* Apply one gate.  q1 < 0: one-qubit gate on q0 (Eq. 1q), u = 2x2.
 * q1 = q0 + 1: two-qubit gate (Eqs. C, C~, svd, Bl) with truncation to
 * min(D, #{sigma_j > cutoff ||sigma||}) singular values and renormalisation
 * to unit norm, u = 4x4.  Any other q1 is MPS_ERR_ARG. */
mps_status mps_apply_gate(mps_handle h, int32_t q0, int32_t q1, const double* u);

/* Apply n gates in order.  u_packed holds 32 doubles per gate (a 4x4 complex
 * matrix; a 2x2 gate uses the first 8).  Consecutive two-qubit gates on
 * disjoint bonds are processed as one batch (one batched SVD).  Where at most
 * four such gates form a batch and both outer bonds of each have capacity
 * min(max_bond, 2^min(b, N-b)) <= 64 (chains of dependent gates, as in
 * Pauli-exponential ladders), each gate runs as one fused device step and the
 * run is queued without host round trips.  On error the gates before the
 * failing gate (fused) or batch stay applied; *n_done (may be NULL) receives
 * the number of gates applied.  The result does not depend on which path a
 * gate takes beyond rounding. */
mps_status mps_apply_gates(mps_handle h, int64_t n, const int32_t* q0, const int32_t* q1,
                           const double* u_packed, int64_t* n_done);

/* Apply one gate list to each of n_handles distinct MPSs (handles[i] gets
 * n_gates[i] gates from q0[i], q1[i], u_packed[i], laid out as for
 * mps_apply_gates) so that the dependent gate chains of several MPSs advance
 * together and share the device (the batching of concurrent requests).
 * When every two-qubit gate satisfies the fused-path limit of
 * mps_apply_gates (both outer bond capacities <= 64), one sequence of device
 * launches on `stream` (a hipStream_t; NULL = the first handle's stream)
 * applies gate s of every list at launch s, one workgroup per MPS, exactly
 * as mps_apply_gates' fused path would.  Otherwise step s applies gate s of
 * every list as one batched step on the first handle's stream: the
 * one-qubit gates, then all two-qubit gates of the step -- on distinct MPSs,
 * hence independent -- as one batch of the multi-workgroup path (one batched
 * contraction, Jacobi SVD and site update; Eqs. C, C~, svd, Bl), the same
 * arithmetic as mps_apply_gates' batched path up to the rotation order of
 * small SVDs.  A failed gate (NOCONV, NONFINITE) stops only its own list,
 * n_done[i] (may be NULL) receives the gates applied to handle i, and the
 * first failure in handle order is returned.  Synchronises `stream` and
 * every handle's stream. */
mps_status mps_apply_gates_multi(int32_t n_handles, const mps_handle* handles,
                                 const int64_t* n_gates, const int32_t* const* q0,
                                 const int32_t* const* q1, const double* const* u_packed,
                                 void* stream, int64_t* n_done);

/* Allow (enabled != 0, the default) or forbid the fused single-gate path of
 * mps_apply_gates; with it forbidden every two-qubit gate takes the batched
 * path.  For comparisons and tests. */
mps_status mps_set_fused_gates(mps_handle h, int32_t enabled);

/* Number of groups (1..3, default 2) into which the batched gate SVDs of
 * one brickwork layer are split, each group's Algorithm 1 rounds (register
 * and wide-row kernels) queued on a stream of its own so that the rounds of one group
 * fill the compute units the others leave idle.  Used only when a round
 * would launch more than 256 workgroups.  Each matrix sees the same
 * rotation rounds for every group count; 1 turns the split off (for
 * comparisons and tests).  MPS_ERR_ARG outside 1..3. */
mps_status mps_set_jacobi_groups(mps_handle h, int32_t groups);

/* Copy the state of src into dst (site tensors, lambdas, bond dimensions,
 * canonical flag, norm, discarded weight), device to device on dst's
 * stream after src's stream has drained; returns when the copy is complete,
 * so later work on either handle cannot race with it.  Both handles need the same qubit
 * count and bond capacities (same n_qubits and max_bond); their cutoffs and
 * sweep limits may differ.  Used for circuit-prefix caching: keep the state
 * after an unchanged gate prefix and continue copies of it with different
 * suffixes.  MPS_ERR_ARG for other shapes, dst unchanged. */
mps_status mps_copy(mps_handle dst, mps_handle src);

/* Restore the exact right-canonical gauge (Eq. rc), exact Schmidt values on
 * every bond and unit norm: a left-to-right orthonormalisation sweep followed
 * by a right-to-left SVD sweep, both by one-sided Jacobi.  Only round-off
 * singular values (<= 1e-14 ||sigma||) are dropped. */
mps_status mps_canonicalize(mps_handle h);

/* Norm ||psi|| found by the last mps_canonicalize (before it normalised the
 * state) or, after gates, by the last mps_expect_pauli_sum; 1 after
 * create/reset. */
mps_status mps_norm(mps_handle h, double* norm);

/* Sum of the relative discarded weights sum_{j>k} sigma_j^2 / sum sigma_j^2
 * of every truncating two-qubit gate since create/reset. */
mps_status mps_discarded_weight(mps_handle h, double* weight);

/* Current bond dimensions D_0 .. D_N (N+1 values). */
mps_status mps_bond_dims(mps_handle h, int32_t* dims);

/* Compile a Pauli sum sum_k coeffs[k] P_k on n_qubits qubits into a plan
 * (Eq. expec2 generalised to every string: prefix and suffix transfer-matrix
 * tries that share common sub-strings, meeting at one bond per string).
 * codes is n_terms x n_qubits bytes.  The plan is independent of any handle
 * with the same n_qubits. */
mps_status mps_pauli_sum_create(int32_t n_qubits, int64_t n_terms, const uint8_t* codes,
                                const double* coeffs, mps_pauli_sum* out);

/* Release a plan.  NULL is a no-op. */
mps_status mps_pauli_sum_destroy(mps_pauli_sum p);

/* Planner statistics: numbers of left and right transfer-matrix updates and
 * of distinct closing pairs per evaluation, and the meeting bond. */
mps_status mps_pauli_sum_stats(mps_pauli_sum p, int64_t* n_left_updates, int64_t* n_right_updates,
                               int64_t* n_closes, int32_t* meet_bond);

/* Copy the plan out for inspection: the left trie (parent reference, site,
 * letter per node; a parent < 0 is the root -(b+1) at bond b, i.e.
 * diag(lambda_b^2)), the right trie (same, roots are identities at bond b,
 * nodes hold transposed right environments) and, per term, the bond and the
 * two references whose closing trace Tr(L R) gives <P_k>.  Arrays are sized
 * by mps_pauli_sum_stats (left, right) and n_terms; any may be NULL. */
mps_status mps_pauli_sum_export(mps_pauli_sum p, int32_t* left_parent, int32_t* left_site,
                                int32_t* left_letter, int32_t* right_parent, int32_t* right_site,
                                int32_t* right_letter, int32_t* close_bond, int32_t* close_left,
                                int32_t* close_right);

/* E = sum_k c_k Re<P_k> (Methods, UCC: the energy from the expectation
 * values of the qubit Hamiltonian; Eqs. expec1/expec2 for each <P_k>).
 * The state is not modified.  In exact canonical form (after create/reset,
 * mps_canonicalize or mps_import) the tries start from diag(lambda^2)
 * and the identity (Eqs. expec1, rc).  After gates, whose truncation leaves
 * the sites only nearly right-orthonormal, they start instead from the
 * identity environments of both boundaries, sum B^+ L B and sum B R B^+
 * (FP64, one chain of N updates each), and every <P_k> is divided by
 * <psi|psi>: the same values, without canonicalisation.  mps_norm then
 * reports sqrt(<psi|psi>).  The transfer-matrix products run in `prec`; the
 * per-string values are summed in FP64 with compensation in string order, so
 * the result does not depend on how strings are batched.  per_term, if not
 * NULL, receives Re<P_k> for every k (n_terms doubles). */
mps_status mps_expect_pauli_sum(mps_handle h, mps_pauli_sum p, mps_precision prec, double* energy,
                                double* per_term);

/* Linear combinations of the expectations of one plan's strings:
 * out[r] = sum_{i = row_ptr[r]}^{row_ptr[r+1]-1} vals[i] Re<P_{cols[i]}>, for
 * r < n_rows (CSR on the host; cols index the plan's strings in the order
 * given to mps_pauli_sum_create; the plan's own coefficients are not used).
 * The strings are evaluated exactly as by mps_expect_pauli_sum (same roots,
 * normalisation, precisions); each row is then summed on the device with the
 * same compensated, order-fixed arithmetic as the energy.  For quantities
 * such as reduced density matrices: an operator's JW expansion sum v_k P_k
 * gives Re<O> and Im<O> as two rows with Re v_k and Im v_k.  Row arrays are
 * validated on the host (row_ptr[0] = 0, non-decreasing, 0 <= cols < number
 * of strings): MPS_ERR_ARG otherwise. */
mps_status mps_expect_pauli_rows(mps_handle h, mps_pauli_sum p, mps_precision prec, int64_t n_rows,
                                 const int64_t* row_ptr, const int64_t* cols, const double* vals,
                                 double* out);

/* E over several plans on one state: the chunks of a Pauli sum whose trie
 * environments would not fit in device memory at once (each chunk a plan of
 * its own, same qubit count).  Each plan is evaluated exactly as by
 * mps_expect_pauli_sum; its compensated (sum, error) pair stays on the
 * device, and the pairs are added there in plan order with the same
 * error-free transformations, so the final sum of c_k Re<P_k> over all
 * chunks (Methods, UCC: the energy from the qubit Hamiltonian's expectation
 * values) is an FP64 device result read once.  per_term, if not NULL,
 * receives Re<P_k> of every plan's strings, concatenated in plan order.
 * MPS_ERR_ARG for n_plans < 1, a NULL plan or a qubit-count mismatch. */
mps_status mps_expect_pauli_sums(mps_handle h, int32_t n_plans, const mps_pauli_sum* plans,
                                 mps_precision prec, double* energy, double* per_term);

/* Several states, each with its own plan (plans[i] for states[i], e.g. the
 * fragments of a DMET-like decomposition; Methods, heterogeneous
 * parallelization: fragments are independent), evaluated together as
 * mps_expect_pauli_sum would evaluate each (Eqs. expec1, expec2, the same
 * roots, boundary environments and normalisation).  The environment updates
 * of equal depth in the states' launch sequences run as one launch per GEMM
 * half, every item carrying its own site tensor and dims, on states[0]'s
 * stream, so count states take the launches of the deepest one instead of
 * the sum; so do the set-up steps (site tensors in environment precision,
 * each depth of the boundary-environment chains, the roots).  The closing
 * traces, string values and compensated energies follow per state.
 * energies[i] receives state i's E; per_term (may be NULL, as may any
 * per_term[i]) receives Re<P_k> of plan i.  The values equal those of count
 * separate calls bit for bit (every tile shape accumulates in the same
 * order).  Each other state's stream is synchronised before the shared
 * launches (its earlier work done); the call returns after the work is done.  Tile autotuning, graph replay and
 * per-state timing do not apply.  MPS_ERR_ARG for count < 0, NULL arrays or
 * plans, repeated states, a qubit-count mismatch or more than 32767 sites
 * (qubits + 1 per state) in one call; count = 0 is a no-op. */
mps_status mps_expect_pauli_sum_multi(int32_t count, const mps_handle* states, const mps_pauli_sum* plans,
                                      mps_precision prec, double* energies, double* const* per_term);

/* The state as a dense vector (Eq. mps: c_{i_1..i_N} = B^{i_1} ... B^{i_N},
 * contracted site by site on the device): psi receives 2^N complex
 * amplitudes as (re, im) pairs, qubit 0 the most significant bit of the
 * index.  The amplitudes are those of the stored tensors (after truncating
 * gates the stored state has unit norm up to rounding; no renormalisation).
 * N <= 26 (1 GiB of amplitudes), else MPS_ERR_ARG.  Allocates two 2^N
 * device buffers for the duration of the call. */
mps_status mps_to_statevector(mps_handle h, double* psi);

/* Copy site q's tensor to the host: *dl, *dr receive D_q, D_{q+1}; b (may be
 * NULL) receives 2*D_q*D_{q+1} complex values as (re, im) pairs in
 * [s][alpha][beta] order; lambda_left (may be NULL) receives the D_q
 * singular values of bond q. */
mps_status mps_export(mps_handle h, int32_t q, int32_t* dl, int32_t* dr, double* b,
                      double* lambda_left);

/* Overwrite site q's tensor and the singular values of bond q.  dl must equal
 * D_{q} of the left neighbour's right bond (or 1 at q = 0) once all sites are
 * imported; the library checks shapes against its capacity only.  Importing
 * marks the state canonical: the caller asserts the imported tensors are in
 * right-canonical form with Schmidt values (use mps_canonicalize otherwise). */
mps_status mps_import(mps_handle h, int32_t q, int32_t dl, int32_t dr, const double* b,
                      const double* lambda_left);

/* Standalone one-sided Jacobi SVD (Algorithm 1) of the n_vec vectors of
 * length vec_len given row-major in `vectors` (host): the vectors are
 * rotated pairwise until mutually orthogonal.  sigma receives the n_vec
 * norms sorted descending; out_vectors (n_vec x vec_len, may be NULL)
 * receives the normalised vectors in the same order (zero where sigma = 0);
 * *sweeps (may be NULL) the number of sweeps.  For a matrix A whose rows are
 * the vectors, A = U diag(sigma) W with W = out_vectors. */
mps_status mps_jacobi_svd(int32_t n_vec, int32_t vec_len, const double* vectors, double* sigma,
                          double* out_vectors, int32_t* sweeps);

/* mps_jacobi_svd for callers that cannot allocate device memory (code
 * running under stream capture, tight serving loops, hosts that forbid
 * hipMalloc): same arguments, same kernels, same results, but every device
 * buffer -- the work and output vectors, norms, rotation counters, sigma and
 * launch descriptors -- lives in a fixed scratch array that the library
 * holds on each device it runs on until the process ends (about 8.1 MiB).
 * It calls no hipMalloc/hipFree and creates no stream: the work is enqueued
 * on `stream` (a hipStream_t; NULL = the null stream), which the call
 * synchronises before it returns.  Limits: 1 <= n_vec <= 512 and
 * 1 <= vec_len <= 512 (one 512 x 512 complex matrix), MPS_ERR_ARG beyond.
 * Every call on one device shares that device's scratch and keeps the last
 * call's contents (the call clears what it accumulates): calls that overlap
 * on one device, from several threads or streams, race and must be
 * serialised by the caller. */
mps_status mps_jacobi_svd_noalloc(int32_t n_vec, int32_t vec_len, const double* vectors, double* sigma,
                                  double* out_vectors, int32_t* sweeps, void* stream);

/* Tile autotuning of the environment-update GEMMs (c128 and c64; the split
 * precisions keep their one tile).  With `enabled` != 0, the first
 * mps_expect_pauli_sum of this handle that meets a launch class without a
 * table entry -- class = (device, precision, GEMM half, D_l, D_r,
 * ceil(log2 of the items in the launch)) -- runs that launch with every tile
 * shape (BM x BN x BK in {64x64x16, 32x32x16, 128x64x16, 64x128x16,
 * 64x64x32, 32x64x16, 128x128x16, 128x128x8}) twice, timed with HIP events, and records the
 * fastest; later launches of the class use it.  The table is process-wide
 * per device and shared by all handles.  Every tile shape gives bitwise
 * identical results (each output element accumulates its K range in the
 * same order), so tuning changes only speed; tuning launches are left out
 * of mps_get_timing's environment figures.  Off by default. */
mps_status mps_set_autotune(mps_handle h, int32_t enabled);

/* HIP-graph replay of the expectation (the batching direction's persistent
 * launch).  With `enabled` != 0, mps_expect_pauli_sum records its device work
 * from the trie roots to the energy -- every environment update, the closing
 * traces, the gather and the compensated sum -- into a HIP graph the first
 * time it meets a (Pauli sum, precision, bond dimensions, root kind)
 * combination, and afterwards replays that graph with one launch.  Work that
 * reads the live site and lambda buffers (site preparation, roots, boundary
 * environments) stays outside the graph and writes the fixed buffers the
 * graph reads, so a replay after gates sees the new state.  While tile
 * autotuning still has classes to measure the call runs eagerly.  The graph
 * holds no memset nodes.  c128 then keeps one more copy of the sites.
 * Results are bitwise those of the eager path.  Disabling frees the graph. */
mps_status mps_set_graphs(mps_handle h, int32_t enabled);

/* Use tile shape `tile` (0..7, in the order listed for mps_set_autotune) for
 * every c128/c64 environment GEMM of this handle, overriding the table;
 * -1 (the default) returns to the table or the default tile 0.  For
 * comparisons and tests.  Other values are MPS_ERR_ARG. */
mps_status mps_set_env_tile(mps_handle h, int32_t tile);

/* The tuning table as text, one line per launch class:
 *   device precision half D_l D_r bucket tile BMxBNxBK ms_0 .. ms_7
 * (half 1: X = L [A^0|A^1], half 2: L' = sum A^+ X; ms_t the faster of two
 * runs of tile t).  *len (may be NULL) receives the bytes needed including
 * the terminating NUL; buf may be NULL to query the length; a non-NULL buf
 * with cap below that length is MPS_ERR_ARG. */
mps_status mps_autotune_table(char* buf, int64_t cap, int64_t* len);

/* Forget every tuned class (all devices). */
mps_status mps_autotune_reset(void);

/* Timing of the transfer-matrix (environment update) kernels, measured with
 * HIP events around each launch while enabled. */
typedef struct {
  double env_ms;            /* summed duration of environment-update launches  */
  int64_t env_launches;     /* number of such launches                         */
  double env_flops;         /* algorithmic FLOPs of those launches (4M complex) */
  int64_t env_updates;      /* transfer-matrix updates performed               */
  double close_ms;          /* summed duration of closing (trace) launches     */
  double close_flops;       /* algorithmic FLOPs of the closing traces: 4 D^2  *
                             * per distinct (prefix, suffix) pair, Re Tr(L R)  */
  double expect_ms;         /* wall time of mps_expect_pauli_sum calls         */
  double gates_ms;          /* wall time of gate application                   */
  double canon_ms;          /* wall time of canonicalisation                   */
  int64_t jacobi_sweeps;    /* total Jacobi sweeps executed                    */
  double jacobi_ms;         /* device time of the multi-launch Jacobi rounds   */
  double jacobi_flops;      /* their algorithmic FLOPs: 32m per rotated pair,   *
                             * 8m per pair visited without rotation (rows of m) */
  int64_t graph_launches;   /* expectation graphs replayed (mps_set_graphs); the *
                             * env and close figures above cover eager launches */
  int64_t jacobi_batch_sweeps; /* sweeps launched for multi-launch Jacobi batches *
                                * (a batch runs until its slowest item converges) */
  int64_t jacobi_multi_items;  /* SVDs that ran as multi-launch rounds (rows of    *
                                * 129..1024 elements, more than 64 x 64 entries)   */
  int64_t jacobi_wide_items;   /* of those, SVDs with rows of 513..1024 elements   */
  int64_t jacobi_split_batches; /* batches whose rounds ran in >= 2 item groups    */
  double close_tile_flops;     /* FLOPs of the 64 x 64 Gram tiles the closing    *
                                * launches compute (every pair of a needed tile)  */
} mps_timing;

mps_status mps_set_timing(mps_handle h, int32_t enabled); /* also resets counters */
mps_status mps_get_timing(mps_handle h, mps_timing* out);

/* Device bytes currently held by the handle. */
mps_status mps_device_bytes(mps_handle h, size_t* bytes);

/* Layout self-check of the matrix-core instructions used by the dense
 * products: runs one product of known operands per instruction (FP64 and
 * FP32 16x16x4, bf16 and f16 16x16x32) on the device and writes each 16x16
 * result, read back through the lane
 * layout the kernels assume, to out (4 x 256 doubles, row-major: FP64
 * 16x16x4, FP32 16x16x4, then bf16 and f16 16x16x32 with
 * A[i][k] = ((i + 2k) mod 7) - 3 and B[k][j] = ((3k + j) mod 5) - 2). */
mps_status mps_selftest_mfma(double* out);

/* Thread-local description of the last error on this thread. */
const char* mps_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MPS_H_ */
