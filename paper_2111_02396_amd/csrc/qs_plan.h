// Host-side planning: Kraus bounds, greedy gate fusion, fused matrices.
// Plain C++17 (no device code), so the planner can be exercised on a CPU.
#pragma once

#include <complex>
#include <cstdint>
#include <vector>

namespace qs {

using cd = std::complex<double>;

// An operation as the planner sees it: matrix bit j <-> q[j].
struct PlanOp {
    int k = 0;
    int q[5] = {0, 0, 0, 0, 0};
};

// A fused block: ascending qubits, time-ordered member operations.
struct Block {
    int k = 0;
    int q[5] = {0, 0, 0, 0, 0};
    std::vector<int> ops;
};

// Smallest eigenvalue of a d x d Hermitian matrix (row-major), via the real
// symmetric 2d x 2d embedding [[Re, -Im], [Im, Re]] and cyclic Jacobi sweeps.
double hermitian_min_eigenvalue(int d, const cd *A);

// G = K^dag K for a d x d matrix.
void gram(int d, const cd *K, cd *G);

// Kraus bounds (Section 3.5): pbar_i = max(lambda_min(K_i^dag K_i), 0);
// mixture = every K_i^dag K_i is c_i I within 1e-12 (entrywise).
void kraus_bounds(int k, int n_kraus, const cd *kraus, double *pbar, bool *mixture);

// Greedy fusion (Section 3.2).  Operations are taken in time order; the
// earliest unassigned operation seeds a block; the block then repeatedly
// absorbs the earliest operation that (a) is the first unassigned operation
// on each of its qubits and (b) touches the block's qubits, preferring those
// that add no new qubit, while the union stays within max_fuse qubits.
// Operations wider than max_fuse form a block of their own.  Condition (a)
// makes "apply the blocks in creation order" equal to "apply the operations
// in time order".
// After the greedy pass, merge_subset_blocks folds a block into the nearest
// later (else earlier) block that shares a qubit with it whenever its qubits
// are a subset of that block's: no block in between touches those qubits, so
// the union of the two blocks' operations in time order keeps every qubit's
// order and the block order stays valid (also restricted to any range of
// operations).  The greedy rule otherwise leaves one-qubit blocks for a
// qubit's first operations when the gate that follows them is not yet ready.
std::vector<Block> fuse_greedy(int n_qubits, const std::vector<PlanOp> &ops, int max_fuse,
                               std::vector<int> *op_block = nullptr);
void merge_subset_blocks(std::vector<Block> &blocks);

// Then merge_cheaper_blocks fuses two blocks that share a qubit (the later
// within a small window) into one of at most max_fuse qubits when the wider
// block costs less than the two (block_cost, by width) and the blocks in
// between touch neither the earlier block's qubits (the union takes the later
// block's place) or not the later one's (it takes the earlier one's place).
double block_cost(int k);
void merge_cheaper_blocks(std::vector<Block> &blocks, int max_fuse);

// Fused matrix of a subset of operations (time-ordered indices) acting on
// the ascending qubit set q[0..k-1]: the product of the embedded operator
// matrices, latest on the left.  mats[o] = matrix of op o (its own target
// order), or nullptr for an identity placeholder.  out: (2^k)^2 row-major.
void fused_matrix(int k, const int *q, const std::vector<int> &members,
                  const std::vector<PlanOp> &ops, const std::vector<const cd *> &mats, cd *out);

// Ascending union of the qubits of `members`; returns its size.
int union_qubits(const std::vector<int> &members, const std::vector<PlanOp> &ops, int *q_out);

// Permute a d x d matrix written for target order t[0..k-1] into ascending
// target order.
void to_ascending_order(int k, const int *t, const cd *in, cd *out, int *t_sorted);

bool is_identity_multiple(int d, const cd *M, double tol, cd *scalar_out);

// A tile sweep: blocks (indices into the block list, in application order)
// whose qubits all lie in the tile's bit set, which always holds bits
// 0..low_bits-1.  `bits` is ascending.
struct Sweep {
    std::vector<int> bits;
    std::vector<int> blocks;
};

// Group an ordered, valid block list into tile sweeps of at most max_bits
// tile bits.  Blocks are taken in a dependency-respecting order (a block
// waits for the previous block on each of its qubits): a sweep repeatedly
// takes a ready block that adds the fewest new bits (earliest first), as
// long as the bit budget, max_blocks and the matrix budget (the sum of
// slot_per_k[k] over the sweep's blocks) allow.  With search, every ready
// block is also tried as the sweep's first pick and the fill that absorbs
// the most block cost (block_cost) is kept.  The result, sweep by sweep, is
// again a valid application order.  A block that fits no tile of max_bits
// gets a sweep of its own whose bit set is wider than max_bits.
std::vector<Sweep> group_sweeps(int n_qubits, const std::vector<Block> &blocks, int max_bits,
                                int low_bits, int max_blocks, int mat_budget,
                                const int *slot_per_k, bool search = true);

// The grouping with the fewest sweeps among group_sweeps' and `restarts`
// randomized fills: each sweep starts from a ready block drawn among those
// that fit and then adds the ready block of least qubit growth, ties drawn
// at random (a counter-based generator seeded with `seed`, so the result is
// reproducible).  A fill is abandoned once it cannot end with fewer sweeps
// than the best so far.
std::vector<Sweep> group_sweeps_best(int n_qubits, const std::vector<Block> &blocks, int max_bits,
                                     int low_bits, int max_blocks, int mat_budget,
                                     const int *slot_per_k, int restarts, uint64_t seed);

}  // namespace qs
