// Internal declarations shared by the library's translation units.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/sv.h"

namespace sv {

using cd = std::complex<double>;

// ---------------------------------------------------------------- errors
// Record a message for sv_last_error() and return `code`.
int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

// ---------------------------------------------------------------- gates
// Arity of a named gate kind (0 for SV_G_MATRIX, -1 for an unknown kind).
int gate_arity(int kind);
// Validate kind / k / params (not positions).
int check_gate_shape(const sv_gate &g);
// Validate positions against n: in range and pairwise distinct.
int check_gate_qubits(const sv_gate &g, int n);
// 2^k x 2^k matrix in the ABI order (q[0] = most significant local bit).
int gate_matrix_abi(const sv_gate &g, std::vector<cd> &out);
// Gate matrix and positions in CANONICAL order: positions sorted ascending,
// local bit j <-> j-th lowest position.
int gate_matrix_canonical(const sv_gate &g, std::vector<cd> &m, int *sorted_q);
// Split FP16 needs norm-preserving blocks: U^dagger U = I to 1e-6 per entry
// (check_unitary), for every MATRIX gate of a list (check_fp16_gates).
int check_unitary(const std::vector<cd> &U, int k, const char *what);
int check_fp16_gates(const sv_gate *g, int G);
// Convert between the ABI order of a block whose positions q[0..k-1] are
// already ascending (q[0] most significant) and the canonical order (q[0]
// least significant): a bit reversal of the local index, an involution.
void reverse_local_bits(const std::vector<cd> &in, int k, std::vector<cd> &out);

// ---------------------------------------------------------------- fusion
// Tile passes (SV_RULE_TILED): at most kTilePassMaxBlocks blocks of <= 4
// qubits; kTilePassMaxUnion bounds the union limit (tile_union_limit).
constexpr int kTilePassMaxBlocks = 16;
constexpr int kTilePassMaxUnion = 10;

struct Block {
    int k = 0;
    int q[SV_MAX_K] = {0};       // ascending positions
    std::vector<int> members;    // gate indices, in an order that keeps the circuit's product
    std::vector<cd> m;           // canonical 2^k x 2^k matrix (row-major)
    int pass = -1;               // tile pass of the block (SV_RULE_TILED), -1 = own launch
};

struct CostTable {
    bool valid = false;
    double ms[SV_MAX_K + 1] = {0};          // one application of a k-qubit block
    double tile[kTilePassMaxBlocks + 1] = {0};  // one tile pass holding s blocks of 4 qubits
};

// Blocks one tile-pass launch of the current launch shape holds with the
// operands of `precision` (SV_PREC_*; -1: of any precision, the split BF16
// capacity, the smallest); the tiled rule plans passes of at most this many
// blocks.
int tile_pass_capacity(int precision = -1);

// Tile bits of the current launch shape (13 or 14).
int tile_pass_bits();

// Union limit of the tile passes that SV_RULE_TILED plans (8 ..
// kTilePassMaxUnion; default 10, or the SV_TILE_UNION environment variable).
int tile_union_limit();
void set_tile_union_limit(int u);
// The tile of a pass whose blocks cover the positions U is U plus the lowest
// positions outside it, tile_bits in all; its amplitudes lie in runs of
// 2^tile_run_bits(U, tile_bits) consecutive ones (its positions 0, 1, .. in a
// row).
int tile_run_bits(uint64_t U, int tile_bits);
// The tiled rule lets a pass cover U when U fits a tile whose runs are at
// least as long as those of any union of `limit` positions, 2^(tile_bits -
// limit) amplitudes: every union of at most `limit` positions, and larger
// ones that hold enough of the lowest positions.  States of fewer than
// tile_bits qubits keep to `limit` positions.
bool tile_union_fits(uint64_t U, int n, int tile_bits, int limit);

// Cost table used when no autotuned table exists (relative units).
CostTable default_costs();
// Lookup of an autotuned table for (n, precision); falls back to defaults.
CostTable lookup_costs(int n, int precision, bool *found);
void store_costs(int n, int precision, const double *ms, const double *tile = nullptr);
// Incremented by every store_costs (invalidates choices priced on older tables).
uint64_t cost_version();

// Greedy fusion.  Gates must be validated first.  `cost` steers the
// enhanced rule.  Fills blocks (with canonical matrices).  The tiled rule
// plans passes of at most tile_pass_capacity(precision) blocks.
int fuse_gates(const sv_gate *g, int G, int n, int max_k, int rule, const CostTable &cost,
               std::vector<Block> &blocks, bool with_matrices = true, int precision = -1);
double plan_cost(const std::vector<Block> &blocks, const CostTable &cost);
// Tile grouping (see group_tile_passes): groups of block indices, in
// application order (consecutive blocks of one tile pass); a group of one is
// applied on its own.
std::vector<std::vector<size_t>> tile_groups(const std::vector<Block> &blocks, int n);
// Cost of the tiled plan of `blocks` with the table's tile and block costs.
double tiled_plan_cost(const std::vector<Block> &blocks, int n, const CostTable &cost);

// Canonical matrix of a block from its member gates.
void block_matrix(const sv_gate *g, Block &b);

// ---------------------------------------------------------------- density matrices
// Rewrite gates g (on qubits 0..n-1) with super operators among them as a
// regular circuit on 2n positions (rho row-major: row index on n..2n-1).  The
// new MATRIX gates point into `store`.
int dm_expand(const sv_gate *g, int G, int n, const sv_super_op *ops, int n_ops, std::vector<sv_gate> &out,
              std::vector<std::vector<double>> &store);
// Kraus channels sampled on pure states (sv_kraus_probabilities and the
// sampled application): validation, Kraus form and canonical matrices.
constexpr int kMaxKrausOps = 64;
struct KrausSet {
    int k = 0, n_ops = 0;
    int q[3] = {0, 0, 0};         // qubits, q[0] the most significant local bit
    int sorted_q[3] = {0, 0, 0};  // ascending
    std::vector<double> abi;      // n_ops matrices, ABI order, interleaved
    std::vector<cd> canon;        // n_ops matrices, canonical order
};
int kraus_canonical(const sv_super_op &op, int n, KrausSet &out);
// Kraus form of a KrausSuperGate (right == left; s NULL or Hermitian PSD):
// n_ops matrices in ABI order (see sv_kraus_form).
int kraus_form(const sv_super_op &op, std::vector<double> &abi, int *n_ops);
// A = V diag(w) V^dagger for a Hermitian n x n matrix (cyclic Jacobi).
void hermitian_eigen(std::vector<cd> A, int n, std::vector<double> &w, std::vector<cd> &V);

}  // namespace sv

struct sv_plan {
    int n = 0;
    int max_k = 0;
    int rule = 0;
    std::vector<sv::Block> blocks;
    // device-side cache (filled by the runtime when the plan is applied)
    void *cache = nullptr;
};
