// Launchers of the gfx950 kernels (device code lives in the *.hip files).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "common.h"

namespace sv {
namespace dev {

constexpr int kRedBlocks = 1024;  // fixed first-stage grid of every reduction
constexpr int kRedThreads = 256;

// ------------------------------------------------------------------ apply
// Register kernel: k <= 3 (k = 4 for complex64), canonical matrix (local bit
// j <-> sorted_q[j]).  Needs n >= 2 + (number of positions >= 2).
bool reg_supported(int dtype, int k, const int *sorted_q, int n);
// psi2 (optional): a second state of the same size and type that receives
// the same block in the same launch (gridDim.y = 2).
hipError_t launch_reg(int dtype, int k, const int *sorted_q, const cd *m, void *psi, int n,
                      hipStream_t st, int grid_cap, void *psi2 = nullptr);
// Generic kernel: k = 1..6, canonical matrix already on the device in the
// state's real type (interleaved re, im).
hipError_t launch_generic(int dtype, int k, const int *sorted_q, const void *d_m, void *psi, int n,
                          hipStream_t st, void *psi2 = nullptr);
// Dense-block MFMA kernels (complex64 state).  k = 4..6, n - k >= 5.
bool mfma_supported(int k, int n);
// FP32: d_a = real-form matrix (2^(k+1) x 2^(k+1) floats, see mfma.hip).
hipError_t launch_mfma_f32(int k, const int *sorted_q, const float *d_a, void *psi, int n,
                           hipStream_t st, int tc_log, int grid_cap, void *psi2 = nullptr);
// Split precision: d_parts[0..2] = the parts of the real-form matrix
// (pack_real_form_split) as BF16 (fp16 = false: three parts) or FP16 (fp16 =
// true: two parts, d_parts[2] unused) bit patterns.
hipError_t launch_mfma_split(int k, bool fp16, const int *sorted_q, const uint16_t *const *d_parts, void *psi,
                             int n, hipStream_t st, int tc_log, int grid_cap);
// Multi-block tile passes (complex64, FP32 or split BF16 / FP16 MFMA): up to
// tile_max_blocks() 4-qubit blocks whose positions have a union of at most
// tile_bits positions, applied in one HBM pass over tiles of
// 2^tile_bits amplitudes held by workgroups of `waves` waves; shapes
// (14, 8), (14, 16), (13, 4), (13, 8).  sub_pos rows ascending.  d_a = the
// blocks' operands (pack_tile_operand), back to back.  Needs n >= tile_bits.
constexpr int kMaxTileSubBlocks = kTilePassMaxBlocks;
constexpr int kMinTileQubits = 14;
constexpr int kMaxTileBits = 14;
constexpr int kMaxTileUnion = kMaxTileBits;
// Layout and blocks of one tile pass over one state.
struct TileArgs {
    uint64_t n_tiles;
    int ubit[kMaxTileBits];            // tile bit -> global position
    int ext_pos[SV_MAX_QUBITS_C64];    // positions outside the tile, ascending
    int n_ext;
    int n_sub;                         // blocks in this launch
    int tbit[kMaxTileSubBlocks][4];    // per block: its tile bits, ascending
    uint32_t swz[kMaxTileBits];        // LDS index of each tile bit (XOR-linear placement)
};
// Tile-pass operand of one 4-qubit block (canonical 16 x 16 matrix m), in
// kTileOperandWords 32-bit words: FP32: Re U then Im U (16 x 16 floats each,
// row-major); split BF16 (both BF16 codes): three parts of U (part p =
// RNE(U - parts before it)), split FP16: two parts, 256 words each, one word
// per entry holding (re, im) as 16-bit values (re in the low half); unused
// words are 0.  The precision codes are also the tile passes' arithmetic:
// kTileOperandBF16X3 splits the tile values into three parts instead of two.
constexpr int kTileOperandWords = 768;
constexpr int kTileOperandF32 = 0, kTileOperandBF16 = 1, kTileOperandF16 = 2, kTileOperandBF16X3 = 3;
void pack_tile_operand(const cd *m, int prec, uint32_t *out);
// Tile arguments of n_sub blocks (positions ascending per block) on an
// n-qubit state with 2^tile_bits-amplitude tiles, for a launch of `waves`
// waves in arithmetic `prec` (the LDS placement is chosen for them).
hipError_t make_tile_args(int n_sub, const int (*sub_pos)[4], int n, int tile_bits, int waves, int prec,
                          TileArgs *out);
// The pass's LDS placement (a.swz) for its blocks (a.tbit, a.n_sub), launch
// shape and arithmetic (placement.cpp; make_tile_args calls it).
void choose_tile_placement(TileArgs &a, int tile_bits, int waves, int prec);
// Extra LDS cycles (bank conflicts) that the placement of `a` leaves in the
// block loop of a split pass, by the bank model of choose_tile_placement; 0
// for FP32.
int tile_placement_conflicts(const TileArgs &a, int tile_bits, int waves, int prec);
// Batched passes (shape (kBatchTileBits, kBatchTileWaves), at most
// tile_max_blocks() blocks per pass, operands of precision `prec` as
// launch_tile_pass): pass p of
// state at complex offset state_off with its operands at pool + op_off
// (pack_tile_operand layout, kTileOperandWords each); each unit is one
// workgroup's tile range of one pass.
constexpr int kBatchTileBits = 14;
constexpr int kBatchTileWaves = 16;
struct TilePass {
    uint64_t state_off;  // complex elements from the start of the batch buffer
    uint64_t op_off;     // 32-bit words into the operand pool
    TileArgs args;
};
struct TileUnit {
    int32_t pass;
    int32_t pad;
    uint64_t t0, t1;     // tiles [t0, t1)
};
hipError_t launch_tile_batch(const TileUnit *units, int n_units, const TilePass *passes, const uint32_t *pool,
                             void *buf, hipStream_t st, int prec);
bool tile_supported(int n, int union_bits);
bool tile_shape_supported(int tile_bits, int waves);
int tile_wgs_per_cu(int tile_bits, int waves);
// Blocks one launch of the shape can hold with operands of precision prec
// (kTileOperand*; they sit in LDS: FP32 and FP16 operands are smaller than
// split BF16 ones, so more fit).
int tile_max_blocks(int tile_bits, int waves, int prec);
// The FP16 tile passes of one run and the state's norm, which their unitary
// blocks keep: the first pass (out) writes each workgroup's sum of squares of
// the values it reads, one double per workgroup of its grid; later passes
// (in, n_in = that grid) scale the whole pass by a power of two from the norm
// instead of scaling each tile from its largest magnitude.  Between such
// passes the state may stay in HBM times that scale: in_scaled = it is read
// that way (no scaling at copy-in), out_scaled = it is left that way (no
// unscaling at copy-out).  Every pass of the run has the same scale, and
// launches in between act on the scaled state linearly.
struct TileNorm {
    const double *in = nullptr;
    int n_in = 0;
    double *out = nullptr;
    int in_scaled = 0, out_scaled = 0;
    // >= 0 (FP32 and split FP16, one state): the pass reads nothing from
    // HBM; its input is the computational basis state |basis> (amplitude 1
    // there, 0 elsewhere), and it writes the whole state as any pass does.
    int64_t basis = -1;
};
// psi2 (optional): a second state of the same size that receives the same
// pass in the same launch (gridDim.y = 2).
// prec: kTileOperandF32, kTileOperandBF16, kTileOperandBF16X3 or
// kTileOperandF16 (FP16 passes scale each tile by a power of two chosen from
// its largest magnitude, or, with norm.in, the whole pass from the norm).
// norm: FP16 and one state only.  *grid_out (may be NULL) receives the
// number of workgroups launched.
hipError_t launch_tile_pass(int n_sub, const int (*sub_pos)[4], const void *d_a, int prec, void *psi, int n,
                            hipStream_t st, int grid_cap, int tile_bits, int waves, void *psi2 = nullptr,
                            const TileNorm &norm = TileNorm{}, int *grid_out = nullptr);
// Host-side packing of the MFMA operands of a canonical k-qubit matrix.
void pack_real_form_f32(const cd *m, int k, float *out);
// Split parts: part p = RNE(A' - parts before it), three for BF16, two for
// FP16 (parts[2] then all zero), real_form_elems(k) each.
void pack_real_form_split(const cd *m, int k, bool fp16, uint16_t *const *parts);
size_t real_form_elems(int k);

// ------------------------------------------------------------------ state init / copy
hipError_t launch_fill_basis(int dtype, void *psi, int n, uint64_t index, hipStream_t st);
// amps[4*p .. 4*p+3] = (re0, im0, re1, im1) of the one-qubit factor at position p
hipError_t launch_product(int dtype, void *psi, int n, const double *amps, hipStream_t st);
hipError_t launch_convert(int src_dtype, const void *src, int dst_dtype, void *dst, uint64_t count,
                          hipStream_t st);

// ------------------------------------------------------------------ reductions
// All write their FP64 result (1 or 2 doubles) to d_out, using d_partials
// (2 * kRedBlocks doubles) as the first-stage buffer.
hipError_t launch_norm(int dtype, const void *psi, int n, double *d_partials, double *d_out,
                       hipStream_t st);
hipError_t launch_inner(int dtype_a, const void *a, int dtype_b, const void *b, int n,
                        double *d_partials, double *d_out, hipStream_t st);
// Pauli terms grouped by x mask: group g covers terms [goff[g], goff[g+1]) all
// with x mask gx[g]; per term the z mask, the coefficient and the power of i
// (number of Y factors mod 4).  Device arrays.
struct PauliDev {
    int n_groups;
    const uint64_t *gx;
    const int32_t *goff;
    const uint64_t *tz;
    const double *tc;
    const int32_t *tpow;
};
hipError_t launch_pauli_expect(int dtype, const void *psi, int n, const PauliDev &H, double *d_partials,
                               double *d_out, hipStream_t st);
hipError_t launch_pauli_apply(int dtype, const void *psi, void *out, int n, const PauliDev &H,
                              hipStream_t st);
// Kraus channel for outcome weights: n_ops operators on k (1..3) ascending
// positions, 2^k x 2^k complex128 each in the canonical local order (bit j
// on pos[j]), back to back in device memory.
constexpr int kMaxKraus = 16;
struct KrausDev {
    int n_ops;
    int k;
    int pos[3];
    const double *m;
};
// p_i = ||K_i psi||^2 for i < n_ops into d_out[0..kMaxKraus) (FP64; d_partials
// holds kRedBlocks * kMaxKraus doubles).
hipError_t launch_kraus_probs(int dtype, const void *psi, int n, const KrausDev &K, double *d_partials,
                              double *d_out, hipStream_t st);
// Tr(rho H) of rho (n qubits) held row-major in a state of 2n qubits.
hipError_t launch_dm_expect(int dtype, const void *rho, int n, const PauliDev &H, double *d_partials, double *d_out,
                            hipStream_t st);

// ------------------------------------------------------------------ adjoint
// One backward step for a k <= 2 gate: if pauli >= 1 (1 = X, 2 = Y, 3 = Z on
// sorted_q[0]), d_partials[slot * kRedBlocks + block] receives the block's
// partial of <lam|P|phi> (re, im: 2 doubles per block); then phi <- U^+ phi and
// lam <- U^+ lam, U^+ given canonically in `mdag`.
hipError_t launch_backward_step(int dtype, int k, const int *sorted_q, const cd *mdag, int pauli,
                                void *phi, void *lam, int n, double *d_partials, int slot,
                                hipStream_t st);
// For Pauli strings t < n_terms (x/z masks, pw = power of i), partials of
// <lam|P_t|phi> into slots slot0 + t (same layout as above).  One pass.
constexpr int kMaxGradTerms = 16;
hipError_t launch_grad_terms(int dtype, int n_terms, const uint64_t *x, const uint64_t *z, const int *pw,
                             const void *phi, const void *lam, int n, double *d_partials, int slot0, hipStream_t st);
// out[s] = sum over blocks of d_partials[s][*] (fixed order), s < n_slots.
hipError_t launch_sum_partials(const double *d_partials, int n_slots, double *d_out, hipStream_t st);

// ------------------------------------------------------------------ batches
struct BatchTables;  // defined in batch.hip
}  // namespace dev
}  // namespace sv
