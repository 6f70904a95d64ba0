/*
 * sv.h -- C ABI of the MI355X (gfx950) state-vector library.
 *
 * The library evolves a 2^n-amplitude complex state by an ordered list of
 * gates, each applied to the amplitude groups it touches, or by gates greedily
 * fused into dense k-qubit blocks.  This is the "evolution" method of the
 * HybridQ paper (Simulations section, State Vector subsection: the state vector
 * is updated by one matrix-vector product per gate; Circuit utilities: compress()
 * fuses gates into blocks of at most max_n_qubits qubits).
 *
 * General conventions
 *   - Every entry point returns SV_OK (0) or a negative SV_ERR_* code; the
 *     thread-local message of the last failure is sv_last_error().  No C++
 *     exception crosses this boundary.
 *   - Arguments are validated on the host before any device work is enqueued:
 *     a call that fails validation has no effect.
 *   - Device work is asynchronous on the state's HIP stream unless an entry
 *     point says it synchronises.  An asynchronous device fault is reported as
 *     SV_ERR_HIP by the next synchronising call.
 *   - Qubits are POSITIONS: position p is bit p of an amplitude index (position
 *     0 = least significant bit).  The paper's (2,)*n arrays with axis j
 *     following order[j] in C order put order[0] at position n-1 (its Grover
 *     example fixes this).
 *   - A k-qubit matrix is 2^k x 2^k complex128, row-major, each entry stored as
 *     (re, im) doubles; the most significant bit of its local index belongs to
 *     q[0].
 *   - States are interleaved complex arrays (re, im), complex64 (SV_C64) or
 *     complex128 (SV_C128), in caller-owned device memory (for example a torch
 *     tensor) or in memory the library allocates.
 *   - A state handle, plan or batch is used from one host thread at a time.
 */
#ifndef SV_H
#define SV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SV_MAX_K 6            /* largest gate / fused block, in qubits        */
#define SV_MAX_QUBITS_C64 35  /* 256 GiB of complex64 amplitudes              */
#define SV_MAX_QUBITS_C128 34 /* 256 GiB of complex128 amplitudes             */
#define SV_MAX_PAULI_TERMS 4096

/* status codes */
#define SV_OK 0
#define SV_ERR_ARG (-1)         /* bad argument (NULL, out of range, bad enum) */
#define SV_ERR_QUBIT (-2)       /* qubit position out of range or repeated     */
#define SV_ERR_SIZE (-3)        /* buffer too small for the requested state    */
#define SV_ERR_HIP (-4)         /* HIP runtime error (message has details)     */
#define SV_ERR_UNSUPPORTED (-5) /* valid request this build cannot serve       */

/* amplitude types */
#define SV_C64 0
#define SV_C128 1

/* arithmetic used to apply fused blocks (sv_run_opts.precision) */
#define SV_PREC_FP32 0       /* complex64 state; FP32 matvec / FP32 MFMA           */
#define SV_PREC_SPLIT_BF16 1 /* complex64 state; k>=4 blocks as hi+lo BF16 MFMA    */
#define SV_PREC_SPLIT_FP16 2 /* complex64 state; k>=4 blocks as hi+lo FP16 MFMA;   */
                             /* MATRIX gates must be unitary (to 1e-6), else       */
                             /* SV_ERR_ARG: tile passes rely on norm-preserving    */
                             /* blocks                                             */
#define SV_PREC_FP64 3       /* complex128 state; FP64 arithmetic throughout       */
#define SV_PREC_SPLIT_BF16X3 4 /* complex64 state; tile passes as BF16 MFMA with   */
                               /* the tile values in three parts as well (six    */
                               /* products, about FP32's accuracy); other blocks */
                               /* as SV_PREC_FP32                                */

/* fusion rules (sv_fuse) */
#define SV_RULE_PAPER 0    /* the paper's compress() rule, reproduced exactly    */
#define SV_RULE_ENHANCED 1 /* paper rule, then cost-aware merging of blocks      */
#define SV_RULE_NONE 2     /* one block per gate (plain per-gate application)    */
#define SV_RULE_TILED 3    /* enhanced blocks of <= 4 qubits, grouped into LDS   */
                           /* tile passes (see sv_run_circuit)                   */
#define SV_RULE_AUTO 4     /* the cheaper of ENHANCED and TILED plans, and its k, */
                           /* by the autotuned cost table (see sv_run_circuit)    */

/* gate kinds.  Matrices (paper, Gates and Properties section, names only; the
 * matrices are the textbook ones):
 *   SQRT_P = ((1+i) I + (1-i) P) / 2 for P in {X, Y, W}, W = (X + Y)/sqrt 2
 *   R_P(t) = cos(t/2) I - i sin(t/2) P                      (params[0] = t)
 *   CZ = diag(1,1,1,-1); CPHASE(a) = diag(1,1,1,e^{ia})     (params[0] = a)
 *   CX: control q[0], target q[1];  SWAP
 *   FSIM(t, f) = [[1,0,0,0],[0,cos t,-i sin t,0],[0,-i sin t,cos t,0],
 *                 [0,0,0,e^{-if}]]                           (params = t, f)
 *   MATRIX: the caller's dense matrix in sv_gate.m (k = 1..SV_MAX_K). */
enum sv_gate_kind {
    SV_G_MATRIX = 0,
    SV_G_I = 1,
    SV_G_X = 2,
    SV_G_Y = 3,
    SV_G_Z = 4,
    SV_G_H = 5,
    SV_G_SQRT_X = 6,
    SV_G_SQRT_Y = 7,
    SV_G_SQRT_W = 8,
    SV_G_RX = 9,
    SV_G_RY = 10,
    SV_G_RZ = 11,
    SV_G_CZ = 12,
    SV_G_CX = 13,
    SV_G_CPHASE = 14,
    SV_G_SWAP = 15,
    SV_G_FSIM = 16,
    SV_G_COUNT = 17
};

/* One gate of a circuit (paper, Circuits section: a circuit is an ordered list
 * of gates acting on qubits).  k must equal the kind's arity (1 or 2) except for
 * SV_G_MATRIX.  `param` is the index of params[0] in the parameter vector that
 * sv_backward differentiates (rotations only), or -1.  The matrix behind `m`
 * is read during the call and not retained. */
typedef struct sv_gate {
    int32_t kind;
    int32_t k;
    int32_t q[SV_MAX_K];
    double params[2];
    int32_t param;
    int32_t reserved; /* must be 0 */
    const double *m;
} sv_gate;

/* Real linear combination of Pauli strings H = sum_t coef[t] P_t.  Bit p of
 * xmask[t] is set when P_t has X or Y at position p, bit p of zmask[t] when it
 * has Z or Y there (Y = i X Z).  Host arrays of n_terms entries. */
typedef struct sv_pauli_sum {
    int32_t n_terms;
    int32_t reserved; /* must be 0 */
    const double *coef;
    const uint64_t *xmask;
    const uint64_t *zmask;
} sv_pauli_sum;

/* Options of sv_run_circuit. */
typedef struct sv_run_opts {
    int32_t max_k;     /* largest fused block, 1..SV_MAX_K; -1 = choose the
                          value with the lowest cost in the autotuned table   */
    int32_t precision; /* SV_PREC_*; must match the state's amplitude type    */
    int32_t rule;      /* SV_RULE_*                                           */
    int32_t use_graph; /* 1: run the launches as one hipGraph, kept per state */
} sv_run_opts;

typedef struct sv_state sv_state;
typedef struct sv_plan sv_plan;
typedef struct sv_batch sv_batch;

/* ---------------------------------------------------------------- misc */
/* Message of the last failing call on this thread ("" if none). */
const char *sv_last_error(void);
/* ABI version (monotone integer). */
int sv_version(void);

/* ---------------------------------------------------------------- states */
/* Bind a handle to an n-qubit state of amplitude type `dtype` (SV_C64 or
 * SV_C128) held in `dev_buf` (device memory of at least 2^n amplitudes,
 * 256-byte aligned; the caller keeps it alive until sv_free and keeps
 * ownership).  dev_buf == NULL makes the library allocate (and later free) the
 * buffer.  `hip_stream` (a hipStream_t, may be NULL = default stream) is the
 * stream every call on this state enqueues on.  The state starts as |0...0>
 * (paper, Initial and Final State Specification section).
 * Errors: SV_ERR_ARG (n < 1, n above SV_MAX_QUBITS_*, bad dtype, out NULL,
 * misaligned buffer), SV_ERR_SIZE (bytes < 2^n amplitudes), SV_ERR_HIP. */
int sv_alloc(int n, int dtype, void *dev_buf, size_t bytes, void *hip_stream, sv_state **out);
/* Release the handle (and the buffer if the library allocated it). Synchronises. */
int sv_free(sv_state *s);
/* Query the handle: qubit count, amplitude type, device pointer. */
int sv_info(const sv_state *s, int *n, int *dtype, void **dev_ptr);
/* Product state from tokens '0' '1' '+' '-' (paper, Initial and Final State
 * Specification section): either n characters, token j describing position
 * n-1-j, or one character broadcast to every qubit.  SV_ERR_ARG otherwise. */
int sv_set_product(sv_state *s, const char *tokens);
/* Computational basis state |index>.  SV_ERR_ARG if index >= 2^n. */
int sv_set_basis(sv_state *s, uint64_t index);
/* Copy amplitudes [first, first+count) to host memory (in the state's own
 * amplitude type).  Synchronises.  SV_ERR_ARG if the range exceeds 2^n. */
int sv_read(sv_state *s, uint64_t first, uint64_t count, void *host);
/* Copy amplitudes from host memory into [first, first+count).  Synchronises.
 * Together with sv_read this checkpoints and resumes a long circuit. */
int sv_write(sv_state *s, uint64_t first, uint64_t count, const void *host);
/* dst <- src amplitude by amplitude (types may differ: complex64 <-> complex128).
 * Both states must have the same n.  Enqueued on dst's stream after src's work. */
int sv_copy(sv_state *dst, sv_state *src);
/* Wait for all work enqueued on the state's stream. */
int sv_synchronize(sv_state *s);

/* ---------------------------------------------------------------- gates */
/* Host only: write the 2^k x 2^k complex128 matrix of gate g into `out`
 * (row-major, (re, im) pairs).  Validates kind, k and parameters but not qubit
 * positions. */
int sv_gate_matrix(const sv_gate *g, double *out);
/* Apply one gate to the state (the paper's per-gate matrix-vector product,
 * State Vector section).  k <= 3 runs the register kernel, k >= 4 the dense
 * block kernels.  complex64 states use FP32 arithmetic, complex128 FP64.
 * Errors: SV_ERR_QUBIT (position >= n or repeated), SV_ERR_ARG. */
int sv_apply_gate(sv_state *s, const sv_gate *g);

/* ---------------------------------------------------------------- fusion */
/* Host only.  Partition the G gates into blocks of at most max_k qubits
 * (paper, Circuit utilities section, compress()).  SV_RULE_PAPER: each gate
 * joins the last block that shares a qubit with it if the union stays within
 * max_k qubits, otherwise it opens a new block.  SV_RULE_ENHANCED: the paper
 * rule, then a gate that meets no block joins the last block when that fits,
 * and adjacent-by-commutation blocks are merged whenever the autotuned cost
 * table (or, without one, the pass count) says the merged block is cheaper.
 * SV_RULE_NONE: one block per gate.  SV_RULE_TILED: the enhanced rule with
 * blocks of at most min(max_k, 4) qubits.  SV_RULE_AUTO: see sv_run_circuit
 * (the plan records the rule and k it chose).  Each block's qubits are sorted
 * ascending (q[0] = most significant local bit) and its matrix is the ordered
 * product of its members (FP64).  n bounds the positions.  max_k = -1 uses the
 * autotuned cost table for n (SV_ERR_ARG if there is none).
 * The plan is owned by the caller and released with sv_plan_free. */
int sv_fuse(const sv_gate *g, int G, int n, int max_k, int rule, sv_plan **out);
/* sv_fuse for a run in `precision` (SV_PREC_*): the plan sv_run_circuit forms
 * with that precision.  The tiled rule then fills each pass up to what one
 * launch holds with that precision's operands (7 blocks for SV_PREC_FP32 and
 * SV_PREC_SPLIT_FP16 at (14, *), 5 for the split BF16 forms; sv_fuse plans
 * for the split BF16 capacity, which every precision takes), and
 * SV_RULE_AUTO and max_k = -1 use
 * that precision's cost table (sv_fuse: FP32's).  A plan applied in another
 * precision stays correct: a pass of more blocks than one launch holds runs
 * as several launches.  SV_ERR_ARG for an unknown precision. */
int sv_fuse_prec(const sv_gate *g, int G, int n, int max_k, int rule, int precision, sv_plan **out);
int sv_plan_free(sv_plan *p);
/* Number of blocks; for block b: its size k, its positions q[0..k-1] (array of
 * SV_MAX_K) and its member count. */
int sv_plan_num_blocks(const sv_plan *p, int *out);
int sv_plan_block(const sv_plan *p, int b, int32_t *k, int32_t *q, int32_t *n_members);
/* Indices (into the fused gate list) of block b's members, in order. */
int sv_plan_block_members(const sv_plan *p, int b, int32_t *members);
/* Block b's 2^k x 2^k complex128 matrix. */
int sv_plan_block_matrix(const sv_plan *p, int b, double *m);
/* The max_k the plan was built with (the chosen one when -1 was asked). */
int sv_plan_max_k(const sv_plan *p, int *out);
/* The rule the plan was built with (the chosen one for SV_RULE_AUTO). */
int sv_plan_rule(const sv_plan *p, int *out);
/* Tile pass of block b (SV_RULE_TILED plans): consecutive blocks with the same
 * pass number >= 0 are applied together in one read and one write of the
 * state; -1 means the block is applied on its own. */
int sv_plan_block_pass(const sv_plan *p, int b, int32_t *pass);
/* Apply a plan's blocks in order with the given SV_PREC_* arithmetic.  With
 * use_graph = 1 the launches are captured into a hipGraph and launched as one;
 * the state keeps the instantiated graph, and a later call whose launches have
 * the same structure (block positions, kernels, launch shapes; the matrices
 * may differ, as when angles change) updates it in place
 * (hipGraphExecUpdate) instead of instantiating a new one.  Asynchronous in
 * both modes.  SV_ERR_QUBIT if the plan's positions do not fit the state. */
int sv_apply_plan(sv_state *s, const sv_plan *p, int precision, int use_graph);

/* ---------------------------------------------------------------- circuits */
/* Validate the G gates, fuse them (sv_fuse with o->max_k, o->rule) and apply
 * the blocks in order (paper, Simulations section: simulate(..., optimize=
 * 'evolution')).  Nothing is applied if any gate is invalid.  Asynchronous
 * (use_graph as for sv_apply_plan).  o == NULL means plain per-gate
 * application: {SV_MAX_K, FP32 or FP64 by amplitude type, SV_RULE_NONE, 0}.
 * With SV_RULE_TILED on a complex64 state of >= 14 qubits, the gates are
 * grouped into passes whose positions U leave contiguous HBM runs no shorter
 * than those of a union of sv_set_tile_union() positions (default 10): the
 * tile of a pass is U plus the lowest positions outside it, 14 (or 13) in
 * all, and its runs, 2^r amplitudes with r its lowest positions 0, 1, .. in
 * a row, must hold at least 2^(tile bits - limit); so every union of <= 10
 * positions qualifies, and up to 14 when U holds the lowest positions.  Each
 * pass is fused into blocks of <= 4 qubits
 * (gates move only where every qubit keeps its own gate order).  Each tile
 * of 2^14 (or 2^13) amplitudes is staged in LDS once, every block of the
 * pass is applied to it (SV_PREC_FP32: FP32 MFMA; SV_PREC_SPLIT_BF16 /
 * SV_PREC_SPLIT_FP16: hi+lo 16-bit MFMA, the FP16 values scaled by a power of
 * two, chosen per tile from its largest magnitude in the call's first FP16
 * pass and per pass from the state's norm, which that pass measures, in the
 * later ones, between which the state stays in HBM times that one scale
 * until the call's last FP16 pass; SV_PREC_SPLIT_BF16X3: BF16 MFMA on three
 * parts of each value), and the tile is written back, so a pass costs one
 * read and one write of the state.  The state is plain again when the
 * call's launches end (asynchronously, like the call).  A
 * block left alone runs as a one-block pass where the cost table prices
 * that lower.
 * SV_RULE_AUTO (with max_k = -1, or max_k as an upper bound) evaluates the
 * enhanced plans for every k and the tiled plans for k <= 4 on block
 * positions only, prices each with the cost table of (n, precision) (from
 * sv_autotune, or relative defaults), and fuses the cheapest. */
int sv_run_circuit(sv_state *s, const sv_gate *g, int G, const sv_run_opts *o);
/* sv_set_basis(s, basis) followed by sv_run_circuit(s, g, G, o) (paper,
 * Simulations section: simulate with a computational-basis initial state),
 * as one call: when the plan starts with an FP32 or split-FP16 tile pass,
 * that pass produces the basis state itself and reads nothing from HBM (the
 * state's earlier contents are not read; no fill runs); otherwise the state
 * is filled first.
 * The result is the same as the two calls'.  Nothing is changed if any gate
 * is invalid.  Asynchronous.  SV_ERR_ARG for basis >= 2^n. */
int sv_run_circuit_basis(sv_state *s, uint64_t basis, const sv_gate *g, int G, const sv_run_opts *o);

/* ---------------------------------------------------------------- reductions */
/* ||psi||^2 in FP64 (fixed-order two-stage reduction).  Synchronises. */
int sv_norm(sv_state *s, double *out);
/* <a|b> = sum_i conj(a_i) b_i in FP64; a and b have the same n, any types.
 * Synchronises (enqueued on b's stream after a's work). */
int sv_inner(sv_state *a, sv_state *b, double *re, double *im);
/* <psi|H|psi> for a Pauli sum H, FP64 accumulation.  Synchronises.
 * SV_ERR_ARG if a mask has bits at or above n or too many terms. */
int sv_expectation(sv_state *s, const sv_pauli_sum *H, double *out);
/* For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the value of
 * sv_expectation for the n-qubit state of amplitude type dtype (SV_C64 or
 * SV_C128) held in dev_psi (device memory of the current device, 2^n
 * amplitudes, 256-byte aligned, owned by the caller), computed on hip_stream
 * (NULL = default stream) by the same kernels.  The call allocates nothing:
 * the term tables and reduction partials live in a fixed 192 KiB array that
 * each GPU holds until the process ends; every call on a GPU reuses it, so
 * calls that overlap on one GPU (from several host threads or streams) race
 * and the library serialises them.  Synchronises.  Errors: SV_ERR_ARG (NULL,
 * bad n, dtype or alignment, malformed sum), SV_ERR_QUBIT (a mask at or above
 * bit n), SV_ERR_SIZE (tables larger than the array; cannot happen within
 * SV_MAX_PAULI_TERMS terms), SV_ERR_HIP. */
int sv_expectation_noalloc(const void *dev_psi, int n, int dtype, void *hip_stream, const sv_pauli_sum *H,
                           double *out);
/* psi <- H psi for a Pauli sum H (into `out`, a second state of the same n
 * and type; psi is unchanged).  Asynchronous. */
int sv_apply_pauli_sum(sv_state *psi, const sv_pauli_sum *H, sv_state *out);

/* ---------------------------------------------------------------- gradients */
/* Adjoint differentiation of E(theta) = <psi|H|psi>, psi = U_G..U_1 psi_0
 * (the paper is silent on gradients; method: adjoint differentiation, Jones &
 * Gacon 2020).  `psi` must hold the forward output of exactly these gates and
 * is consumed (it ends as U_1^+ .. U_G^+ psi, i.e. psi_0 up to rounding);
 * `scratch` is a second state of the same n and type (lam = H psi, then swept
 * back with psi: two buffers, no stored trajectory).  For every gate with
 * param >= 0 (which must be SV_G_RX, SV_G_RY or SV_G_RZ),
 * grad[param] += dE/dtheta = Im <lam|P|phi>, accumulated in FP64; other
 * entries are untouched, so the caller zeroes grad first.  A run of
 * consecutive rotations on distinct qubits shares one gradient pass (they
 * commute); runs of other gates are undone as fused dagger blocks.
 * Synchronises.  Errors: SV_ERR_ARG (param >= n_params, a param on a
 * non-rotation). */
int sv_backward(sv_state *psi, sv_state *scratch, const sv_gate *g, int G, const sv_pauli_sum *H,
                double *grad, int n_params);
/* sv_backward with the undoing of the gate runs in `precision` (SV_PREC_*,
 * as for sv_run_circuit: split FP16 needs unitary MATRIX gates and scales
 * each tile of either state by a power of two from its own largest
 * magnitude).  sv_backward is this call with FP32 (complex64) or FP64
 * (complex128).  Errors as sv_backward, and SV_ERR_ARG for a precision the
 * state's amplitude type does not take. */
int sv_backward_prec(sv_state *psi, sv_state *scratch, const sv_gate *g, int G, const sv_pauli_sum *H,
                     double *grad, int n_params, int precision);

/* ---------------------------------------------------------- density matrices */
/* Density-matrix evolution by the state-vector path (paper, Simulations
 * section: the density-matrix entry point rewrites a super circuit as a
 * regular circuit and simulates that).  The density matrix rho of n qubits is a
 * state of 2n qubits holding rho row-major, as kron(psi, conj(psi)) lays out a
 * pure state (the paper's State Vector section example): amplitude
 * r * 2^n + c holds rho[r][c], so the row index sits on positions n..2n-1 and
 * the column index on positions 0..n-1.  Qubit q of rho is position q + n of
 * the row index and position q of the column index.  A gate U on qubits Q
 * becomes U on Q + n and conj(U) on Q; a super operator becomes one dense gate
 * on the 2k positions (Q + n, Q).
 *
 * A super operator on k = 1..3 qubits q[0..k-1] (q[0] the most significant bit
 * of its local index, as for gates) is either
 *   - a KrausSuperGate (paper, Gates and Properties section):
 *       rho -> sum_ij s[i][j] L_i rho R_j^dagger,
 *     n_left matrices L_i and n_right matrices R_j (2^k x 2^k complex each,
 *     row-major, re/im interleaved, back to back), s an n_left x n_right
 *     complex matrix (row-major, interleaved) or NULL for the identity (then
 *     n_left == n_right: the Kraus channel sum_i K_i rho K_i^dagger when
 *     left == right); or
 *   - a MatrixSuperGate: `superop` is the 4^k x 4^k complex matrix acting on
 *     the row-major vectorisation of the k-qubit rho (local index r 2^k + c),
 *     with n_left = n_right = 0 and left = right = s = NULL.
 * It acts after the first `after` gates of the circuit's gate list (0..G;
 * operators with equal `after` act in array order, and `after` must not
 * decrease along the array).  Matrices are read during the call and not
 * retained. */
typedef struct sv_super_op {
    int32_t after;
    int32_t k;
    int32_t q[3];
    int32_t n_left;
    int32_t n_right;
    int32_t reserved; /* must be 0 */
    const double *left;
    const double *right;
    const double *s;
    const double *superop;
} sv_super_op;

/* The 4^k x 4^k matrix of a super operator on the row-major vectorisation of
 * its k-qubit rho: sum_ij s[i][j] kron(L_i, conj(R_j)), or `superop` itself.
 * Host only.  out: 2 * 16^k doubles (row-major, interleaved).  SV_ERR_ARG on a
 * malformed operator. */
int sv_super_op_matrix(const sv_super_op *op, double *out);

/* Evolve the density matrix held in rho (2n qubits, see above) by the G gates
 * g (on qubits 0..n-1) with the n_ops super operators inserted among them,
 * fused and applied exactly as sv_run_circuit applies a circuit of 2n qubits
 * (same options; a max_k other than -1 must be at least 2k for the largest
 * super operator, whose gate spans 2k positions).  Start from |0..0><0..0|
 * with sv_set_basis(rho, 0).
 * SV_PREC_SPLIT_FP16 is refused (SV_ERR_ARG): its tile passes rely on blocks
 * that cannot raise the 2-norm, which super operators may.  Errors:
 * SV_ERR_ARG (odd rho->n, malformed operator, `after` out of order),
 * SV_ERR_QUBIT (a qubit >= n or repeated). */
int sv_dm_run(sv_state *rho, const sv_gate *g, int G, const sv_super_op *ops, int n_ops, const sv_run_opts *o);

/* Tr(rho H) = sum_t coef[t] Re Tr(rho P_t) for a Pauli sum over the n qubits of
 * rho (masks below bit n), summed in FP64 in a fixed order: Tr(rho P) is the
 * sum over a of omega(a) rho[a][a ^ x], with P|a> = omega(a)|a ^ x>.
 * Synchronises.  An identity term (x = z = 0) gives the trace. */
int sv_dm_expectation(sv_state *rho, const sv_pauli_sum *H, double *out);

/* ------------------------------------------ Kraus channels sampled on states */
/* Pure-state sampling of Kraus channels (paper, Simulations with noise
 * section: noise is simulated exactly on density matrices or by sampling the
 * Kraus operators on pure states).  The operator must be a KrausSuperGate
 * whose right operators equal its left ones (n_left = n_right, at most 64,
 * superop = NULL), either in Kraus form (s = NULL): the channel sum_i K_i rho
 * K_i^dagger, or with a Hermitian positive semidefinite s (a GlobalPauliChannel
 * with a general s, for example), which is first turned into its Kraus form
 * as sv_kraus_form does.  Its qubits index the state directly (`after` is
 * used only by sv_run_trajectory).  Outcome i has weight p_i = ||K_i psi||^2,
 * which depends on the state (amplitude damping, for example).
 *
 * sv_kraus_probabilities: p_out[i] = ||K_i psi||^2 for the operators K_i of
 * the Kraus form (n_left of them when s = NULL, the rank of s otherwise, in
 * the order sv_kraus_form gives; the other of the n_left entries are set to
 * 0), summed in FP64 in one pass over the state per 16 operators.
 * Synchronises.
 *
 * sv_apply_kraus_sampled: with S = sum_i p_i, picks the first operator with a
 * nonzero weight whose running sum exceeds u * S (u in [0, 1), drawn by the
 * caller) and replaces psi by K_i psi / sqrt(p_i).  chosen (may be NULL)
 * receives i, p_chosen (may be NULL) p_i / S.  Synchronises.
 *
 * sv_run_trajectory: applies the gates g with the operators ops sampled among
 * them (operator j after the first ops[j].after gates, `after`
 * nondecreasing) using uniforms[j]; the gate runs between operators are fused
 * and applied as by sv_run_circuit with options o.  outcomes (may be NULL)
 * receives the n_ops chosen indices.
 *
 * Errors: SV_ERR_ARG (not a Kraus channel, more than 16 operators, u outside
 * [0, 1), all weights zero), SV_ERR_QUBIT. */
int sv_kraus_probabilities(sv_state *s, const sv_super_op *op, double *p_out);
int sv_apply_kraus_sampled(sv_state *s, const sv_super_op *op, double u, int32_t *chosen, double *p_chosen);
int sv_run_trajectory(sv_state *s, const sv_gate *g, int G, const sv_super_op *ops, int n_ops,
                      const double *uniforms, const sv_run_opts *o, int32_t *outcomes);

/* ------------------------------------------------------------ noise channels */
/* The channels of the paper's Noisy gates section as KrausSuperGates.  Each
 * call fills `out` (with the given `after`) and writes the operators
 * (2^k x 2^k complex matrices, row-major, (re, im) interleaved, back to back)
 * into the caller's `mats`, which out->left and out->right point to; the
 * caller keeps `mats` (and `s`) alive while `out` is used.  Except for
 * sv_channel_pauli the result is in Kraus form (s = NULL), so it serves
 * sv_dm_run and the sampled entry points alike.  The paper's Local versions
 * (noise applied independently to each qubit) are one single-qubit channel
 * per qubit, in any order (they act on different qubits and commute).
 *
 * sv_channel_depolarizing: rho -> (1 - p) rho + p I/d on the k = 1..3 qubits
 * q (d = 2^k, p in [0, 1]), as the identity with weight 1 - p + p/d^2 and the
 * other d^2 - 1 Pauli strings with weight p/d^2, K = sqrt(weight) P.  mats:
 * 4^k matrices (2 * 16^k doubles).
 *
 * sv_channel_dephasing: rho -> (1 - p) rho + p sigma rho sigma on one qubit,
 * sigma = X, Y or Z (pauli = 1, 2 or 3), p in [0, 1].  mats: 2 matrices (16
 * doubles).
 *
 * sv_channel_amplitude_damping: K0 = sqrt(1 - beta)|0><0| + sqrt(1 - gamma)
 * |1><1|, K1 = sqrt(gamma)|0><1| and, for an excitation rate beta > 0, K2 =
 * sqrt(beta)|1><0| (gamma, beta in [0, 1]).  beta = 0 gives the paper's two
 * operators; beta > 0 the generalized channel with |1> -> |0> at rate gamma and
 * |0> -> |1> at rate beta.  mats: room for 3 matrices (24 doubles);
 * out->n_left is 2 or 3.
 *
 * sv_channel_pauli: the GlobalPauliChannel rho -> sum_ij s_ij sigma_i rho
 * sigma_j on the k = 1..3 qubits q: left = right = the 4^k Pauli strings,
 * string i = sum_j i_j 4^(k-1-j) with i_j in {0, 1, 2, 3} = {I, X, Y, Z}
 * acting on q[j], and out->s = s, the caller's 4^k x 4^k complex matrix
 * (row-major, interleaved).  mats: 4^k matrices.
 *
 * sv_kraus_form: the Kraus form sum_m K_m rho K_m^dagger of a KrausSuperGate
 * sum_ij s_ij L_i rho L_j^dagger whose right operators equal its left ones
 * and whose s is NULL (the operators are copied) or Hermitian positive
 * semidefinite (to 1e-12 relative): with s = V diag(lambda) V^dagger (FP64
 * Jacobi eigendecomposition), K_m = sqrt(lambda_m) sum_i V_im L_i for every
 * lambda_m above 1e-14 times the largest.  mats: room for n_left matrices;
 * out (may alias in) receives the Kraus form and its operator count.
 *
 * Errors: SV_ERR_ARG (NULL, parameters out of range, k outside 1..3, s not
 * Hermitian or not positive semidefinite, right != left), SV_ERR_QUBIT
 * (negative or repeated qubit). */
int sv_channel_depolarizing(int k, const int32_t *q, double p, int after, double *mats, sv_super_op *out);
int sv_channel_dephasing(int qubit, int pauli, double p, int after, double *mats, sv_super_op *out);
int sv_channel_amplitude_damping(int qubit, double gamma, double beta, int after, double *mats, sv_super_op *out);
int sv_channel_pauli(int k, const int32_t *q, const double *s, int after, double *mats, sv_super_op *out);
int sv_kraus_form(const sv_super_op *in, double *mats, sv_super_op *out);

/* ---------------------------------------------------------------- batches */
/* Many independent circuits of different qubit counts (noisy trajectories:
 * the paper's Simulations with noise section samples noise channels on pure
 * states instead of evolving density matrices).  Trajectory t has n_qubits[t]
 * qubits (1..SV_MAX_QUBITS_C64) and gates [gate_offsets[t], gate_offsets[t+1])
 * of `gates`; every state starts at |0...0>.  Noise draws are already
 * materialised as gates by the caller. */
typedef struct sv_batch_desc {
    int32_t n_traj;
    int32_t max_k;          /* fusion limit per trajectory (1..SV_MAX_K) or -1 */
    const int32_t *n_qubits;
    const int64_t *gate_offsets; /* n_traj + 1 entries */
    const sv_gate *gates;
    int32_t precision;      /* SV_PREC_FP32 (0), SV_PREC_SPLIT_BF16,
                               SV_PREC_SPLIT_FP16 or SV_PREC_SPLIT_BF16X3:
                               the arithmetic of the tile
                               passes of trajectories with 14 or more qubits;
                               smaller ones and all reductions stay FP32 / FP64 */
} sv_batch_desc;
/* Device bytes sv_batch_create needs in dev_buf for this batch. */
int sv_batch_required_bytes(const sv_batch_desc *d, size_t *out);
/* Fuse every trajectory, upload the work tables and build the launch
 * schedule on `hip_stream`.  dev_buf (caller-owned, >= required bytes) holds
 * every trajectory's complex64 state back to back. */
int sv_batch_create(const sv_batch_desc *d, void *dev_buf, size_t bytes, void *hip_stream,
                    sv_batch **out);
/* Run every trajectory from |0...0> and write <Z_0> (FP64) of each into
 * z0_out[n_traj].  use_graph = 1 replays one captured hipGraph.  Synchronises. */
int sv_batch_run(sv_batch *b, int use_graph, double *z0_out);
/* Read amplitudes of trajectory t (after sv_batch_run).  Synchronises. */
int sv_batch_read(sv_batch *b, int t, uint64_t first, uint64_t count, void *host);
int sv_batch_free(sv_batch *b);

/* ---------------------------------------------------------------- tuning */
/* Time the block kernels for k = 1..SV_MAX_K (and their launch shapes) on
 * the given scratch state (its contents are destroyed) with SV_PREC_*
 * arithmetic, keep the fastest launch shape per k, and store the cost table
 * (milliseconds per block application, cost_ms[k], cost_ms[0] unused) for
 * this (n, precision).  Synchronises. */
int sv_autotune(sv_state *scratch, int precision, double *cost_ms);
/* Install a cost table for (n, precision) without timing. */
int sv_set_cost_table(int n, int precision, const double *cost_ms);
/* Tuning cache.  When the environment variable SV_TUNE_CACHE names a file,
 * every successful sv_autotune records there, under the key (GPU architecture,
 * e.g. gfx950; n; precision), the cost table of every block size k (and of
 * tile passes of 1..16 blocks) and the launch shapes it chose, replacing the
 * older record of that key; the first sv_alloc of the process installs the
 * records of the current device's architecture.  sv_tune_cache_load installs
 * them from `path` (NULL: SV_TUNE_CACHE) on demand; the launch shapes come
 * from the file's last matching record.  *loaded (may be NULL) receives the
 * number of records installed.  Errors: SV_ERR_ARG (no path, unreadable
 * file), SV_ERR_HIP. */
int sv_tune_cache_load(const char *path, int *loaded);
/* Select the launch shape of the multi-block tile passes (SV_RULE_TILED):
 * tiles of 2^tile_bits amplitudes held in LDS by workgroups of `waves`
 * 64-lane waves.  Supported: (14, 8) and (14, 16), one 128 KiB tile per
 * compute unit; (13, 4), two 64 KiB workgroups per compute unit; (13, 8).
 * A launch holds at most 5 blocks ((14, *)), 2 ((13, 4)) or 15 ((13, 8))
 * with split BF16 operands, and 7, 3 or 16 with the smaller FP32 and split
 * FP16 ones; the tiled rule plans passes of at most that many blocks for the
 * run's precision (the gates of a further block go to the next pass).
 * sv_autotune
 * picks one itself; this call overrides it for the whole process (later
 * launches on every state).  SV_ERR_ARG for other pairs. */
int sv_set_tile_shape(int tile_bits, int waves);
/* The current launch shape of the tile passes and the number of blocks one
 * launch of it holds with split BF16 operands, the fewest of any precision
 * (pointers may be NULL). */
int sv_get_tile_shape(int *tile_bits, int *waves, int *max_blocks);
/* Layout of one tile pass of n_sub 4-qubit blocks (sub_pos: 4 ascending
 * positions per block, n_sub rows) on an n-qubit complex64 state, as the
 * tile passes lay it out for launch shape (tile_bits, waves) and tile
 * arithmetic `precision` (SV_PREC_FP32, _SPLIT_BF16, _SPLIT_FP16 or
 * _SPLIT_BF16X3).  Host
 * only: no device work.  tile_pos[b] (tile_bits entries) receives the state
 * position of tile bit b: the blocks' union, then the lowest positions
 * outside it, ascending.  lds_image[b] receives where tile bit b lands in
 * the tile's LDS copy: tile index i sits at LDS index XOR of lds_image[b]
 * over the set bits b of i, a permutation of 0 .. 2^tile_bits - 1 that keeps
 * bit 0; it is chosen per pass so that the 16-byte LDS accesses of the
 * blocks hit distinct banks.  *conflicts (may be NULL) receives the extra
 * LDS cycles left by that choice (0 when it is free of bank conflicts; 0
 * for FP32).  Errors: SV_ERR_ARG. */
int sv_tile_placement(int n_sub, const int32_t *sub_pos, int n, int tile_bits, int waves, int precision,
                      int32_t *tile_pos, uint32_t *lds_image, int32_t *conflicts);
/* Union limit of the passes that SV_RULE_TILED plans (8..10; default 10,
 * or the SV_TILE_UNION environment variable at load time): every pass's tile
 * is made of contiguous HBM runs of at least 2^(tile_bits - limit)
 * amplitudes, the runs a union of `limit` positions leaves.  A larger limit
 * holds more gates per pass but allows shorter runs.  Applies to later
 * sv_fuse / sv_run_circuit calls in the process.  SV_ERR_ARG outside
 * 8..10. */
int sv_set_tile_union(int max_positions);

/* ----------------------------------- projections, measurement and control */
/* Non-unitary and controlled operations (paper, Gates and Properties section:
 * Projection(state, qubits), Measure(qubits), Control(c_qubits, gate); the
 * Grover Oracle section builds its oracle as psi - 2 P psi with P the
 * projection on |0..0>).
 *
 * sv_project: psi -> P psi with P = |bits><bits| on the k (1..SV_MAX_K) qubits
 * q (q[0] the most significant bit of bits); *prob (may be NULL) receives
 * ||P psi||^2 (FP64); renormalize != 0 then divides by sqrt(prob)
 * (SV_ERR_ARG if prob is 0, the state then being left at P psi = 0).
 * Synchronises.
 *
 * sv_measure: measures the k qubits q one after another, qubit q[j] with the
 * caller's uniform uniforms[j] in [0, 1) by the rule of
 * sv_apply_kraus_sampled on {|0><0|, |1><1|} (outcome 0 when u < p_0 / (p_0 +
 * p_1)); the state collapses and is renormalised.  *bits (q[0] most
 * significant) and *prob (the probability of the outcome) may be NULL.
 * Synchronises.
 *
 * sv_controlled_gate (host): the gate g controlled by the n_c qubits controls
 * (acting when all are 1), as a MATRIX gate on (controls..., g's qubits) with
 * the controls as the most significant local bits, n_c + g->k <= SV_MAX_K.
 * m_out (2 * 4^(n_c + k) doubles) receives its matrix, which out->m points
 * to; the caller keeps it alive while the gate is used.
 *
 * Errors: SV_ERR_ARG, SV_ERR_QUBIT. */
int sv_project(sv_state *s, int k, const int32_t *q, uint64_t bits, int renormalize, double *prob);
int sv_measure(sv_state *s, int k, const int32_t *q, const double *uniforms, uint64_t *bits, double *prob);
int sv_controlled_gate(const sv_gate *g, int n_c, const int32_t *controls, sv_gate *out, double *m_out);

/* ------------------------------------------------------- circuit utilities */
/* Host-only cuts applied before fusion (paper, Circuits section, Circuit
 * utilities: pop, which removes gates outside the light cone of pinned qubits
 * from either side of the circuit, and simplify).  Both write the indices of
 * the gates to keep, ascending, into keep (room for G entries) and their count
 * into n_keep; the kept gates are applied in the original order.
 *
 * sv_lightcone (pop): direction SV_POP_RIGHT walks backwards from the end: a
 * gate touching the light cone of the `pinned` qubits (bit p = position p) is
 * kept and adds its qubits to the cone; others are dropped.  Exact for
 * expectations <O> of any observable O on the pinned qubits, from any initial
 * state (the dropped gates commute with O and with every later kept gate).
 * SV_POP_LEFT is the same walk forwards from the start (the right walk of the
 * inverted circuit): the circuit equals K D, K the kept gates and D the
 * dropped ones, which act only on unpinned qubits and commute with every
 * earlier kept gate; so the kept gates give the same output state whenever D
 * leaves the input unchanged (inputs rho_pinned (x) sigma with sigma
 * maximally mixed, or invariant under D).  Errors: SV_ERR_ARG (bad direction),
 * SV_ERR_QUBIT.
 *
 * sv_compact_qubits: renames the qubits that the G gates touch, plus the
 * pinned ones, to positions 0 .. n_used - 1 in ascending order of their old
 * positions: out[i] is g[i] on the new positions (matrix pointers shared),
 * pos_map[p] (n entries) the new position of old position p or -1.  Run on
 * the kept gates of a light cone, it moves a circuit onto the cone's qubits.
 * From a product initial state, every expectation on the kept qubits is
 * unchanged: an untouched qubit keeps its own product factor.  Errors:
 * SV_ERR_ARG, SV_ERR_QUBIT.
 *
 * sv_simplify: drops gates equal to the identity and pairs (a, b), b after a
 * on the same qubits with b a = I, when every kept gate between them commutes
 * with a: through disjoint qubits, or, if use_matrix_commutation != 0, through
 * commuting matrices (tested on unions of at most 10 qubits); repeated until
 * nothing changes.  Entries compare with absolute tolerance 1e-12.  The kept
 * gates have the same product as the circuit.  Errors: SV_ERR_ARG,
 * SV_ERR_QUBIT. */
#define SV_POP_RIGHT 0
#define SV_POP_LEFT 1
int sv_lightcone(const sv_gate *g, int G, int n, uint64_t pinned, int direction, int32_t *keep, int *n_keep);
int sv_compact_qubits(const sv_gate *g, int G, int n, uint64_t pinned, sv_gate *out, int32_t *pos_map, int *n_used);
int sv_simplify(const sv_gate *g, int G, int n, int use_matrix_commutation, int32_t *keep, int *n_keep);

/* ---------------------------------------------------------- measurement */
/* The achievable rate of one state pass: `reps` streaming read + write passes
 * over the complex64 state (n >= 14; every value is written back where it was
 * read, so the state is unchanged) in tiles of 2^14 amplitudes spanned by
 * the 14 positions set in tile_positions (position 0 among them), the HBM
 * layout of a tile pass with those tile positions, with no LDS staging and no
 * block work.  Positions 0..13 give whole 128 KiB runs; 0..3 with the top ten
 * positions the 128-byte runs of a pass over the highest positions.  One
 * workgroup per compute unit, as the tile passes.  *ms_per_pass receives the
 * mean device milliseconds per pass (HIP events on the state's stream).
 * Synchronises.  Errors: SV_ERR_ARG, SV_ERR_QUBIT, SV_ERR_HIP. */
int sv_stream_probe(sv_state *s, uint64_t tile_positions, int reps, double *ms_per_pass);

/* ---------------------------------------------------------------- stats */
/* Per-kernel device timing.  While enabled every kernel launch is bracketed
 * by HIP events on its stream; sv_stats_query synchronises the recorded
 * launches and returns, for a kernel class, the launch count and the summed
 * device milliseconds.  Classes: 100*family + k, families 1 = register
 * apply, 2 = generic apply, 3 = MFMA FP32, 4 = MFMA split BF16, 5 = MFMA split
 * FP16, 6 = reductions, 7 = adjoint, 8 = batch, 9 = FP32 tile passes, 10 =
 * split-BF16 tile passes, 11 = split-FP16 tile passes; k is the block size,
 * for tile passes the number of blocks in the launch, and for reductions 1 =
 * norm, 2 = inner product, 3 = expectation, 4 = Pauli-sum matvec, 5 =
 * density-matrix trace Tr(rho H), 6 = Kraus outcome weights. */
int sv_stats_enable(int on);
/* Graph runs of a state (use_graph = 1 calls): their count and how many of
 * them reused the state's instantiated graph (updated in place). */
int sv_graph_stats(const sv_state *s, int64_t *runs, int64_t *reused);
int sv_stats_reset(void);
int sv_stats_query(int cls, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif
#endif /* SV_H */
