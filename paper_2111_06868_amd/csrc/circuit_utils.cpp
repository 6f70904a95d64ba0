// Host circuit utilities that cut work before fusion (paper, Circuits section,
// Circuit utilities: pop removes gates outside the light cone of pinned
// qubits; simplify removes gates that cancel, optionally using the gates'
// matrices to decide whether two gates commute).
#include <algorithm>
#include <cmath>

#include "common.h"

namespace sv {

namespace {

uint64_t qubit_mask(const sv_gate &g)
{
    uint64_t m = 0;
    for (int j = 0; j < g.k; ++j) m |= uint64_t(1) << g.q[j];
    return m;
}

// Matrix of gate g embedded on the positions listed in `pos` (ascending, a
// superset of g's qubits): local bit b of the result <-> pos[b].
void embed(const sv_gate &g, const std::vector<cd> &M, const std::vector<int> &pos, std::vector<cd> &out)
{
    const int u = int(pos.size()), k = g.k;
    const size_t D = size_t(1) << u, d = size_t(1) << k;
    int where[SV_MAX_K];  // gate qubit j (q[0] most significant local bit) -> bit in the embedding
    for (int j = 0; j < k; ++j) where[j] = int(std::find(pos.begin(), pos.end(), g.q[j]) - pos.begin());
    uint64_t gmask = 0;
    for (int j = 0; j < k; ++j) gmask |= uint64_t(1) << where[j];
    auto local = [&](size_t x) {
        size_t m = 0;
        for (int j = 0; j < k; ++j) m |= ((x >> where[j]) & 1) << (k - 1 - j);
        return m;
    };
    out.assign(D * D, cd(0));
    for (size_t r = 0; r < D; ++r)
        for (size_t c = 0; c < D; ++c)
            if ((r & ~gmask) == (c & ~gmask)) out[r * D + c] = M[local(r) * d + local(c)];
}

std::vector<int> union_positions(const sv_gate &a, const sv_gate &b)
{
    std::vector<int> p;
    for (int j = 0; j < a.k; ++j) p.push_back(a.q[j]);
    for (int j = 0; j < b.k; ++j)
        if (std::find(p.begin(), p.end(), b.q[j]) == p.end()) p.push_back(b.q[j]);
    std::sort(p.begin(), p.end());
    return p;
}

void matmul(const std::vector<cd> &A, const std::vector<cd> &B, size_t D, std::vector<cd> &C)
{
    C.assign(D * D, cd(0));
    for (size_t i = 0; i < D; ++i)
        for (size_t l = 0; l < D; ++l) {
            const cd a = A[i * D + l];
            if (a == cd(0)) continue;
            for (size_t j = 0; j < D; ++j) C[i * D + j] += a * B[l * D + j];
        }
}

constexpr double kAtol = 1e-12;
constexpr int kMaxCommuteUnion = 10;  // largest union for a matrix commutation test

struct GateInfo {
    uint64_t mask;
    std::vector<cd> m;  // ABI-order matrix
};

bool commute(const sv_gate &a, const GateInfo &ia, const sv_gate &b, const GateInfo &ib, bool use_matrix)
{
    if (!(ia.mask & ib.mask)) return true;
    if (!use_matrix) return false;
    const std::vector<int> pos = union_positions(a, b);
    if (int(pos.size()) > kMaxCommuteUnion) return false;
    const size_t D = size_t(1) << pos.size();
    std::vector<cd> A, B, AB, BA;
    embed(a, ia.m, pos, A);
    embed(b, ib.m, pos, B);
    matmul(A, B, D, AB);
    matmul(B, A, D, BA);
    for (size_t i = 0; i < D * D; ++i)
        if (std::abs(AB[i] - BA[i]) > kAtol) return false;
    return true;
}

// b a == identity on their common qubits (same qubit set required)
bool cancel(const sv_gate &a, const GateInfo &ia, const sv_gate &b, const GateInfo &ib)
{
    if (ia.mask != ib.mask) return false;
    const std::vector<int> pos = union_positions(a, b);
    const size_t D = size_t(1) << pos.size();
    std::vector<cd> A, B, P;
    embed(a, ia.m, pos, A);
    embed(b, ib.m, pos, B);
    matmul(B, A, D, P);
    for (size_t i = 0; i < D; ++i)
        for (size_t j = 0; j < D; ++j)
            if (std::abs(P[i * D + j] - cd(i == j ? 1.0 : 0.0)) > kAtol) return false;
    return true;
}

bool is_identity(const GateInfo &ig, int k)
{
    const size_t d = size_t(1) << k;
    for (size_t i = 0; i < d; ++i)
        for (size_t j = 0; j < d; ++j)
            if (std::abs(ig.m[i * d + j] - cd(i == j ? 1.0 : 0.0)) > kAtol) return false;
    return true;
}

}  // namespace

}  // namespace sv

// Light cone (pop).  SV_POP_RIGHT walks from the end of the circuit: the cone
// starts as the pinned qubits; a gate that touches the cone is kept and adds
// its qubits, any other gate is dropped.  A dropped gate acts only on qubits
// outside the cone of every later kept gate, so it commutes with all of them
// and with any observable on the pinned qubits, and cancels in
// <psi| U^dagger O U |psi>.  SV_POP_LEFT is the same walk from the start: a
// dropped gate is disjoint from every earlier kept gate and from the pinned
// qubits, so U = K D with K the kept gates and D the dropped ones, acting on
// the other qubits only; the pinned qubits' influence (U (rho_pinned (x)
// sigma) U^dagger for any sigma that D leaves unchanged, e.g. I/2^m) needs K
// only.  It is the right walk of the inverted circuit.
extern "C" int sv_lightcone(const sv_gate *g, int G, int n, uint64_t pinned, int direction, int32_t *keep,
                            int *n_keep)
{
    sv::clear_error();
    if (!keep || !n_keep) return sv::fail(SV_ERR_ARG, "NULL output");
    if (n < 1 || n > 64) return sv::fail(SV_ERR_ARG, "n = %d outside 1..64", n);
    if (direction != SV_POP_RIGHT && direction != SV_POP_LEFT)
        return sv::fail(SV_ERR_ARG, "direction %d (SV_POP_RIGHT or SV_POP_LEFT)", direction);
    if (n < 64 && (pinned >> n)) return sv::fail(SV_ERR_QUBIT, "pinned qubits beyond qubit %d", n - 1);
    if (G < 0 || (G && !g)) return sv::fail(SV_ERR_ARG, "bad gate array");
    for (int i = 0; i < G; ++i) {
        int rc = sv::check_gate_shape(g[i]);
        if (!rc) rc = sv::check_gate_qubits(g[i], n);
        if (rc) return rc;
    }
    uint64_t cone = pinned;
    std::vector<int32_t> kept;
    const bool right = direction == SV_POP_RIGHT;
    for (int t = 0; t < G; ++t) {
        const int i = right ? G - 1 - t : t;
        const uint64_t m = sv::qubit_mask(g[i]);
        if (m & cone) {
            cone |= m;
            kept.push_back(i);
        }
    }
    if (right) std::reverse(kept.begin(), kept.end());
    std::copy(kept.begin(), kept.end(), keep);
    *n_keep = int(kept.size());
    return SV_OK;
}

// Compaction: the qubits that the gates touch, plus the pinned ones, renamed
// to positions 0, 1, .. in ascending order of their old positions.  A qubit
// that no gate touches keeps its initial product factor, which drops out of
// every reduced state of the others.
extern "C" int sv_compact_qubits(const sv_gate *g, int G, int n, uint64_t pinned, sv_gate *out, int32_t *pos_map,
                                 int *n_used)
{
    sv::clear_error();
    if (!pos_map || !n_used || (G && !out)) return sv::fail(SV_ERR_ARG, "NULL output");
    if (n < 1 || n > 64) return sv::fail(SV_ERR_ARG, "n = %d outside 1..64", n);
    if (n < 64 && (pinned >> n)) return sv::fail(SV_ERR_QUBIT, "pinned qubits beyond qubit %d", n - 1);
    if (G < 0 || (G && !g)) return sv::fail(SV_ERR_ARG, "bad gate array");
    uint64_t used = pinned;
    for (int i = 0; i < G; ++i) {
        int rc = sv::check_gate_shape(g[i]);
        if (!rc) rc = sv::check_gate_qubits(g[i], n);
        if (rc) return rc;
        used |= sv::qubit_mask(g[i]);
    }
    int next = 0;
    for (int p = 0; p < n; ++p) pos_map[p] = ((used >> p) & 1) ? next++ : -1;
    for (int i = 0; i < G; ++i) {
        out[i] = g[i];
        for (int j = 0; j < g[i].k; ++j) out[i].q[j] = pos_map[g[i].q[j]];
    }
    *n_used = next;
    return SV_OK;
}

// Simplify: drop gates equal to the identity, and pairs (a, b) with b a = I
// on the same qubits when every kept gate between them commutes with a
// (disjoint qubits, or, with use_matrix_commutation, commuting matrices on a
// union of at most 10 qubits).  Repeated until nothing changes.  The kept
// gates, in order, have the same product as the circuit (to 1e-12 per entry
// of each cancelled product).
extern "C" int sv_simplify(const sv_gate *g, int G, int n, int use_matrix_commutation, int32_t *keep, int *n_keep)
{
    sv::clear_error();
    if (!keep || !n_keep) return sv::fail(SV_ERR_ARG, "NULL output");
    if (n < 1 || n > 64) return sv::fail(SV_ERR_ARG, "n = %d outside 1..64", n);
    if (G < 0 || (G && !g)) return sv::fail(SV_ERR_ARG, "bad gate array");
    std::vector<sv::GateInfo> info(G);
    for (int i = 0; i < G; ++i) {
        int rc = sv::check_gate_shape(g[i]);
        if (!rc) rc = sv::check_gate_qubits(g[i], n);
        if (!rc) rc = sv::gate_matrix_abi(g[i], info[i].m);
        if (rc) return rc;
        info[i].mask = sv::qubit_mask(g[i]);
    }
    const bool use_m = use_matrix_commutation != 0;
    std::vector<char> alive(G, 1);
    for (bool changed = true; changed;) {
        changed = false;
        for (int i = 0; i < G; ++i) {
            if (!alive[i]) continue;
            if (sv::is_identity(info[i], g[i].k)) {
                alive[i] = 0;
                changed = true;
                continue;
            }
            for (int j = i + 1; j < G; ++j) {
                if (!alive[j]) continue;
                if (sv::cancel(g[i], info[i], g[j], info[j])) {
                    alive[i] = alive[j] = 0;
                    changed = true;
                    break;
                }
                if (!sv::commute(g[i], info[i], g[j], info[j], use_m)) break;
            }
        }
    }
    int c = 0;
    for (int i = 0; i < G; ++i)
        if (alive[i]) keep[c++] = i;
    *n_keep = c;
    return SV_OK;
}
