// Density matrices as states of 2n qubits (paper, Simulations section: the
// density-matrix entry point rewrites a super circuit as a regular circuit
// and simulates that; KrausSuperGate and MatrixSuperGate of the Gates and
// Properties section).
//
// rho is held row-major: amplitude r * 2^n + c is rho[r][c], the layout of
// kron(psi, conj(psi)) for a pure state.  The row-major vectorisation obeys
// vec(A rho B) = kron(A, B^T) vec(rho), so
//   gate U:                 rho -> U rho U^dagger  = kron(U, conj(U)) vec(rho),
//   super operator:         rho -> sum_ij s_ij L_i rho R_j^dagger
//                                = sum_ij s_ij kron(L_i, conj(R_j)) vec(rho).
// Qubit q of rho is position q + n of the row index and position q of the
// column index, so U acts on positions Q + n and conj(U) on Q, and a super
// operator is one gate on the 2k positions (Q + n, Q) whose local index is
// r 2^k + c (row bits most significant).
#include <cmath>
#include <cstring>

#include "common.h"

namespace sv {

namespace {

int check_super_op(const sv_super_op &op)
{
    if (op.reserved != 0) return fail(SV_ERR_ARG, "sv_super_op.reserved must be 0");
    if (op.k < 1 || op.k > 3) return fail(SV_ERR_ARG, "super operator on %d qubits (1..3)", op.k);
    const size_t D = size_t(1) << op.k;
    auto finite = [](const double *p, size_t count) {
        for (size_t i = 0; i < count; ++i)
            if (!std::isfinite(p[i])) return false;
        return true;
    };
    if (op.superop) {
        if (op.n_left || op.n_right || op.left || op.right || op.s)
            return fail(SV_ERR_ARG, "a matrix super operator takes no left/right/s operands");
        if (!finite(op.superop, 2 * D * D * D * D)) return fail(SV_ERR_ARG, "non-finite super operator entry");
        return SV_OK;
    }
    if (op.n_left < 1 || op.n_right < 1 || op.n_left > 64 || op.n_right > 64)
        return fail(SV_ERR_ARG, "super operator with %d left and %d right operators (1..64 each)", op.n_left,
                    op.n_right);
    if (!op.left || !op.right) return fail(SV_ERR_ARG, "NULL left or right operators");
    if (!op.s && op.n_left != op.n_right)
        return fail(SV_ERR_ARG, "s = NULL (identity) needs n_left == n_right, got %d and %d", op.n_left, op.n_right);
    if (!finite(op.left, 2 * D * D * op.n_left) || !finite(op.right, 2 * D * D * op.n_right))
        return fail(SV_ERR_ARG, "non-finite operator entry");
    if (op.s && !finite(op.s, 2 * size_t(op.n_left) * op.n_right)) return fail(SV_ERR_ARG, "non-finite s entry");
    return SV_OK;
}

// 4^k x 4^k matrix (row-major) of a checked super operator.
void super_matrix(const sv_super_op &op, std::vector<cd> &S)
{
    const size_t D = size_t(1) << op.k, DD = D * D;
    S.assign(DD * DD, cd(0));
    if (op.superop) {
        for (size_t i = 0; i < DD * DD; ++i) S[i] = cd(op.superop[2 * i], op.superop[2 * i + 1]);
        return;
    }
    auto L = [&](int i, size_t a, size_t b) {
        const double *p = op.left + 2 * (DD * i + a * D + b);
        return cd(p[0], p[1]);
    };
    auto R = [&](int j, size_t a, size_t b) {
        const double *p = op.right + 2 * (DD * j + a * D + b);
        return cd(p[0], p[1]);
    };
    for (int i = 0; i < op.n_left; ++i)
        for (int j = 0; j < op.n_right; ++j) {
            cd s = op.s ? cd(op.s[2 * (size_t(i) * op.n_right + j)], op.s[2 * (size_t(i) * op.n_right + j) + 1])
                        : cd(i == j ? 1.0 : 0.0);
            if (s == cd(0)) continue;
            // S[(r, c)][(r', c')] += s L_i[r][r'] conj(R_j[c][c'])
            for (size_t r = 0; r < D; ++r)
                for (size_t c = 0; c < D; ++c)
                    for (size_t r2 = 0; r2 < D; ++r2) {
                        const cd lr = s * L(i, r, r2);
                        if (lr == cd(0)) continue;
                        cd *row = &S[(r * D + c) * DD + r2 * D];
                        for (size_t c2 = 0; c2 < D; ++c2) row[c2] += lr * std::conj(R(j, c, c2));
                    }
        }
}

}  // namespace

// Rewrite the super circuit (gates g with super operators ops among them) as a
// regular circuit on 2n positions.  Matrices of the new MATRIX gates live in
// `store` (one vector per gate, never reallocated after the gates point at it).
int dm_expand(const sv_gate *g, int G, int n, const sv_super_op *ops, int n_ops, std::vector<sv_gate> &out,
              std::vector<std::vector<double>> &store)
{
    if (G < 0 || n_ops < 0) return fail(SV_ERR_ARG, "negative gate or operator count");
    if ((G && !g) || (n_ops && !ops)) return fail(SV_ERR_ARG, "NULL gate or operator array");
    for (int j = 0; j < n_ops; ++j) {
        if (int rc = check_super_op(ops[j])) return rc;
        for (int a = 0; a < ops[j].k; ++a) {
            if (ops[j].q[a] < 0 || ops[j].q[a] >= n)
                return fail(SV_ERR_QUBIT, "super operator %d: qubit %d outside 0..%d", j, ops[j].q[a], n - 1);
            for (int b = 0; b < a; ++b)
                if (ops[j].q[a] == ops[j].q[b]) return fail(SV_ERR_QUBIT, "super operator %d: qubit repeated", j);
        }
        if (ops[j].after < 0 || ops[j].after > G || (j && ops[j].after < ops[j - 1].after))
            return fail(SV_ERR_ARG, "super operator %d: after = %d out of order (0..%d, nondecreasing)", j,
                        ops[j].after, G);
    }
    out.clear();
    store.clear();
    store.reserve(size_t(G) + n_ops);
    out.reserve(2 * size_t(G) + n_ops);
    int next_op = 0;
    auto emit_ops_until = [&](int after) {
        for (; next_op < n_ops && ops[next_op].after <= after; ++next_op) {
            const sv_super_op &op = ops[next_op];
            std::vector<cd> S;
            super_matrix(op, S);
            store.emplace_back(2 * S.size());
            std::memcpy(store.back().data(), S.data(), sizeof(cd) * S.size());
            sv_gate h{};
            h.kind = SV_G_MATRIX;
            h.k = 2 * op.k;
            for (int a = 0; a < op.k; ++a) {
                h.q[a] = op.q[a] + n;
                h.q[op.k + a] = op.q[a];
            }
            h.param = -1;
            h.m = store.back().data();
            out.push_back(h);
        }
    };
    for (int i = 0; i < G; ++i) {
        emit_ops_until(i);
        std::vector<cd> U;
        if (int rc = gate_matrix_abi(g[i], U)) return rc;
        if (int rc = check_gate_qubits(g[i], n)) return rc;
        sv_gate row = g[i];  // U on the row positions
        for (int a = 0; a < row.k; ++a) row.q[a] += n;
        row.param = -1;
        out.push_back(row);
        store.emplace_back(2 * U.size());
        for (size_t e = 0; e < U.size(); ++e) {
            store.back()[2 * e] = U[e].real();
            store.back()[2 * e + 1] = -U[e].imag();
        }
        sv_gate col{};  // conj(U) on the column positions
        col.kind = SV_G_MATRIX;
        col.k = g[i].k;
        for (int a = 0; a < col.k; ++a) col.q[a] = g[i].q[a];
        col.param = -1;
        col.m = store.back().data();
        out.push_back(col);
    }
    emit_ops_until(G);
    return SV_OK;
}

// A Kraus channel sum_i K_i rho K_i^dagger for sampling on pure states: a
// KrausSuperGate on qubits below n in Kraus form (s = NULL) or with a
// Hermitian positive semidefinite s (turned into Kraus form, kraus_form),
// right == left, at most kMaxKrausOps operators.  Fills the ABI-order and the
// canonical matrices (local bit j on the j-th lowest position), their count
// and the sorted positions.
int kraus_canonical(const sv_super_op &op, int n, KrausSet &out)
{
    if (int rc = check_super_op(op)) return rc;
    if (op.superop) return fail(SV_ERR_ARG, "sampling needs a Kraus channel, not a matrix super operator");
    if (int rc = kraus_form(op, out.abi, &out.n_ops)) return rc;
    if (out.n_ops > kMaxKrausOps) return fail(SV_ERR_ARG, "%d Kraus operators (at most %d)", out.n_ops, kMaxKrausOps);
    const size_t D = size_t(1) << op.k;
    sv_gate h{};
    h.kind = SV_G_MATRIX;
    h.k = op.k;
    h.param = -1;
    for (int a = 0; a < op.k; ++a) h.q[a] = op.q[a];
    if (int rc = check_gate_qubits(h, n)) return rc;
    out.k = op.k;
    for (int a = 0; a < 3; ++a) out.q[a] = a < op.k ? op.q[a] : 0;
    out.canon.clear();
    for (int i = 0; i < out.n_ops; ++i) {
        h.m = out.abi.data() + 2 * D * D * i;
        std::vector<cd> m;
        if (int rc = gate_matrix_canonical(h, m, out.sorted_q)) return rc;
        out.canon.insert(out.canon.end(), m.begin(), m.end());
    }
    return SV_OK;
}

}  // namespace sv

extern "C" int sv_super_op_matrix(const sv_super_op *op, double *out)
{
    sv::clear_error();
    if (!op || !out) return sv::fail(SV_ERR_ARG, "NULL argument");
    if (int rc = sv::check_super_op(*op)) return rc;
    std::vector<sv::cd> S;
    sv::super_matrix(*op, S);
    std::memcpy(out, S.data(), sizeof(sv::cd) * S.size());
    return SV_OK;
}
