// Noise channels of the paper's Noisy gates section (global and local Pauli
// channels, depolarizing, dephasing, amplitude damping with an optional
// excitation rate), written as Kraus super operators, and the Kraus form of a
// KrausSuperGate whose s matrix is Hermitian positive semidefinite (the form
// that pure-state sampling needs).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "common.h"

namespace sv {

namespace {

constexpr double kHermTol = 1e-12;  // relative: s Hermitian and PSD to this
constexpr double kDropTol = 1e-14;  // relative: eigenvalues kept as Kraus operators

// 2 x 2 Paulis I, X, Y, Z (row-major)
const cd kPauli[4][4] = {{1, 0, 0, 1}, {0, 1, 1, 0}, {0, cd(0, -1), cd(0, 1), 0}, {1, 0, 0, -1}};

// Pauli string `idx` (digit j, base 4 most significant first, acts on local
// qubit j, i.e. local bit k-1-j) as a 2^k x 2^k matrix in ABI order.
void pauli_string(int k, int idx, cd *out)
{
    const size_t D = size_t(1) << k;
    int digit[3];
    for (int j = k - 1; j >= 0; --j) {
        digit[j] = idx & 3;
        idx >>= 2;
    }
    for (size_t r = 0; r < D; ++r)
        for (size_t c = 0; c < D; ++c) {
            cd v = 1.0;
            for (int j = 0; j < k; ++j) {
                const int br = int(r >> (k - 1 - j)) & 1, bc = int(c >> (k - 1 - j)) & 1;
                v *= kPauli[digit[j]][2 * br + bc];
            }
            out[r * D + c] = v;
        }
}

void put(double *mats, size_t index, size_t D, const cd *m, double scale)
{
    for (size_t e = 0; e < D * D; ++e) {
        mats[2 * (index * D * D + e)] = scale * m[e].real();
        mats[2 * (index * D * D + e) + 1] = scale * m[e].imag();
    }
}

int check_qubits(int k, const int32_t *q)
{
    if (k < 1 || k > 3) return fail(SV_ERR_ARG, "channel on %d qubits (1..3)", k);
    if (!q) return fail(SV_ERR_ARG, "NULL qubit list");
    for (int a = 0; a < k; ++a) {
        if (q[a] < 0) return fail(SV_ERR_QUBIT, "negative qubit %d", q[a]);
        for (int b = 0; b < a; ++b)
            if (q[a] == q[b]) return fail(SV_ERR_QUBIT, "qubit %d repeated", q[a]);
    }
    return SV_OK;
}

void kraus_out(int k, const int32_t *q, int n_ops, int after, const double *mats, sv_super_op *out)
{
    std::memset(out, 0, sizeof *out);
    out->after = after;
    out->k = k;
    for (int a = 0; a < k; ++a) out->q[a] = q[a];
    out->n_left = out->n_right = n_ops;
    out->left = out->right = mats;
}

bool probability(double p) { return p >= 0.0 && p <= 1.0; }

}  // namespace

// Eigen-decomposition of the Hermitian n x n matrix A (row-major) by cyclic
// complex Jacobi rotations: A = V diag(w) V^dagger, V unitary (column m is
// the eigenvector of w[m]).  Each rotation first turns the (p, q) entry real
// by a phase on column q, then annihilates it with a real plane rotation.
void hermitian_eigen(std::vector<cd> A, int n, std::vector<double> &w, std::vector<cd> &V)
{
    V.assign(size_t(n) * n, cd(0));
    for (int i = 0; i < n; ++i) V[size_t(i) * n + i] = 1.0;
    auto at = [&](int r, int c) -> cd & { return A[size_t(r) * n + c]; };
    double scale = 0.0;
    for (const cd &x : A) scale = std::max(scale, std::abs(x));
    for (int sweep = 0; sweep < 100 && scale > 0.0; ++sweep) {
        double off = 0.0;
        for (int r = 0; r < n; ++r)
            for (int c = r + 1; c < n; ++c) off = std::max(off, std::abs(at(r, c)));
        if (off <= 1e-16 * scale) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                const cd b = at(p, q);
                const double ab = std::abs(b);
                if (ab <= 1e-300) continue;
                const cd ph = b / ab;  // e^{i phi}
                const double alpha = at(p, p).real(), gamma = at(q, q).real();
                const double theta = (gamma - alpha) / (2.0 * ab);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (std::abs(theta) + std::sqrt(theta * theta + 1.0));
                const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
                // U = diag(1, conj(ph)) [[c, s], [-s, c]]: A <- U^dagger A U, V <- V U
                const cd u00 = c, u01 = s, u10 = -s * std::conj(ph), u11 = c * std::conj(ph);
                for (int r = 0; r < n; ++r) {  // columns p, q
                    const cd ap = at(r, p), aq = at(r, q);
                    at(r, p) = ap * u00 + aq * u10;
                    at(r, q) = ap * u01 + aq * u11;
                    const cd vp = V[size_t(r) * n + p], vq = V[size_t(r) * n + q];
                    V[size_t(r) * n + p] = vp * u00 + vq * u10;
                    V[size_t(r) * n + q] = vp * u01 + vq * u11;
                }
                for (int c2 = 0; c2 < n; ++c2) {  // rows p, q
                    const cd ap = at(p, c2), aq = at(q, c2);
                    at(p, c2) = std::conj(u00) * ap + std::conj(u10) * aq;
                    at(q, c2) = std::conj(u01) * ap + std::conj(u11) * aq;
                }
                at(p, q) = at(q, p) = 0.0;
                at(p, p) = at(p, p).real();
                at(q, q) = at(q, q).real();
            }
    }
    w.resize(n);
    for (int i = 0; i < n; ++i) w[i] = at(i, i).real();
}

// Kraus form of a checked KrausSuperGate (no matrix form): with s = NULL the
// left operators themselves; otherwise right must equal left and s must be
// Hermitian PSD; then K_m = sqrt(lambda_m) sum_i V_im L_i.  abi receives
// n_ops matrices (ABI order, interleaved doubles).
int kraus_form(const sv_super_op &op, std::vector<double> &abi, int *n_ops)
{
    const size_t D = size_t(1) << op.k, DD = D * D;
    if (op.superop) return fail(SV_ERR_ARG, "a matrix super operator has no Kraus form here");
    if (op.n_left != op.n_right || std::memcmp(op.left, op.right, sizeof(double) * 2 * DD * op.n_left) != 0)
        return fail(SV_ERR_ARG, "the Kraus form needs right operators equal to the left ones");
    const int L = op.n_left;
    if (!op.s) {
        abi.assign(op.left, op.left + 2 * DD * L);
        *n_ops = L;
        return SV_OK;
    }
    std::vector<cd> S(size_t(L) * L);
    double smax = 0.0;
    for (size_t e = 0; e < S.size(); ++e) {
        S[e] = cd(op.s[2 * e], op.s[2 * e + 1]);
        smax = std::max(smax, std::abs(S[e]));
    }
    for (int i = 0; i < L; ++i)
        for (int j = 0; j <= i; ++j)
            if (std::abs(S[size_t(i) * L + j] - std::conj(S[size_t(j) * L + i])) > kHermTol * std::max(smax, 1.0))
                return fail(SV_ERR_ARG, "s is not Hermitian (entries %d,%d and %d,%d)", i, j, j, i);
    std::vector<double> w;
    std::vector<cd> V;
    hermitian_eigen(S, L, w, V);
    const double wmax = w.empty() ? 0.0 : *std::max_element(w.begin(), w.end());
    abi.clear();
    int count = 0;
    for (int m = 0; m < L; ++m) {
        if (w[m] < -kHermTol * std::max(wmax, 1.0))
            return fail(SV_ERR_ARG, "s is not positive semidefinite (eigenvalue %g)", w[m]);
        if (!(w[m] > kDropTol * wmax)) continue;
        const double r = std::sqrt(w[m]);
        const size_t base = abi.size();
        abi.resize(base + 2 * DD, 0.0);
        for (int i = 0; i < L; ++i) {
            const cd c = r * V[size_t(i) * L + m];
            if (c == cd(0)) continue;
            for (size_t e = 0; e < DD; ++e) {
                const cd x = c * cd(op.left[2 * (DD * i + e)], op.left[2 * (DD * i + e) + 1]);
                abi[base + 2 * e] += x.real();
                abi[base + 2 * e + 1] += x.imag();
            }
        }
        ++count;
    }
    if (!count) return fail(SV_ERR_ARG, "s is zero: the channel has no Kraus operator");
    *n_ops = count;
    return SV_OK;
}

}  // namespace sv

extern "C" int sv_channel_depolarizing(int k, const int32_t *q, double p, int after, double *mats, sv_super_op *out)
{
    sv::clear_error();
    if (!mats || !out) return sv::fail(SV_ERR_ARG, "NULL output");
    if (int rc = sv::check_qubits(k, q)) return rc;
    if (!sv::probability(p)) return sv::fail(SV_ERR_ARG, "depolarizing p = %g outside [0, 1]", p);
    if (after < 0) return sv::fail(SV_ERR_ARG, "after = %d", after);
    const size_t D = size_t(1) << k, n_ops = D * D;
    std::vector<sv::cd> P(D * D);
    for (size_t i = 0; i < n_ops; ++i) {
        sv::pauli_string(k, int(i), P.data());
        const double weight = p / double(n_ops) + (i == 0 ? 1.0 - p : 0.0);
        sv::put(mats, i, D, P.data(), std::sqrt(weight));
    }
    sv::kraus_out(k, q, int(n_ops), after, mats, out);
    return SV_OK;
}

extern "C" int sv_channel_dephasing(int qubit, int pauli, double p, int after, double *mats, sv_super_op *out)
{
    sv::clear_error();
    if (!mats || !out) return sv::fail(SV_ERR_ARG, "NULL output");
    const int32_t q[1] = {qubit};
    if (int rc = sv::check_qubits(1, q)) return rc;
    if (pauli < 1 || pauli > 3) return sv::fail(SV_ERR_ARG, "dephasing Pauli %d (1 = X, 2 = Y, 3 = Z)", pauli);
    if (!sv::probability(p)) return sv::fail(SV_ERR_ARG, "dephasing p = %g outside [0, 1]", p);
    if (after < 0) return sv::fail(SV_ERR_ARG, "after = %d", after);
    sv::put(mats, 0, 2, sv::kPauli[0], std::sqrt(1.0 - p));
    sv::put(mats, 1, 2, sv::kPauli[pauli], std::sqrt(p));
    sv::kraus_out(1, q, 2, after, mats, out);
    return SV_OK;
}

extern "C" int sv_channel_amplitude_damping(int qubit, double gamma, double beta, int after, double *mats,
                                            sv_super_op *out)
{
    sv::clear_error();
    if (!mats || !out) return sv::fail(SV_ERR_ARG, "NULL output");
    const int32_t q[1] = {qubit};
    if (int rc = sv::check_qubits(1, q)) return rc;
    if (!sv::probability(gamma) || !sv::probability(beta))
        return sv::fail(SV_ERR_ARG, "damping rate %g or excitation rate %g outside [0, 1]", gamma, beta);
    if (after < 0) return sv::fail(SV_ERR_ARG, "after = %d", after);
    const sv::cd K0[4] = {std::sqrt(1.0 - beta), 0, 0, std::sqrt(1.0 - gamma)};
    const sv::cd K1[4] = {0, std::sqrt(gamma), 0, 0};  // |0><1|
    const sv::cd K2[4] = {0, 0, std::sqrt(beta), 0};   // |1><0|
    sv::put(mats, 0, 2, K0, 1.0);
    sv::put(mats, 1, 2, K1, 1.0);
    int n_ops = 2;
    if (beta > 0.0) sv::put(mats, n_ops++, 2, K2, 1.0);
    sv::kraus_out(1, q, n_ops, after, mats, out);
    return SV_OK;
}

extern "C" int sv_channel_pauli(int k, const int32_t *q, const double *s, int after, double *mats, sv_super_op *out)
{
    sv::clear_error();
    if (!mats || !out || !s) return sv::fail(SV_ERR_ARG, "NULL argument");
    if (int rc = sv::check_qubits(k, q)) return rc;
    if (after < 0) return sv::fail(SV_ERR_ARG, "after = %d", after);
    const size_t D = size_t(1) << k, n_ops = D * D;
    for (size_t e = 0; e < 2 * n_ops * n_ops; ++e)
        if (!std::isfinite(s[e])) return sv::fail(SV_ERR_ARG, "non-finite s entry");
    std::vector<sv::cd> P(D * D);
    for (size_t i = 0; i < n_ops; ++i) {
        sv::pauli_string(k, int(i), P.data());
        sv::put(mats, i, D, P.data(), 1.0);
    }
    sv::kraus_out(k, q, int(n_ops), after, mats, out);
    out->s = s;
    return SV_OK;
}

extern "C" int sv_kraus_form(const sv_super_op *in, double *mats, sv_super_op *out)
{
    sv::clear_error();
    if (!in || !mats || !out) return sv::fail(SV_ERR_ARG, "NULL argument");
    if (int rc = sv::check_qubits(in->k, in->q)) return rc;
    if (in->n_left < 1 || in->n_left > 64 || !in->left || !in->right)
        return sv::fail(SV_ERR_ARG, "a KrausSuperGate with 1..64 operators is needed");
    std::vector<double> abi;
    int n_ops = 0;
    if (int rc = sv::kraus_form(*in, abi, &n_ops)) return rc;
    const sv_super_op copy = *in;  // `out` may alias `in`
    std::memcpy(mats, abi.data(), sizeof(double) * abi.size());
    sv::kraus_out(copy.k, copy.q, n_ops, copy.after, mats, out);
    return SV_OK;
}
