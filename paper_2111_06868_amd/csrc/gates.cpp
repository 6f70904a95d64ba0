// Gate table and gate validation (host only, no HIP calls).
//
// The paper names the gates (Gates and Properties section: H, X, RX, CPHASE,
// CX, ISWAP, FSIM, ...) but prints no matrices; these are the textbook ones.
// Rotations are R_P(t) = exp(-i t P / 2), which the paper's statement that
// RX(pi)**2.2 is the rotation by 2.2 pi fixes (principal-branch power).
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include <string>

#include "common.h"

namespace sv {

static thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

void clear_error() { g_last_error.clear(); }

const char *last_error_cstr() { return g_last_error.c_str(); }

int gate_arity(int kind)
{
    switch (kind) {
    case SV_G_MATRIX: return 0;
    case SV_G_I: case SV_G_X: case SV_G_Y: case SV_G_Z: case SV_G_H:
    case SV_G_SQRT_X: case SV_G_SQRT_Y: case SV_G_SQRT_W:
    case SV_G_RX: case SV_G_RY: case SV_G_RZ:
        return 1;
    case SV_G_CZ: case SV_G_CX: case SV_G_CPHASE: case SV_G_SWAP: case SV_G_FSIM:
        return 2;
    default:
        return -1;
    }
}

int check_gate_shape(const sv_gate &g)
{
    int a = gate_arity(g.kind);
    if (a < 0) return fail(SV_ERR_ARG, "unknown gate kind %d", g.kind);
    if (g.reserved != 0) return fail(SV_ERR_ARG, "sv_gate.reserved must be 0");
    if (a == 0) {
        if (g.k < 1 || g.k > SV_MAX_K) return fail(SV_ERR_ARG, "matrix gate with k=%d (1..%d)", g.k, SV_MAX_K);
        if (!g.m) return fail(SV_ERR_ARG, "matrix gate without a matrix");
        size_t D = size_t(1) << g.k;
        for (size_t i = 0; i < 2 * D * D; ++i)
            if (!std::isfinite(g.m[i])) return fail(SV_ERR_ARG, "matrix gate has a non-finite entry");
    } else if (g.k != a) {
        return fail(SV_ERR_ARG, "gate kind %d acts on %d qubits, got k=%d", g.kind, a, g.k);
    }
    if (!std::isfinite(g.params[0]) || !std::isfinite(g.params[1]))
        return fail(SV_ERR_ARG, "non-finite gate parameter");
    if (g.param >= 0 && g.kind != SV_G_RX && g.kind != SV_G_RY && g.kind != SV_G_RZ)
        return fail(SV_ERR_ARG, "only RX/RY/RZ gates can carry a differentiable parameter");
    if (g.param < -1) return fail(SV_ERR_ARG, "param index %d", g.param);
    return SV_OK;
}

int check_gate_qubits(const sv_gate &g, int n)
{
    for (int j = 0; j < g.k; ++j) {
        if (g.q[j] < 0 || g.q[j] >= n)
            return fail(SV_ERR_QUBIT, "qubit position %d outside 0..%d", g.q[j], n - 1);
        for (int i = 0; i < j; ++i)
            if (g.q[i] == g.q[j]) return fail(SV_ERR_QUBIT, "qubit position %d repeated in a gate", g.q[j]);
    }
    return SV_OK;
}

static void set2(std::vector<cd> &m, cd a, cd b, cd c, cd d)
{
    m = {a, b, c, d};
}

int gate_matrix_abi(const sv_gate &g, std::vector<cd> &out)
{
    int rc = check_gate_shape(g);
    if (rc) return rc;
    const cd I(0, 1);
    const double s2 = std::sqrt(0.5);
    const cd hp = cd(0.5, 0.5), hm = cd(0.5, -0.5);  // (1+i)/2, (1-i)/2
    switch (g.kind) {
    case SV_G_MATRIX: {
        size_t D = size_t(1) << g.k;
        out.resize(D * D);
        for (size_t i = 0; i < D * D; ++i) out[i] = cd(g.m[2 * i], g.m[2 * i + 1]);
        return SV_OK;
    }
    case SV_G_I: set2(out, 1, 0, 0, 1); return SV_OK;
    case SV_G_X: set2(out, 0, 1, 1, 0); return SV_OK;
    case SV_G_Y: set2(out, 0, -I, I, 0); return SV_OK;
    case SV_G_Z: set2(out, 1, 0, 0, -1); return SV_OK;
    case SV_G_H: set2(out, s2, s2, s2, -s2); return SV_OK;
    // sqrt(P) = (1+i)/2 I + (1-i)/2 P
    case SV_G_SQRT_X: set2(out, hp, hm, hm, hp); return SV_OK;
    case SV_G_SQRT_Y: set2(out, hp, hm * (-I), hm * I, hp); return SV_OK;
    case SV_G_SQRT_W: {
        // W = (X + Y)/sqrt2 = [[0, (1-i)/sqrt2], [(1+i)/sqrt2, 0]]
        cd w01 = cd(s2, -s2), w10 = cd(s2, s2);
        set2(out, hp, hm * w01, hm * w10, hp);
        return SV_OK;
    }
    case SV_G_RX: case SV_G_RY: case SV_G_RZ: {
        double c = std::cos(0.5 * g.params[0]), s = std::sin(0.5 * g.params[0]);
        if (g.kind == SV_G_RX) set2(out, c, -I * s, -I * s, c);
        else if (g.kind == SV_G_RY) set2(out, c, -s, s, c);
        else set2(out, cd(c, -s), 0, 0, cd(c, s));
        return SV_OK;
    }
    default: break;
    }
    out.assign(16, cd(0));
    auto at = [&](int r, int c) -> cd & { return out[r * 4 + c]; };
    switch (g.kind) {
    case SV_G_CZ: at(0, 0) = at(1, 1) = at(2, 2) = 1; at(3, 3) = -1; break;
    case SV_G_CPHASE: at(0, 0) = at(1, 1) = at(2, 2) = 1; at(3, 3) = std::exp(I * g.params[0]); break;
    case SV_G_CX: at(0, 0) = at(1, 1) = 1; at(2, 3) = at(3, 2) = 1; break;
    case SV_G_SWAP: at(0, 0) = at(3, 3) = 1; at(1, 2) = at(2, 1) = 1; break;
    case SV_G_FSIM: {
        double c = std::cos(g.params[0]), s = std::sin(g.params[0]);
        at(0, 0) = 1;
        at(1, 1) = at(2, 2) = c;
        at(1, 2) = at(2, 1) = -I * s;
        at(3, 3) = std::exp(-I * g.params[1]);
        break;
    }
    default: return fail(SV_ERR_ARG, "unknown gate kind %d", g.kind);
    }
    return SV_OK;
}

int gate_matrix_canonical(const sv_gate &g, std::vector<cd> &m, int *sorted_q)
{
    std::vector<cd> abi;
    int rc = gate_matrix_abi(g, abi);
    if (rc) return rc;
    const int k = g.k;
    // rank[j] = number of positions below q[j] = canonical bit of q[j]
    int rank[SV_MAX_K];
    for (int j = 0; j < k; ++j) {
        rank[j] = 0;
        for (int i = 0; i < k; ++i) rank[j] += g.q[i] < g.q[j];
        sorted_q[rank[j]] = g.q[j];
    }
    const int D = 1 << k;
    std::vector<int> to_can(D);
    for (int a = 0; a < D; ++a) {
        int c = 0;
        for (int j = 0; j < k; ++j)
            if ((a >> (k - 1 - j)) & 1) c |= 1 << rank[j];
        to_can[a] = c;
    }
    m.assign(size_t(D) * D, cd(0));
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) m[size_t(to_can[a]) * D + to_can[b]] = abi[size_t(a) * D + b];
    return SV_OK;
}

void reverse_local_bits(const std::vector<cd> &in, int k, std::vector<cd> &out)
{
    const int D = 1 << k;
    auto rev = [k](int a) {
        int r = 0;
        for (int j = 0; j < k; ++j)
            if ((a >> j) & 1) r |= 1 << (k - 1 - j);
        return r;
    };
    out.assign(size_t(D) * D, cd(0));
    for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b) out[size_t(rev(a)) * D + rev(b)] = in[size_t(a) * D + b];
}

// Split-FP16 tile passes hold each tile scaled so that its largest value is
// below 2^8 and rely on blocks that cannot raise the tile's 2-norm; a unitary
// (checked to 1e-6 per entry of U^dagger U) cannot.
int check_unitary(const std::vector<cd> &U, int k, const char *what)
{
    const size_t d = size_t(1) << k;
    for (size_t i = 0; i < d; ++i)
        for (size_t j = 0; j < d; ++j) {
            cd acc = 0;
            for (size_t r = 0; r < d; ++r) acc += std::conj(U[r * d + i]) * U[r * d + j];
            if (std::abs(acc - cd(i == j ? 1.0 : 0.0)) > 1e-6)
                return fail(SV_ERR_ARG, "%s is not unitary (|U^dagger U - I| > 1e-6); split FP16 needs unitary gates",
                            what);
        }
    return SV_OK;
}

int check_fp16_gates(const sv_gate *g, int G)
{
    for (int i = 0; i < G; ++i) {
        if (g[i].kind != SV_G_MATRIX) continue;  // the named gates are unitary
        std::vector<cd> U;
        if (int rc = gate_matrix_abi(g[i], U)) return rc;
        std::string what = "matrix gate " + std::to_string(i);
        if (int rc = check_unitary(U, g[i].k, what.c_str())) return rc;
    }
    return SV_OK;
}

}  // namespace sv
