// FP64 reductions over a state: norm, inner product, Pauli-sum expectation,
// the Pauli-sum matvec used by the adjoint method, and Tr(rho H) of a density
// matrix held as a state of 2n qubits.
//
// Every reduction is a fixed-shape two-stage tree (kRedBlocks x kRedThreads
// first stage with a fixed grid-stride assignment, LDS tree inside a block,
// then one block summing the partials in a fixed order), so results are
// bitwise reproducible run to run.  Amplitudes are widened to FP64 before any
// product.
//
// Pauli strings: P = i^{#Y} X^x Z^z (per qubit Y = i X Z), hence
//   (P psi)[i] = i^{#Y} (-1)^{popcount((i ^ x) & z)} psi[i ^ x].
// Terms are grouped by their x mask on the host so that each partner
// amplitude psi[i ^ x] is loaded once per group.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sv {
namespace dev {

namespace {

template <int C>
struct Acc {
    double v[C];
};

template <int C>
__device__ __forceinline__ void block_reduce_store(Acc<C> a, double *__restrict__ out)
{
    __shared__ double sh[C][kRedThreads];
    const int t = threadIdx.x;
#pragma unroll
    for (int c = 0; c < C; ++c) sh[c][t] = a.v[c];
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int c = 0; c < C; ++c) sh[c][t] += sh[c][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
#pragma unroll
        for (int c = 0; c < C; ++c) out[c] = sh[c][0];
    }
}

__device__ __forceinline__ void ld(const float *p, uint64_t i, double &re, double &im)
{
    const float2 v = reinterpret_cast<const float2 *>(p)[i];
    re = v.x;
    im = v.y;
}
__device__ __forceinline__ void ld(const double *p, uint64_t i, double &re, double &im)
{
    const double2 v = reinterpret_cast<const double2 *>(p)[i];
    re = v.x;
    im = v.y;
}

template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_norm(const T *__restrict__ psi, uint64_t N, double *partials)
{
    Acc<1> a{{0.0}};
    for (uint64_t i = uint64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < N; i += uint64_t(kRedBlocks) * kRedThreads) {
        double r, m;
        ld(psi, i, r, m);
        a.v[0] = fma(r, r, fma(m, m, a.v[0]));
    }
    block_reduce_store<1>(a, partials + blockIdx.x);
}

// complex64 norm: each thread takes 4 consecutive 16-byte pairs of
// amplitudes per step (4 loads in flight), in a fixed assignment
__global__ void __launch_bounds__(kRedThreads) k_norm_c64(const float4 *__restrict__ psi, uint64_t N4,
                                                          double *partials)
{
    Acc<1> a{{0.0}};
    constexpr uint64_t kStep = uint64_t(kRedBlocks) * kRedThreads * 4;
    for (uint64_t i0 = (uint64_t(blockIdx.x) * kRedThreads + threadIdx.x) * 4; i0 < N4; i0 += kStep) {
        float4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = i0 + u < N4 ? psi[i0 + u] : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a.v[0] = fma(double(v[u].x), double(v[u].x), a.v[0]);
            a.v[0] = fma(double(v[u].y), double(v[u].y), a.v[0]);
            a.v[0] = fma(double(v[u].z), double(v[u].z), a.v[0]);
            a.v[0] = fma(double(v[u].w), double(v[u].w), a.v[0]);
        }
    }
    block_reduce_store<1>(a, partials + blockIdx.x);
}

template <typename A, typename B>
__global__ void __launch_bounds__(kRedThreads) k_inner(const A *__restrict__ a, const B *__restrict__ b, uint64_t N,
                                                      double *partials)
{
    Acc<2> s{{0.0, 0.0}};
    for (uint64_t i = uint64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < N; i += uint64_t(kRedBlocks) * kRedThreads) {
        double ar, ai, br, bi;
        ld(a, i, ar, ai);
        ld(b, i, br, bi);
        // conj(a) * b
        s.v[0] = fma(ar, br, fma(ai, bi, s.v[0]));
        s.v[1] = fma(ar, bi, fma(-ai, br, s.v[1]));
    }
    block_reduce_store<2>(s, partials + 2 * blockIdx.x);
}

// weight of group g at partner index j: sum_t c_t i^{pow_t} (-1)^{popcount(j & z_t)}
__device__ __forceinline__ void group_weight(const PauliDev &H, int g, uint64_t j, double &wr, double &wi)
{
    wr = 0.0;
    wi = 0.0;
    for (int t = H.goff[g]; t < H.goff[g + 1]; ++t) {
        double c = H.tc[t];
        if (__popcll(j & H.tz[t]) & 1) c = -c;
        switch (H.tpow[t] & 3) {
        case 0: wr += c; break;
        case 1: wi += c; break;
        case 2: wr -= c; break;
        default: wi -= c; break;
        }
    }
}

template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_pauli_expect(const T *__restrict__ psi, uint64_t N, const PauliDev H,
                                                             double *partials)
{
    Acc<1> a{{0.0}};
    for (uint64_t i = uint64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < N; i += uint64_t(kRedBlocks) * kRedThreads) {
        double cr, ci;
        ld(psi, i, cr, ci);
        double sr = 0.0, si = 0.0;
        for (int g = 0; g < H.n_groups; ++g) {
            const uint64_t j = i ^ H.gx[g];
            double pr, pi, wr, wi;
            ld(psi, j, pr, pi);
            group_weight(H, g, j, wr, wi);
            sr = fma(wr, pr, fma(-wi, pi, sr));
            si = fma(wr, pi, fma(wi, pr, si));
        }
        // Re(conj(psi_i) * s)
        a.v[0] = fma(cr, sr, fma(ci, si, a.v[0]));
    }
    block_reduce_store<1>(a, partials + blockIdx.x);
}

// Tr(rho H) for rho held row-major in a state of 2n qubits (rho[r][c] at
// r 2^n + c).  With P|a> = omega(a)|a ^ x>, Tr(rho P) = sum_a omega(a)
// rho[a][a ^ x]; omega(a) is the group weight at a (group_weight), and only
// the real part is summed (H is Hermitian).
template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_dm_expect(const T *__restrict__ rho, int n, const PauliDev H,
                                                          double *partials)
{
    Acc<1> acc{{0.0}};
    const uint64_t N = uint64_t(1) << n;
    for (uint64_t a = uint64_t(blockIdx.x) * kRedThreads + threadIdx.x; a < N; a += uint64_t(kRedBlocks) * kRedThreads) {
        for (int g = 0; g < H.n_groups; ++g) {
            double rr, ri, wr, wi;
            ld(rho, (a << n) | (a ^ H.gx[g]), rr, ri);
            group_weight(H, g, a, wr, wi);
            acc.v[0] = fma(rr, wr, fma(-ri, wi, acc.v[0]));
        }
    }
    block_reduce_store<1>(acc, partials + blockIdx.x);
}

// Outcome weights of a Kraus channel on k sorted positions: p_i = ||K_i psi||^2
// (paper, Simulations with noise section: channels sampled on pure states).
// Each thread gathers the 2^k amplitudes of U groups (local bit j on the j-th
// lowest position; all loads issued before any arithmetic, so that U groups
// are in flight per thread), forms K_i x for every operator and adds
// |K_i x|^2, all in FP64.  The per-thread order of the groups is fixed, so the
// result is reproducible.
template <typename T, int K>
__global__ void __launch_bounds__(kRedThreads) k_kraus_probs(const T *__restrict__ psi, int n, const KrausDev Kd,
                                                            double *partials)
{
    constexpr int D = 1 << K;
    constexpr int U = K == 3 ? 2 : 4;
    Acc<kMaxKraus> acc;
#pragma unroll
    for (int i = 0; i < kMaxKraus; ++i) acc.v[i] = 0.0;
    const uint64_t groups = uint64_t(1) << (n - K);
    const uint64_t stride = uint64_t(kRedBlocks) * kRedThreads;
    for (uint64_t g0 = uint64_t(blockIdx.x) * kRedThreads + threadIdx.x; g0 < groups; g0 += U * stride) {
        double xr[U][D], xi[U][D];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t g = g0 + u * stride;
            uint64_t base = g < groups ? g : 0;
#pragma unroll
            for (int j = 0; j < K; ++j) {  // insert a zero bit at each position, lowest first
                const uint64_t low = base & ((uint64_t(1) << Kd.pos[j]) - 1);
                base = ((base - low) << 1) | low;
            }
#pragma unroll
            for (int m = 0; m < D; ++m) {
                uint64_t idx = base;
#pragma unroll
                for (int j = 0; j < K; ++j)
                    if ((m >> j) & 1) idx |= uint64_t(1) << Kd.pos[j];
                ld(psi, idx, xr[u][m], xi[u][m]);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (g0 + u * stride >= groups) continue;
#pragma unroll
            for (int i = 0; i < kMaxKraus; ++i) {
                if (i >= Kd.n_ops) continue;  // uniform
                const double *M = Kd.m + size_t(2) * D * D * i;
                double s = 0.0;
#pragma unroll
                for (int r = 0; r < D; ++r) {
                    double yr = 0.0, yi = 0.0;
#pragma unroll
                    for (int c = 0; c < D; ++c) {
                        const double mr = M[2 * (r * D + c)], mi = M[2 * (r * D + c) + 1];
                        yr = fma(mr, xr[u][c], fma(-mi, xi[u][c], yr));
                        yi = fma(mr, xi[u][c], fma(mi, xr[u][c], yi));
                    }
                    s = fma(yr, yr, fma(yi, yi, s));
                }
                acc.v[i] += s;
            }
        }
    }
    block_reduce_store<kMaxKraus>(acc, partials + size_t(blockIdx.x) * kMaxKraus);
}

// The same for complex64 states with 16-byte loads: when the channel's lowest
// position is 0 (LOW0), amplitudes m and m + 1 of a group are adjacent; else
// the groups 2h and 2h + 1 differ only in position 0, so amplitude m of both is
// one float4.  Each thread takes U units (groups, or pairs of groups) per step.
template <int K, bool LOW0>
__global__ void __launch_bounds__(kRedThreads) k_kraus_probs_c64(const float4 *__restrict__ psi, int n,
                                                                const KrausDev Kd, double *partials)
{
    constexpr int D = 1 << K;
    constexpr int G = LOW0 ? 1 : 2;                // groups per unit
    constexpr int L = LOW0 ? D / 2 : D;            // float4 loads per unit
    constexpr int U = K == 3 ? (LOW0 ? 2 : 1) : 4;
    Acc<kMaxKraus> acc;
#pragma unroll
    for (int i = 0; i < kMaxKraus; ++i) acc.v[i] = 0.0;
    const uint64_t units = uint64_t(1) << (n - K - (LOW0 ? 0 : 1));
    const uint64_t stride = uint64_t(kRedBlocks) * kRedThreads;
    for (uint64_t h0 = uint64_t(blockIdx.x) * kRedThreads + threadIdx.x; h0 < units; h0 += U * stride) {
        float4 v[U][L];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint64_t h = h0 + u * stride;
            uint64_t base = h < units ? (LOW0 ? h : h << 1) : 0;
#pragma unroll
            for (int j = 0; j < K; ++j) {
                const uint64_t low = base & ((uint64_t(1) << Kd.pos[j]) - 1);
                base = ((base - low) << 1) | low;
            }
#pragma unroll
            for (int l = 0; l < L; ++l) {
                const int m = LOW0 ? 2 * l : l;
                uint64_t idx = base;
#pragma unroll
                for (int j = 0; j < K; ++j)
                    if ((m >> j) & 1) idx |= uint64_t(1) << Kd.pos[j];
                v[u][l] = psi[idx >> 1];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (h0 + u * stride >= units) continue;
#pragma unroll
            for (int gsel = 0; gsel < G; ++gsel) {
                double xr[D], xi[D];
#pragma unroll
                for (int m = 0; m < D; ++m) {
                    const float4 w = LOW0 ? v[u][m >> 1] : v[u][m];
                    const bool hi = LOW0 ? (m & 1) : gsel;
                    xr[m] = hi ? w.z : w.x;
                    xi[m] = hi ? w.w : w.y;
                }
#pragma unroll
                for (int i = 0; i < kMaxKraus; ++i) {
                    if (i >= Kd.n_ops) continue;  // uniform
                    const double *M = Kd.m + size_t(2) * D * D * i;
                    double s = 0.0;
#pragma unroll
                    for (int r = 0; r < D; ++r) {
                        double yr = 0.0, yi = 0.0;
#pragma unroll
                        for (int c = 0; c < D; ++c) {
                            const double mr = M[2 * (r * D + c)], mi = M[2 * (r * D + c) + 1];
                            yr = fma(mr, xr[c], fma(-mi, xi[c], yr));
                            yi = fma(mr, xi[c], fma(mi, xr[c], yi));
                        }
                        s = fma(yr, yr, fma(yi, yi, s));
                    }
                    acc.v[i] += s;
                }
            }
        }
    }
    block_reduce_store<kMaxKraus>(acc, partials + size_t(blockIdx.x) * kMaxKraus);
}

template <typename T>
__global__ void __launch_bounds__(256) k_pauli_apply(const T *__restrict__ psi, T *__restrict__ out, uint64_t N,
                                                    const PauliDev H)
{
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
        double sr = 0.0, si = 0.0;
        for (int g = 0; g < H.n_groups; ++g) {
            const uint64_t j = i ^ H.gx[g];
            double pr, pi, wr, wi;
            ld(psi, j, pr, pi);
            group_weight(H, g, j, wr, wi);
            sr = fma(wr, pr, fma(-wi, pi, sr));
            si = fma(wr, pi, fma(wi, pr, si));
        }
        out[2 * i] = T(sr);
        out[2 * i + 1] = T(si);
    }
}

// Second stage: sums C-component partials of `nb` blocks for `slots` slots
// (one workgroup per slot) in a fixed order.
template <int C>
__global__ void __launch_bounds__(kRedThreads) k_final(const double *__restrict__ partials, int nb, double *out)
{
    const double *p = partials + size_t(blockIdx.x) * nb * C;
    Acc<C> a;
#pragma unroll
    for (int c = 0; c < C; ++c) a.v[c] = 0.0;
    for (int i = threadIdx.x; i < nb; i += kRedThreads) {
#pragma unroll
        for (int c = 0; c < C; ++c) a.v[c] += p[size_t(i) * C + c];
    }
    block_reduce_store<C>(a, out + size_t(blockIdx.x) * C);
}

}  // namespace

hipError_t launch_norm(int dtype, const void *psi, int n, double *d_partials, double *d_out, hipStream_t st)
{
    const uint64_t N = uint64_t(1) << n;
    if (dtype == SV_C64 && n >= 1)
        hipLaunchKernelGGL(k_norm_c64, dim3(kRedBlocks), dim3(kRedThreads), 0, st, static_cast<const float4 *>(psi), N / 2,
                           d_partials);
    else if (dtype == SV_C64)
        hipLaunchKernelGGL(k_norm<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, static_cast<const float *>(psi), N, d_partials);
    else
        hipLaunchKernelGGL(k_norm<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, static_cast<const double *>(psi), N, d_partials);
    hipLaunchKernelGGL(k_final<1>, dim3(1), dim3(kRedThreads), 0, st, d_partials, kRedBlocks, d_out);
    return hipGetLastError();
}

hipError_t launch_inner(int dtype_a, const void *a, int dtype_b, const void *b, int n, double *d_partials,
                        double *d_out, hipStream_t st)
{
    const uint64_t N = uint64_t(1) << n;
    const dim3 g(kRedBlocks), t(kRedThreads);
    if (dtype_a == SV_C64 && dtype_b == SV_C64)
        hipLaunchKernelGGL((k_inner<float, float>), g, t, 0, st, static_cast<const float *>(a), static_cast<const float *>(b), N, d_partials);
    else if (dtype_a == SV_C64)
        hipLaunchKernelGGL((k_inner<float, double>), g, t, 0, st, static_cast<const float *>(a), static_cast<const double *>(b), N, d_partials);
    else if (dtype_b == SV_C64)
        hipLaunchKernelGGL((k_inner<double, float>), g, t, 0, st, static_cast<const double *>(a), static_cast<const float *>(b), N, d_partials);
    else
        hipLaunchKernelGGL((k_inner<double, double>), g, t, 0, st, static_cast<const double *>(a), static_cast<const double *>(b), N, d_partials);
    hipLaunchKernelGGL(k_final<2>, dim3(1), dim3(kRedThreads), 0, st, d_partials, kRedBlocks, d_out);
    return hipGetLastError();
}

hipError_t launch_pauli_expect(int dtype, const void *psi, int n, const PauliDev &H, double *d_partials,
                               double *d_out, hipStream_t st)
{
    const uint64_t N = uint64_t(1) << n;
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_pauli_expect<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, static_cast<const float *>(psi), N, H, d_partials);
    else
        hipLaunchKernelGGL(k_pauli_expect<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, static_cast<const double *>(psi), N, H, d_partials);
    hipLaunchKernelGGL(k_final<1>, dim3(1), dim3(kRedThreads), 0, st, d_partials, kRedBlocks, d_out);
    return hipGetLastError();
}

hipError_t launch_dm_expect(int dtype, const void *rho, int n, const PauliDev &H, double *d_partials, double *d_out,
                            hipStream_t st)
{
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_dm_expect<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, static_cast<const float *>(rho), n, H, d_partials);
    else
        hipLaunchKernelGGL(k_dm_expect<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, static_cast<const double *>(rho), n, H, d_partials);
    hipLaunchKernelGGL(k_final<1>, dim3(1), dim3(kRedThreads), 0, st, d_partials, kRedBlocks, d_out);
    return hipGetLastError();
}

hipError_t launch_kraus_probs(int dtype, const void *psi, int n, const KrausDev &K, double *d_partials,
                              double *d_out, hipStream_t st)
{
    if (K.k < 1 || K.k > 3 || K.k > n || K.n_ops < 1 || K.n_ops > kMaxKraus) return hipErrorInvalidValue;
    const dim3 g(kRedBlocks), t(kRedThreads);
    const bool c64 = dtype == SV_C64;
    const float *pf = static_cast<const float *>(psi);
    const double *pd = static_cast<const double *>(psi);
    // complex64 with 16-byte loads (needs a pair of groups when position 0 is free)
    if (c64 && (K.pos[0] == 0 || n - K.k >= 1)) {
        const float4 *p4 = static_cast<const float4 *>(psi);
        const bool low0 = K.pos[0] == 0;
        switch (K.k) {
        case 1:
            if (low0) hipLaunchKernelGGL((k_kraus_probs_c64<1, true>), g, t, 0, st, p4, n, K, d_partials);
            else hipLaunchKernelGGL((k_kraus_probs_c64<1, false>), g, t, 0, st, p4, n, K, d_partials);
            break;
        case 2:
            if (low0) hipLaunchKernelGGL((k_kraus_probs_c64<2, true>), g, t, 0, st, p4, n, K, d_partials);
            else hipLaunchKernelGGL((k_kraus_probs_c64<2, false>), g, t, 0, st, p4, n, K, d_partials);
            break;
        default:
            if (low0) hipLaunchKernelGGL((k_kraus_probs_c64<3, true>), g, t, 0, st, p4, n, K, d_partials);
            else hipLaunchKernelGGL((k_kraus_probs_c64<3, false>), g, t, 0, st, p4, n, K, d_partials);
            break;
        }
        hipLaunchKernelGGL(k_final<kMaxKraus>, dim3(1), dim3(kRedThreads), 0, st, d_partials, kRedBlocks, d_out);
        return hipGetLastError();
    }
    switch (K.k) {
    case 1:
        if (c64) hipLaunchKernelGGL((k_kraus_probs<float, 1>), g, t, 0, st, pf, n, K, d_partials);
        else hipLaunchKernelGGL((k_kraus_probs<double, 1>), g, t, 0, st, pd, n, K, d_partials);
        break;
    case 2:
        if (c64) hipLaunchKernelGGL((k_kraus_probs<float, 2>), g, t, 0, st, pf, n, K, d_partials);
        else hipLaunchKernelGGL((k_kraus_probs<double, 2>), g, t, 0, st, pd, n, K, d_partials);
        break;
    default:
        if (c64) hipLaunchKernelGGL((k_kraus_probs<float, 3>), g, t, 0, st, pf, n, K, d_partials);
        else hipLaunchKernelGGL((k_kraus_probs<double, 3>), g, t, 0, st, pd, n, K, d_partials);
        break;
    }
    hipLaunchKernelGGL(k_final<kMaxKraus>, dim3(1), dim3(kRedThreads), 0, st, d_partials, kRedBlocks, d_out);
    return hipGetLastError();
}

hipError_t launch_pauli_apply(int dtype, const void *psi, void *out, int n, const PauliDev &H, hipStream_t st)
{
    const uint64_t N = uint64_t(1) << n;
    uint64_t blocks = (N + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_pauli_apply<float>, dim3(unsigned(blocks)), dim3(256), 0, st, static_cast<const float *>(psi),
                           static_cast<float *>(out), N, H);
    else
        hipLaunchKernelGGL(k_pauli_apply<double>, dim3(unsigned(blocks)), dim3(256), 0, st, static_cast<const double *>(psi),
                           static_cast<double *>(out), N, H);
    return hipGetLastError();
}

hipError_t launch_sum_partials(const double *d_partials, int n_slots, double *d_out, hipStream_t st)
{
    if (n_slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_final<2>, dim3(n_slots), dim3(kRedThreads), 0, st, d_partials, kRedBlocks, d_out);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace sv
