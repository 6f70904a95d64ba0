// Adjoint-method backward step (one gate, two states in one pass).
//
// E(theta) = <psi|H|psi>, psi = U_G..U_1 psi_0.  With phi = U_{g+1}^+..U_G^+ psi
// and lam = U_{g+1}^+..U_G^+ H psi, and a rotation U_g = exp(-i theta P / 2),
//   dE/dtheta_g = 2 Re <lam| dU_g/dtheta |phi_{g-1}> = 2 Re <lam| (-i/2) P |phi>
//               = Im <lam|P|phi>,
// evaluated before both states move one gate back (phi <- U_g^+ phi,
// lam <- U_g^+ lam).  One kernel per gate reads both states once, adds the
// group's share of <lam|P|phi> (FP64) to a per-block partial, and writes both
// updated states: two buffers, no stored trajectory.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sv {
namespace dev {

namespace {

template <typename T, int K>
struct BwdArgs {
    T mr[(1 << K) * (1 << K)];
    T mi[(1 << K) * (1 << K)];
    int pos[K];
    int pauli;
    uint64_t n_groups;
    double pmat[8];  // generator P as a 2x2 complex matrix (re, im), row-major
};

__device__ __forceinline__ uint64_t insert_zero_b(uint64_t x, int p)
{
    return ((x >> p) << (p + 1)) | (x & ((uint64_t(1) << p) - 1));
}

template <typename T, int K>
__device__ __forceinline__ void matvec(const BwdArgs<T, K> &a, const T *vr, const T *vi, T *orr, T *oi)
{
    constexpr int D = 1 << K;
#pragma unroll
    for (int m = 0; m < D; ++m) {
        T sr = 0, si = 0;
#pragma unroll
        for (int mp = 0; mp < D; ++mp) {
            const T ar = a.mr[m * D + mp], ai = a.mi[m * D + mp];
            sr = fma(ar, vr[mp], sr);
            sr = fma(-ai, vi[mp], sr);
            si = fma(ar, vi[mp], si);
            si = fma(ai, vr[mp], si);
        }
        orr[m] = sr;
        oi[m] = si;
    }
}

template <typename T, int K>
__global__ void __launch_bounds__(kRedThreads) k_backward(T *__restrict__ phi, T *__restrict__ lam,
                                                         const BwdArgs<T, K> a, double *__restrict__ partials)
{
    constexpr int D = 1 << K;
    double gr = 0.0, gi = 0.0;
    for (uint64_t g = uint64_t(blockIdx.x) * kRedThreads + threadIdx.x; g < a.n_groups;
         g += uint64_t(kRedBlocks) * kRedThreads) {
        uint64_t base = g;
#pragma unroll
        for (int j = 0; j < K; ++j) base = insert_zero_b(base, a.pos[j]);
        uint64_t idx[D];
        T fr[D], fi[D], lr[D], li[D];
#pragma unroll
        for (int m = 0; m < D; ++m) {
            uint64_t o = base;
#pragma unroll
            for (int j = 0; j < K; ++j)
                if ((m >> j) & 1) o += uint64_t(1) << a.pos[j];
            idx[m] = o;
            fr[m] = phi[2 * o];
            fi[m] = phi[2 * o + 1];
            lr[m] = lam[2 * o];
            li[m] = lam[2 * o + 1];
        }
        if (K == 1 && a.pauli) {
            // s = <lam|P|phi> restricted to this group, P (2x2, on local bit 0)
            // given as a matrix: (P phi)_r = sum_c P[r][c] phi_c
            double pr[2], pi[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                pr[r] = 0.0;
                pi[r] = 0.0;
#pragma unroll
                for (int c = 0; c < 2; ++c) {
                    const double gr_ = a.pmat[4 * r + 2 * c], gi_ = a.pmat[4 * r + 2 * c + 1];
                    const double vr = fr[c * (D - 1)], vi = fi[c * (D - 1)];
                    pr[r] += gr_ * vr - gi_ * vi;
                    pi[r] += gr_ * vi + gi_ * vr;
                }
            }
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const double ur = lr[r * (D - 1)], ui = li[r * (D - 1)];
                // conj(lam_r) * (P phi)_r
                gr += ur * pr[r] + ui * pi[r];
                gi += ur * pi[r] - ui * pr[r];
            }
        }
        T or_[D], oi[D];
        matvec<T, K>(a, fr, fi, or_, oi);
#pragma unroll
        for (int m = 0; m < D; ++m) {
            phi[2 * idx[m]] = or_[m];
            phi[2 * idx[m] + 1] = oi[m];
        }
        matvec<T, K>(a, lr, li, or_, oi);
#pragma unroll
        for (int m = 0; m < D; ++m) {
            lam[2 * idx[m]] = or_[m];
            lam[2 * idx[m] + 1] = oi[m];
        }
    }
    if (a.pauli) {
        __shared__ double sr[kRedThreads], si[kRedThreads];
        const int t = threadIdx.x;
        sr[t] = gr;
        si[t] = gi;
        __syncthreads();
        for (int s = kRedThreads / 2; s > 0; s >>= 1) {
            if (t < s) {
                sr[t] += sr[t + s];
                si[t] += si[t + s];
            }
            __syncthreads();
        }
        if (t == 0) {
            partials[2 * blockIdx.x] = sr[0];
            partials[2 * blockIdx.x + 1] = si[0];
        }
    }
}

template <typename T, int K>
hipError_t bwd_launch_t(const int *sorted_q, const cd *mdag, int pauli, T *phi, T *lam, int n, double *d_partials,
                        int slot, hipStream_t st)
{
    BwdArgs<T, K> a;
    constexpr int D = 1 << K;
    for (int i = 0; i < D * D; ++i) {
        a.mr[i] = T(mdag[i].real());
        a.mi[i] = T(mdag[i].imag());
    }
    for (int j = 0; j < K; ++j) a.pos[j] = sorted_q[j];
    a.pauli = pauli;
    // X, Y, Z as 2x2 complex matrices
    static const double P[4][8] = {{0, 0, 0, 0, 0, 0, 0, 0},
                                   {0, 0, 1, 0, 1, 0, 0, 0},
                                   {0, 0, 0, -1, 0, 1, 0, 0},
                                   {1, 0, 0, 0, 0, 0, -1, 0}};
    for (int i = 0; i < 8; ++i) a.pmat[i] = P[pauli & 3][i];
    a.n_groups = uint64_t(1) << (n - K);
    double *part = d_partials + size_t(slot < 0 ? 0 : slot) * kRedBlocks * 2;
    hipLaunchKernelGGL((k_backward<T, K>), dim3(kRedBlocks), dim3(kRedThreads), 0, st, phi, lam, a, part);
    return hipGetLastError();
}

// <lam| P_t |phi> for up to kMaxGradTerms Pauli strings in one pass over the
// two states (used for a run of commuting rotations: every rotation of the
// run sees the same phi and lam, see sv_backward).
struct GradTerms {
    int n_terms;
    uint64_t x[kMaxGradTerms];
    uint64_t z[kMaxGradTerms];
    int pw[kMaxGradTerms];  // power of i (number of Y factors mod 4)
    uint64_t N;
};

__device__ __forceinline__ void ld2(const float *p, uint64_t i, double &re, double &im)
{
    const float2 v = reinterpret_cast<const float2 *>(p)[i];
    re = v.x;
    im = v.y;
}
__device__ __forceinline__ void ld2(const double *p, uint64_t i, double &re, double &im)
{
    const double2 v = reinterpret_cast<const double2 *>(p)[i];
    re = v.x;
    im = v.y;
}

// Sum over the 64 lanes of a wave in a fixed butterfly order.
__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T, int NT>
__global__ void __launch_bounds__(kRedThreads) k_grad_terms(const T *__restrict__ phi, const T *__restrict__ lam,
                                                           const GradTerms a, double *__restrict__ partials)
{
    double sr[NT], si[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) sr[t] = si[t] = 0.0;
    for (uint64_t i = uint64_t(blockIdx.x) * kRedThreads + threadIdx.x; i < a.N; i += uint64_t(kRedBlocks) * kRedThreads) {
        double lr, li, fr, fi;
        ld2(lam, i, lr, li);
        ld2(phi, i, fr, fi);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            if (t >= a.n_terms) break;
            const uint64_t j = i ^ a.x[t];
            double pr = fr, pi = fi;
            if (a.x[t]) ld2(phi, j, pr, pi);  // Z-type terms (x = 0) reuse phi_i
            if (__popcll(j & a.z[t]) & 1) {
                pr = -pr;
                pi = -pi;
            }
            // multiply by i^pw
            double qr = pr, qi = pi;
            switch (a.pw[t] & 3) {
            case 1: qr = -pi; qi = pr; break;
            case 2: qr = -pr; qi = -pi; break;
            case 3: qr = pi; qi = -pr; break;
            default: break;
            }
            // conj(lam_i) * (P phi)_i
            sr[t] += lr * qr + li * qi;
            si[t] += lr * qi - li * qr;
        }
    }
    // workgroup sums: wave butterflies, then the waves' values in wave order
    constexpr int kWaves = kRedThreads / 64;
    __shared__ double sh[kWaves][2 * NT];
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        if (t >= a.n_terms) break;
        const double r = wave_sum(sr[t]), m = wave_sum(si[t]);
        if (lane == 0) {
            sh[wv][2 * t] = r;
            sh[wv][2 * t + 1] = m;
        }
    }
    __syncthreads();
    if (tid < 2 * a.n_terms) {
        double v = 0.0;
        for (int w = 0; w < kWaves; ++w) v += sh[w][tid];
        partials[(size_t(tid >> 1) * kRedBlocks + blockIdx.x) * 2 + (tid & 1)] = v;
    }
}

}  // namespace

hipError_t launch_grad_terms(int dtype, int n_terms, const uint64_t *x, const uint64_t *z, const int *pw,
                             const void *phi, const void *lam, int n, double *d_partials, int slot0, hipStream_t st)
{
    if (n_terms < 1 || n_terms > kMaxGradTerms) return hipErrorInvalidValue;
    GradTerms a;
    a.n_terms = n_terms;
    for (int t = 0; t < kMaxGradTerms; ++t) {
        a.x[t] = t < n_terms ? x[t] : 0;
        a.z[t] = t < n_terms ? z[t] : 0;
        a.pw[t] = t < n_terms ? pw[t] : 0;
    }
    a.N = uint64_t(1) << n;
    double *part = d_partials + size_t(slot0) * kRedBlocks * 2;
    if (dtype == SV_C64)
        hipLaunchKernelGGL((k_grad_terms<float, kMaxGradTerms>), dim3(kRedBlocks), dim3(kRedThreads), 0, st,
                           static_cast<const float *>(phi), static_cast<const float *>(lam), a, part);
    else
        hipLaunchKernelGGL((k_grad_terms<double, kMaxGradTerms>), dim3(kRedBlocks), dim3(kRedThreads), 0, st,
                           static_cast<const double *>(phi), static_cast<const double *>(lam), a, part);
    return hipGetLastError();
}

hipError_t launch_backward_step(int dtype, int k, const int *sorted_q, const cd *mdag, int pauli, void *phi,
                                void *lam, int n, double *d_partials, int slot, hipStream_t st)
{
    if (n < k || (pauli && k != 1)) return hipErrorInvalidValue;
    if (dtype == SV_C64) {
        float *f = static_cast<float *>(phi), *l = static_cast<float *>(lam);
        if (k == 1) return bwd_launch_t<float, 1>(sorted_q, mdag, pauli, f, l, n, d_partials, slot, st);
        if (k == 2) return bwd_launch_t<float, 2>(sorted_q, mdag, pauli, f, l, n, d_partials, slot, st);
        return hipErrorInvalidValue;
    }
    double *f = static_cast<double *>(phi), *l = static_cast<double *>(lam);
    if (k == 1) return bwd_launch_t<double, 1>(sorted_q, mdag, pauli, f, l, n, d_partials, slot, st);
    if (k == 2) return bwd_launch_t<double, 2>(sorted_q, mdag, pauli, f, l, n, d_partials, slot, st);
    return hipErrorInvalidValue;
}

}  // namespace dev
}  // namespace sv
