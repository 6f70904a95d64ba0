// Gate-application kernels for small gates and fused blocks of k <= 3 (4 for
// complex64), plus a generic kernel for any k <= 6, and state initialisation.
//
// The paper's state-vector core applies each gate as a matrix-vector product
// on the groups of amplitudes the gate couples (State Vector section).  A
// group is fixed by a base index b with zeros at the gate's positions; its
// 2^k members are b + (sum of 2^{q_j} over the set local bits).
//
// Register kernel layout (gfx950, wave64):
//   * each thread owns a CHUNK of 4 consecutive amplitudes (32 B of complex64,
//     two 16-byte loads) for every combination of the gate's HIGH positions
//     (positions >= 2); the chunk's base has zeros at those positions
//     (bit insertion);
//   * targets at positions 0 and 1 fall inside the chunk and are handled in
//     registers, so low targets need no shuffle and every load is a full,
//     contiguous 16-byte access; consecutive threads touch consecutive
//     chunks, so each of the 2^kh sub-streams is coalesced across the wave;
//   * the matrix is a kernel argument (uniform -> scalar registers), the
//     complex matvec runs in VGPRs, results are written back in place: every
//     amplitude is read once and written once per pass.
// Which of positions 0/1 are targets is a template parameter (LOWMASK) so all
// register indexing is static.
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sv {
namespace dev {

namespace {

template <int LM>
__host__ __device__ constexpr int popc2() { return (LM & 1) + ((LM >> 1) & 1); }

// deposit the low popc2<LM>() bits of m into the bit positions set in LM
template <int LM>
__device__ __forceinline__ constexpr int low_deposit(int m)
{
    return LM == 0 ? 0 : LM == 1 ? (m & 1) : LM == 2 ? ((m & 1) << 1) : (m & 3);
}

__device__ __forceinline__ void load_chunk(const float *p, float re[4], float im[4])
{
    const float4 *q = reinterpret_cast<const float4 *>(p);
    const float4 a = q[0], b = q[1];
    re[0] = a.x; im[0] = a.y; re[1] = a.z; im[1] = a.w;
    re[2] = b.x; im[2] = b.y; re[3] = b.z; im[3] = b.w;
}
__device__ __forceinline__ void store_chunk(float *p, const float re[4], const float im[4])
{
    float4 *q = reinterpret_cast<float4 *>(p);
    q[0] = make_float4(re[0], im[0], re[1], im[1]);
    q[1] = make_float4(re[2], im[2], re[3], im[3]);
}
__device__ __forceinline__ void load_chunk(const double *p, double re[4], double im[4])
{
    const double2 *q = reinterpret_cast<const double2 *>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double2 v = q[i];
        re[i] = v.x; im[i] = v.y;
    }
}
__device__ __forceinline__ void store_chunk(double *p, const double re[4], const double im[4])
{
    double2 *q = reinterpret_cast<double2 *>(p);
#pragma unroll
    for (int i = 0; i < 4; ++i) q[i] = make_double2(re[i], im[i]);
}

template <typename T, int K>
struct RegArgs {
    T mr[(1 << K) * (1 << K)];
    T mi[(1 << K) * (1 << K)];
    uint64_t n_groups;
    T *psi2;                // second state for gridDim.y = 2 (same block on both)
    int hp[K > 0 ? K : 1];  // high positions (>= 2), ascending; first kh used
};

__device__ __forceinline__ uint64_t insert_zero(uint64_t x, int p)
{
    return ((x >> p) << (p + 1)) | (x & ((uint64_t(1) << p) - 1));
}

template <typename T, int K, int LM>
__global__ void __launch_bounds__(256) k_apply_reg(T *__restrict__ psi0, const RegArgs<T, K> a)
{
    T *__restrict__ psi = blockIdx.y ? a.psi2 : psi0;
    constexpr int KL = popc2<LM>();
    constexpr int KH = K - KL;
    constexpr int NH = 1 << KH;
    constexpr int D = 1 << K;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < a.n_groups; g += stride) {
        uint64_t base = g << 2;
#pragma unroll
        for (int j = 0; j < KH; ++j) base = insert_zero(base, a.hp[j]);
        T re[NH][4], im[NH][4];
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            uint64_t o = base;
#pragma unroll
            for (int j = 0; j < KH; ++j)
                if ((h >> j) & 1) o += uint64_t(1) << a.hp[j];
            load_chunk(psi + 2 * o, re[h], im[h]);
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            if (f & LM) continue;
            T vr[D], vi[D];
#pragma unroll
            for (int m = 0; m < D; ++m) {
                const int l = f | low_deposit<LM>(m);
                vr[m] = re[m >> KL][l];
                vi[m] = im[m >> KL][l];
            }
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
                const int l = f | low_deposit<LM>(m);
                re[m >> KL][l] = sr;
                im[m >> KL][l] = si;
            }
        }
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            uint64_t o = base;
#pragma unroll
            for (int j = 0; j < KH; ++j)
                if ((h >> j) & 1) o += uint64_t(1) << a.hp[j];
            store_chunk(psi + 2 * o, re[h], im[h]);
        }
    }
}

template <typename T, int K, int LM>
hipError_t reg_launch_t(const int *sorted_q, const cd *m, T *psi, T *psi2, int n, hipStream_t st, int grid_cap)
{
    RegArgs<T, K> a;
    a.psi2 = psi2;
    constexpr int D = 1 << K;
    for (int i = 0; i < D * D; ++i) {
        a.mr[i] = T(m[i].real());
        a.mi[i] = T(m[i].imag());
    }
    int kh = 0;
    for (int j = 0; j < K; ++j)
        if (sorted_q[j] >= 2) a.hp[kh++] = sorted_q[j];
    for (int j = kh; j < K; ++j) a.hp[j] = 0;
    a.n_groups = uint64_t(1) << (n - 2 - kh);
    uint64_t blocks = (a.n_groups + 255) / 256;
    if (grid_cap > 0 && blocks > uint64_t(grid_cap)) blocks = grid_cap;
    hipLaunchKernelGGL((k_apply_reg<T, K, LM>), dim3(unsigned(blocks), psi2 ? 2 : 1), dim3(256), 0, st, psi, a);
    return hipGetLastError();
}

template <typename T, int K>
hipError_t reg_dispatch_lm(const int *sorted_q, const cd *m, T *psi, T *psi2, int n, hipStream_t st, int grid_cap)
{
    int lm = 0;
    for (int j = 0; j < K; ++j)
        if (sorted_q[j] < 2) lm |= 1 << sorted_q[j];
    switch (lm) {
    case 0: return reg_launch_t<T, K, 0>(sorted_q, m, psi, psi2, n, st, grid_cap);
    case 1: return reg_launch_t<T, K, 1>(sorted_q, m, psi, psi2, n, st, grid_cap);
    case 2: return reg_launch_t<T, K, 2>(sorted_q, m, psi, psi2, n, st, grid_cap);
    default:
        if constexpr (K >= 2) return reg_launch_t<T, K, 3>(sorted_q, m, psi, psi2, n, st, grid_cap);
        return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ generic
template <int K>
struct GenArgs {
    int pos[K];  // ascending
    uint64_t n_groups;
    void *psi2;  // second state for gridDim.y = 2 (same block on both)
};

template <typename T, int K>
__global__ void __launch_bounds__(256) k_apply_generic(T *__restrict__ psi0, const T *__restrict__ m,
                                                       const GenArgs<K> a)
{
    T *__restrict__ psi = blockIdx.y ? static_cast<T *>(a.psi2) : psi0;
    constexpr int D = 1 << K;
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t g = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; g < a.n_groups; g += stride) {
        uint64_t base = g;
#pragma unroll
        for (int j = 0; j < K; ++j) base = insert_zero(base, a.pos[j]);
        T vr[D], vi[D];
#pragma unroll
        for (int mm = 0; mm < D; ++mm) {
            uint64_t o = base;
#pragma unroll
            for (int j = 0; j < K; ++j)
                if ((mm >> j) & 1) o += uint64_t(1) << a.pos[j];
            vr[mm] = psi[2 * o];
            vi[mm] = psi[2 * o + 1];
        }
#pragma unroll
        for (int mm = 0; mm < D; ++mm) {
            T sr = 0, si = 0;
#pragma unroll
            for (int mp = 0; mp < D; ++mp) {
                const T ar = m[2 * (mm * D + mp)], ai = m[2 * (mm * D + mp) + 1];
                sr = fma(ar, vr[mp], sr);
                sr = fma(-ai, vi[mp], sr);
                si = fma(ar, vi[mp], si);
                si = fma(ai, vr[mp], si);
            }
            uint64_t o = base;
#pragma unroll
            for (int j = 0; j < K; ++j)
                if ((mm >> j) & 1) o += uint64_t(1) << a.pos[j];
            psi[2 * o] = sr;
            psi[2 * o + 1] = si;
        }
    }
}

template <typename T, int K>
hipError_t generic_launch_t(const int *sorted_q, const T *d_m, T *psi, T *psi2, int n, hipStream_t st)
{
    GenArgs<K> a;
    a.psi2 = psi2;
    for (int j = 0; j < K; ++j) a.pos[j] = sorted_q[j];
    a.n_groups = uint64_t(1) << (n - K);
    uint64_t blocks = (a.n_groups + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL((k_apply_generic<T, K>), dim3(unsigned(blocks), psi2 ? 2 : 1), dim3(256), 0, st, psi, d_m, a);
    return hipGetLastError();
}

template <typename T>
hipError_t generic_dispatch(int k, const int *sorted_q, const T *d_m, T *psi, T *psi2, int n, hipStream_t st)
{
    switch (k) {
    case 1: return generic_launch_t<T, 1>(sorted_q, d_m, psi, psi2, n, st);
    case 2: return generic_launch_t<T, 2>(sorted_q, d_m, psi, psi2, n, st);
    case 3: return generic_launch_t<T, 3>(sorted_q, d_m, psi, psi2, n, st);
    case 4: return generic_launch_t<T, 4>(sorted_q, d_m, psi, psi2, n, st);
    case 5: return generic_launch_t<T, 5>(sorted_q, d_m, psi, psi2, n, st);
    case 6: return generic_launch_t<T, 6>(sorted_q, d_m, psi, psi2, n, st);
    default: return hipErrorInvalidValue;
    }
}

// ------------------------------------------------------------------ init / copy
template <typename T>
__global__ void k_fill_basis(T *__restrict__ psi, uint64_t N, uint64_t index)
{
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
        psi[2 * i] = (i == index) ? T(1) : T(0);
        psi[2 * i + 1] = T(0);
    }
}

struct ProductArgs {
    double a[4 * 35];
    int n;
};

template <typename T>
__global__ void k_product(T *__restrict__ psi, uint64_t N, const ProductArgs a)
{
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < N; i += stride) {
        double vr = 1.0, vi = 0.0;
        for (int p = 0; p < a.n; ++p) {
            const int b = (i >> p) & 1;
            const double fr = a.a[4 * p + 2 * b], fi = a.a[4 * p + 2 * b + 1];
            const double tr = vr * fr - vi * fi;
            vi = vr * fi + vi * fr;
            vr = tr;
        }
        psi[2 * i] = T(vr);
        psi[2 * i + 1] = T(vi);
    }
}

template <typename S, typename D>
__global__ void k_convert(const S *__restrict__ src, D *__restrict__ dst, uint64_t count2)
{
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count2; i += stride)
        dst[i] = D(src[i]);
}

unsigned stream_blocks(uint64_t work)
{
    uint64_t b = (work + 255) / 256;
    return unsigned(b > 16384 ? 16384 : (b ? b : 1));
}

}  // namespace

bool reg_supported(int dtype, int k, const int *sorted_q, int n)
{
    if (k < 1 || k > (dtype == SV_C64 ? 4 : 3)) return false;
    int kh = 0;
    for (int j = 0; j < k; ++j) kh += sorted_q[j] >= 2;
    return n >= 2 + kh;
}

hipError_t launch_reg(int dtype, int k, const int *sorted_q, const cd *m, void *psi, int n,
                      hipStream_t st, int grid_cap, void *psi2)
{
    if (dtype == SV_C64) {
        float *p = static_cast<float *>(psi), *p2 = static_cast<float *>(psi2);
        switch (k) {
        case 1: return reg_dispatch_lm<float, 1>(sorted_q, m, p, p2, n, st, grid_cap);
        case 2: return reg_dispatch_lm<float, 2>(sorted_q, m, p, p2, n, st, grid_cap);
        case 3: return reg_dispatch_lm<float, 3>(sorted_q, m, p, p2, n, st, grid_cap);
        case 4: return reg_dispatch_lm<float, 4>(sorted_q, m, p, p2, n, st, grid_cap);
        default: return hipErrorInvalidValue;
        }
    }
    double *p = static_cast<double *>(psi), *p2 = static_cast<double *>(psi2);
    switch (k) {
    case 1: return reg_dispatch_lm<double, 1>(sorted_q, m, p, p2, n, st, grid_cap);
    case 2: return reg_dispatch_lm<double, 2>(sorted_q, m, p, p2, n, st, grid_cap);
    case 3: return reg_dispatch_lm<double, 3>(sorted_q, m, p, p2, n, st, grid_cap);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_generic(int dtype, int k, const int *sorted_q, const void *d_m, void *psi, int n,
                          hipStream_t st, void *psi2)
{
    if (n < k) return hipErrorInvalidValue;
    if (dtype == SV_C64)
        return generic_dispatch<float>(k, sorted_q, static_cast<const float *>(d_m), static_cast<float *>(psi),
                                       static_cast<float *>(psi2), n, st);
    return generic_dispatch<double>(k, sorted_q, static_cast<const double *>(d_m), static_cast<double *>(psi),
                                    static_cast<double *>(psi2), n, st);
}

hipError_t launch_fill_basis(int dtype, void *psi, int n, uint64_t index, hipStream_t st)
{
    const uint64_t N = uint64_t(1) << n;
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_fill_basis<float>, dim3(stream_blocks(N)), dim3(256), 0, st, static_cast<float *>(psi), N, index);
    else
        hipLaunchKernelGGL(k_fill_basis<double>, dim3(stream_blocks(N)), dim3(256), 0, st, static_cast<double *>(psi), N, index);
    return hipGetLastError();
}

hipError_t launch_product(int dtype, void *psi, int n, const double *amps, hipStream_t st)
{
    ProductArgs a;
    a.n = n;
    for (int i = 0; i < 4 * n; ++i) a.a[i] = amps[i];
    const uint64_t N = uint64_t(1) << n;
    if (dtype == SV_C64)
        hipLaunchKernelGGL(k_product<float>, dim3(stream_blocks(N)), dim3(256), 0, st, static_cast<float *>(psi), N, a);
    else
        hipLaunchKernelGGL(k_product<double>, dim3(stream_blocks(N)), dim3(256), 0, st, static_cast<double *>(psi), N, a);
    return hipGetLastError();
}

hipError_t launch_convert(int src_dtype, const void *src, int dst_dtype, void *dst, uint64_t count,
                          hipStream_t st)
{
    const uint64_t c2 = 2 * count;
    const unsigned b = stream_blocks(c2);
    if (src_dtype == SV_C64 && dst_dtype == SV_C64)
        hipLaunchKernelGGL((k_convert<float, float>), dim3(b), dim3(256), 0, st, static_cast<const float *>(src), static_cast<float *>(dst), c2);
    else if (src_dtype == SV_C64)
        hipLaunchKernelGGL((k_convert<float, double>), dim3(b), dim3(256), 0, st, static_cast<const float *>(src), static_cast<double *>(dst), c2);
    else if (dst_dtype == SV_C64)
        hipLaunchKernelGGL((k_convert<double, float>), dim3(b), dim3(256), 0, st, static_cast<const double *>(src), static_cast<float *>(dst), c2);
    else
        hipLaunchKernelGGL((k_convert<double, double>), dim3(b), dim3(256), 0, st, static_cast<const double *>(src), static_cast<double *>(dst), c2);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace sv
