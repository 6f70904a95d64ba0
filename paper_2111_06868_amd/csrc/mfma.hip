// Dense k-qubit blocks (k = 4..6) as MFMA complex GEMMs on gfx950.
//
// View the state as Psi (2^k x 2^(n-k)): row r = local index over the block's
// positions (canonical: bit j <-> j-th lowest block position), column c = the
// remaining n-k bits in ascending position order.  Applying the block is
// Psi <- U Psi, done in place one column tile at a time.
//
// Real form.  With K = 2^(k+1) interleaved real rows (2i = Re, 2i+1 = Im of
// complex row i) the complex product is one real GEMM
//     A' = [[Ur, -Ui], [Ui, Ur]] interleaved:  A'[2i+s][2j+t] =
//          s=t: Ur[i][j];  s=0,t=1: -Ui[i][j];  s=1,t=0: Ui[i][j],
// and the tile's interleaved (re, im) storage IS the interleaved B operand,
// so the staged tile feeds the matrix cores without any shuffling.
//
// Work split per workgroup (one column tile of TC = 2^TCL columns):
//   * all 2^k x TC amplitudes of the tile are copied HBM -> LDS with 16-byte
//     loads; tile-linear index t's bits map to the union of the block
//     positions and the lowest TCL non-block positions (ascending), so the
//     copy is a run of contiguous segments whatever the block positions;
//     positions 0.. of that union are contiguous, so every 16-byte load is
//     a full, aligned pair of amplitudes;
//   * the LDS tile is stored [row][column] (pitch TC + 1), i.e. transposed
//     into the GEMM layout during the copy;
//   * wave w owns M-slab w / NB (32 real rows of A', held in VGPRs for the
//     whole kernel) and N-block w % NB (32 columns); it runs 2^k
//     v_mfma_f32_32x32x2f32 (FP32) per tile, B operands read from LDS;
//   * results go back through LDS and out with 16-byte stores;
//   * the grid is persistent over tiles; the next tile's HBM loads are
//     issued before the current tile's MFMA work (register double buffer).
//
// Split precision (16-bit parts, FP32 accumulation): the host writes A' as
// three BF16 parts A' = A_0 + A_1 + A_2 (part p = RNE(A' - parts before it),
// about FP32's 24 significand bits in all) or two FP16 parts; X = Xh + Xl,
// and A'X ~ sum_p A_p Xh + A_0 Xl.  The dropped products (A_1 Xl and below:
// ~2^-16 relative for BF16, ~2^-22 for FP16) vary with X, so they do not
// add up coherently over blocks; the matrix itself is represented to about
// 2^-24, which keeps the norm.  X is split once, while staging into LDS, in
// the v_mfma_f32_32x32x16 operand layout (8 consecutive K values per lane).
// FP16 tiles are scaled by a power of two chosen from the tile's largest
// component (exact), so small amplitudes stay in FP16's normal range.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>

#include "kernels.h"

namespace sv {
namespace dev {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int kMaxTileBits = 6 + 7;

struct MfmaArgs {
    uint64_t n_tiles;
    float *psi2;                 // second state for gridDim.y = 2 (FP32 kernel: same block on both)
    int kpos[SV_MAX_K];          // block positions, ascending
    int ubit[kMaxTileBits];      // tile-linear bit b -> global position
    int lweight[kMaxTileBits];   // tile-linear bit b -> LDS element offset
};

__device__ __forceinline__ uint64_t ins0(uint64_t x, int p)
{
    return ((x >> p) << (p + 1)) | (x & ((uint64_t(1) << p) - 1));
}

template <int K>
__device__ __forceinline__ uint64_t tile_base(uint64_t T, int tcl, const MfmaArgs &a)
{
    uint64_t x = T << tcl;
#pragma unroll
    for (int j = 0; j < K; ++j) x = ins0(x, a.kpos[j]);
    return x;
}

// offsets of tile-linear index t (global element offset, LDS element offset)
template <int NBITS>
__device__ __forceinline__ void tile_offsets(uint32_t t, const MfmaArgs &a, uint64_t &g, uint32_t &l)
{
    g = 0;
    l = 0;
#pragma unroll
    for (int b = 0; b < NBITS; ++b)
        if ((t >> b) & 1) {
            g += uint64_t(1) << a.ubit[b];
            l += uint32_t(a.lweight[b]);
        }
}

// ---------------------------------------------------------------- FP32
template <int K, int TCL>
struct F32Cfg {
    static constexpr int R = 1 << K;
    static constexpr int TC = 1 << TCL;
    static constexpr int MS = (2 * R) / 32;
    static constexpr int NB = TC / 32;
    static constexpr int NW = MS * NB;
    static constexpr int THREADS = 64 * NW;
    static constexpr int P = TC + 1;                  // LDS pitch (complex)
    static constexpr int NBITS = K + TCL;
    static constexpr int IT = (R * TC) / (2 * THREADS);  // 16-byte chunks per thread
    static_assert(IT == 4, "tile shape");
};

template <int K, int TCL>
__global__ void __launch_bounds__((F32Cfg<K, TCL>::THREADS))
    k_mfma_f32(float *__restrict__ psi0, const float *__restrict__ A, const MfmaArgs args)
{
    float *__restrict__ psi = blockIdx.y ? args.psi2 : psi0;
    using C = F32Cfg<K, TCL>;
    __shared__ float2 X[C::R * C::P];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int mslab = w / C::NB, nb = w % C::NB;
    const int half = lane >> 5, l32 = lane & 31;

    // A' slab in registers: a[j] = A'[mslab*32 + l32][2j + half]
    float a[C::R];
#pragma unroll
    for (int j = 0; j < C::R; ++j) a[j] = A[(mslab * 32 + l32) * (2 * C::R) + 2 * j + half];

    // per-thread tile offsets: t = 2*tid + i*2*THREADS
    uint64_t g_lo;
    uint32_t l_lo;
    tile_offsets<C::NBITS>(uint32_t(2 * tid), args, g_lo, l_lo);
    uint64_t g_hi[C::IT];
    uint32_t l_hi[C::IT];
#pragma unroll
    for (int i = 0; i < C::IT; ++i) tile_offsets<C::NBITS>(uint32_t(i * 2 * C::THREADS), args, g_hi[i], l_hi[i]);
    const uint32_t w0 = uint32_t(args.lweight[0]);  // LDS step of tile bit 0

    uint64_t T = blockIdx.x;
    float4 buf[C::IT];
    if (T < args.n_tiles) {
        const uint64_t base = tile_base<K>(T, TCL, args);
#pragma unroll
        for (int i = 0; i < C::IT; ++i)
            buf[i] = *reinterpret_cast<const float4 *>(psi + 2 * (base + g_lo + g_hi[i]));
    }
    for (; T < args.n_tiles; T += gridDim.x) {
        const uint64_t base = tile_base<K>(T, TCL, args);
#pragma unroll
        for (int i = 0; i < C::IT; ++i) {
            const uint32_t l = l_lo + l_hi[i];
            X[l] = make_float2(buf[i].x, buf[i].y);
            X[l + w0] = make_float2(buf[i].z, buf[i].w);
        }
        __syncthreads();
        const uint64_t Tn = T + gridDim.x;
        if (Tn < args.n_tiles) {
            const uint64_t nbase = tile_base<K>(Tn, TCL, args);
#pragma unroll
            for (int i = 0; i < C::IT; ++i)
                buf[i] = *reinterpret_cast<const float4 *>(psi + 2 * (nbase + g_lo + g_hi[i]));
        }
        f32x16 acc;
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[v] = 0.f;
        const float *Xf = reinterpret_cast<const float *>(X);
        const int col = nb * 32 + l32;
#pragma unroll
        for (int j = 0; j < C::R; ++j) {
            const float b = Xf[2 * (j * C::P + col) + half];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a[j], b, acc, 0, 0, 0);
        }
        __syncthreads();
        // D row = 8*(v/4) + 4*half + v%4 (real rows); complex row = row/2
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int r0 = mslab * 16 + 4 * g + 2 * half;
            X[r0 * C::P + col] = make_float2(acc[4 * g + 0], acc[4 * g + 1]);
            X[(r0 + 1) * C::P + col] = make_float2(acc[4 * g + 2], acc[4 * g + 3]);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < C::IT; ++i) {
            const uint32_t l = l_lo + l_hi[i];
            const float2 u = X[l], v = X[l + w0];
            *reinterpret_cast<float4 *>(psi + 2 * (base + g_lo + g_hi[i])) = make_float4(u.x, u.y, v.x, v.y);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- split
__device__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even (finite inputs)
    return uint16_t(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }
__device__ __forceinline__ uint16_t f2h(float x)
{
    _Float16 h = (_Float16)x;
    uint16_t r;
    __builtin_memcpy(&r, &h, 2);
    return r;
}
__device__ __forceinline__ float h2f(uint16_t r)
{
    _Float16 h;
    __builtin_memcpy(&h, &r, 2);
    return (float)h;
}

template <bool F16>
__device__ __forceinline__ void split2(float x, uint16_t &hi, uint16_t &lo)
{
    if (F16) {
        hi = f2h(x);
        lo = f2h(x - h2f(hi));
    } else {
        hi = f2bf(x);
        lo = f2bf(x - bf2f(hi));
    }
}

template <int K, int TCL>
struct SplitCfg {
    static constexpr int R = 1 << K;
    static constexpr int TC = 1 << TCL;
    static constexpr int MS = (2 * R) / 32;
    static constexpr int NB = TC / 32;
    static constexpr int NW = MS * NB;
    static constexpr int THREADS = 64 * NW;
    static constexpr int P = TC + 1;
    static constexpr int NBITS = K + TCL;
    static constexpr int IT = (R * TC) / (2 * THREADS);
    static constexpr int NI = (2 * R) / 16;  // MFMA steps along K
    static_assert(IT == 4, "tile shape");
};

template <int K, int TCL, bool F16>
__global__ void __launch_bounds__((SplitCfg<K, TCL>::THREADS))
    k_mfma_split(float *__restrict__ psi, const uint16_t *__restrict__ A0, const uint16_t *__restrict__ A1,
                 const uint16_t *__restrict__ A2, const MfmaArgs args)
{
    constexpr int NP = F16 ? 2 : 3;  // parts of A'
    const uint16_t *const parts[3] = {A0, A1, A2};
    using C = SplitCfg<K, TCL>;
    // B operand planes: [R/4 groups][TC columns][8 halves] for hi and lo
    __shared__ uint4 Bh[(C::R / 4) * C::TC];
    __shared__ uint4 Bl[(C::R / 4) * C::TC];
    __shared__ float2 Y[C::R * C::P];
    __shared__ float wmax[C::NW];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = tid >> 6;
    const int mslab = w / C::NB, nb = w % C::NB;
    const int half = lane >> 5, l32 = lane & 31;

    // A' slab: for step i, lane holds part p of A'[mslab*32 + l32][16 i + 8 half + e], e < 8
    uint4 ap[NP][C::NI];
#pragma unroll
    for (int p = 0; p < NP; ++p)
#pragma unroll
        for (int i = 0; i < C::NI; ++i) {
            const size_t off = size_t(mslab * 32 + l32) * (2 * C::R) + 16 * i + 8 * half;
            ap[p][i] = *reinterpret_cast<const uint4 *>(parts[p] + off);
        }

    uint64_t g_lo;
    uint32_t l_lo;
    tile_offsets<C::NBITS>(uint32_t(2 * tid), args, g_lo, l_lo);
    uint64_t g_hi[C::IT];
    uint32_t l_hi[C::IT];
#pragma unroll
    for (int i = 0; i < C::IT; ++i) tile_offsets<C::NBITS>(uint32_t(i * 2 * C::THREADS), args, g_hi[i], l_hi[i]);
    const uint32_t w0 = uint32_t(args.lweight[0]);

    uint64_t T = blockIdx.x;
    float4 buf[C::IT];
    if (T < args.n_tiles) {
        const uint64_t base = tile_base<K>(T, TCL, args);
#pragma unroll
        for (int i = 0; i < C::IT; ++i)
            buf[i] = *reinterpret_cast<const float4 *>(psi + 2 * (base + g_lo + g_hi[i]));
    }
    for (; T < args.n_tiles; T += gridDim.x) {
        const uint64_t base = tile_base<K>(T, TCL, args);
        float scale = 1.f, unscale = 1.f;
        if (F16) {
            float m = 0.f;
#pragma unroll
            for (int i = 0; i < C::IT; ++i)
                m = fmaxf(m, fmaxf(fmaxf(fabsf(buf[i].x), fabsf(buf[i].y)), fmaxf(fabsf(buf[i].z), fabsf(buf[i].w))));
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
            if (lane == 0) wmax[w] = m;
            __syncthreads();
            m = 0.f;
#pragma unroll
            for (int i = 0; i < C::NW; ++i) m = fmaxf(m, wmax[i]);
            if (m > 0.f) {
                int e;
                frexpf(m, &e);  // m in [2^(e-1), 2^e)
                int s = 15 - e;  // largest component in [2^14, 2^15)
                s = s > 120 ? 120 : (s < -120 ? -120 : s);
                scale = ldexpf(1.f, s);
                unscale = ldexpf(1.f, -s);
            }
        }
#pragma unroll
        for (int i = 0; i < C::IT; ++i) {
            const uint32_t l = l_lo + l_hi[i];
            const float v[4] = {buf[i].x * scale, buf[i].y * scale, buf[i].z * scale, buf[i].w * scale};
#pragma unroll
            for (int e = 0; e < 2; ++e) {
                const uint32_t le = l + (e ? w0 : 0);  // [row][col] element index
                const uint32_t row = le / C::P, col = le % C::P;
                uint16_t hr, lr, hi_, li_;
                split2<F16>(v[2 * e], hr, lr);
                split2<F16>(v[2 * e + 1], hi_, li_);
                // B plane word: group row/4, column col, halves 2*(row%4), +1
                uint32_t *ph = reinterpret_cast<uint32_t *>(&Bh[(row >> 2) * C::TC + col]) + (row & 3);
                uint32_t *pl = reinterpret_cast<uint32_t *>(&Bl[(row >> 2) * C::TC + col]) + (row & 3);
                *ph = uint32_t(hr) | (uint32_t(hi_) << 16);
                *pl = uint32_t(lr) | (uint32_t(li_) << 16);
            }
        }
        __syncthreads();
        const uint64_t Tn = T + gridDim.x;
        if (Tn < args.n_tiles) {
            const uint64_t nbase = tile_base<K>(Tn, TCL, args);
#pragma unroll
            for (int i = 0; i < C::IT; ++i)
                buf[i] = *reinterpret_cast<const float4 *>(psi + 2 * (nbase + g_lo + g_hi[i]));
        }
        f32x16 acc;
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[v] = 0.f;
        const int col = nb * 32 + l32;
#pragma unroll
        for (int i = 0; i < C::NI; ++i) {
            const uint4 bh = Bh[(2 * i + half) * C::TC + col];
            const uint4 bl = Bl[(2 * i + half) * C::TC + col];
            if (F16) {
                f16x8 xa[NP], xb_h, xb_l;
#pragma unroll
                for (int p = 0; p < NP; ++p) __builtin_memcpy(&xa[p], &ap[p][i], 16);
                __builtin_memcpy(&xb_h, &bh, 16);
                __builtin_memcpy(&xb_l, &bl, 16);
                // A_1 is held times 2^11 (FP16's normal range): it meets X_h 2^-11
                f16x8 k11;
#pragma unroll
                for (int e = 0; e < 8; ++e) k11[e] = _Float16(0x1p-11f);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(xa[0], xb_l, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(xa[1], xb_h * k11, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_f16(xa[0], xb_h, acc, 0, 0, 0);
            } else {
                bf16x8 xa[NP], xb_h, xb_l;
#pragma unroll
                for (int p = 0; p < NP; ++p) __builtin_memcpy(&xa[p], &ap[p][i], 16);
                __builtin_memcpy(&xb_h, &bh, 16);
                __builtin_memcpy(&xb_l, &bl, 16);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[0], xb_h, acc, 0, 0, 0);
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[0], xb_l, acc, 0, 0, 0);
#pragma unroll
                for (int p = 1; p < NP; ++p) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[p], xb_h, acc, 0, 0, 0);
            }
        }
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            const int r0 = mslab * 16 + 4 * g + 2 * half;
            Y[r0 * C::P + col] = make_float2(acc[4 * g + 0] * unscale, acc[4 * g + 1] * unscale);
            Y[(r0 + 1) * C::P + col] = make_float2(acc[4 * g + 2] * unscale, acc[4 * g + 3] * unscale);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < C::IT; ++i) {
            const uint32_t l = l_lo + l_hi[i];
            const float2 u = Y[l], v = Y[l + w0];
            *reinterpret_cast<float4 *>(psi + 2 * (base + g_lo + g_hi[i])) = make_float4(u.x, u.y, v.x, v.y);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- host helpers
int fill_args(int k, int tcl, const int *sorted_q, int n, MfmaArgs &a)
{
    std::memset(&a, 0, sizeof a);
    for (int j = 0; j < k; ++j) a.kpos[j] = sorted_q[j];
    // union of block positions and the lowest tcl non-block positions
    int nb_rank = 0, b = 0;
    for (int p = 0; p < n && b < k + tcl; ++p) {
        int j = -1;
        for (int i = 0; i < k; ++i)
            if (sorted_q[i] == p) j = i;
        if (j >= 0) {
            a.ubit[b] = p;
            a.lweight[b] = (1 << j) * ((1 << tcl) + 1);  // row bit j (pitch TC + 1)
            ++b;
        } else if (nb_rank < tcl) {
            a.ubit[b] = p;
            a.lweight[b] = 1 << nb_rank;  // column bit
            ++nb_rank;
            ++b;
        }
    }
    if (b != k + tcl) return -1;
    a.n_tiles = uint64_t(1) << (n - k - tcl);
    return 0;
}

unsigned grid_for(uint64_t n_tiles, int cap)
{
    uint64_t g = n_tiles;
    if (cap > 0 && g > uint64_t(cap)) g = cap;
    return unsigned(g);
}

template <int K, int TCL>
hipError_t f32_launch(const int *q, const float *d_a, float *psi, float *psi2, int n, hipStream_t st, int cap)
{
    MfmaArgs a;
    if (fill_args(K, TCL, q, n, a)) return hipErrorInvalidValue;
    a.psi2 = psi2;
    hipLaunchKernelGGL((k_mfma_f32<K, TCL>), dim3(grid_for(a.n_tiles, cap), psi2 ? 2 : 1), dim3(F32Cfg<K, TCL>::THREADS),
                       0, st, psi, d_a, a);
    return hipGetLastError();
}

template <int K, int TCL, bool F16>
hipError_t split_launch(const int *q, const uint16_t *const *parts, float *psi, int n, hipStream_t st, int cap)
{
    MfmaArgs a;
    if (fill_args(K, TCL, q, n, a)) return hipErrorInvalidValue;
    a.psi2 = nullptr;
    hipLaunchKernelGGL((k_mfma_split<K, TCL, F16>), dim3(grid_for(a.n_tiles, cap)),
                       dim3(SplitCfg<K, TCL>::THREADS), 0, st, psi, parts[0], parts[1], parts[2], a);
    return hipGetLastError();
}

uint16_t host_f2bf(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
float host_bf2f(uint16_t h)
{
    uint32_t u = uint32_t(h) << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}
uint16_t host_f2h(float x)
{
    _Float16 h = (_Float16)x;
    uint16_t r;
    std::memcpy(&r, &h, 2);
    return r;
}
float host_h2f(uint16_t r)
{
    _Float16 h;
    std::memcpy(&h, &r, 2);
    return (float)h;
}

}  // namespace

bool mfma_supported(int k, int n) { return k >= 4 && k <= 6 && n - k >= 5; }

size_t real_form_elems(int k)
{
    const size_t R2 = size_t(2) << k;
    return R2 * R2;
}

void pack_real_form_f32(const cd *m, int k, float *out)
{
    const int R = 1 << k, R2 = 2 * R;
    for (int i = 0; i < R; ++i)
        for (int j = 0; j < R; ++j) {
            const double ur = m[size_t(i) * R + j].real(), ui = m[size_t(i) * R + j].imag();
            out[size_t(2 * i) * R2 + 2 * j] = float(ur);
            out[size_t(2 * i) * R2 + 2 * j + 1] = float(-ui);
            out[size_t(2 * i + 1) * R2 + 2 * j] = float(ui);
            out[size_t(2 * i + 1) * R2 + 2 * j + 1] = float(ur);
        }
}

void pack_real_form_split(const cd *m, int k, bool fp16, uint16_t *const *parts)
{
    const int R = 1 << k, R2 = 2 * R;
    const int np = fp16 ? 2 : 3;
    for (int i = 0; i < R; ++i)
        for (int j = 0; j < R; ++j) {
            const double ur = m[size_t(i) * R + j].real(), ui = m[size_t(i) * R + j].imag();
            const double v[2][2] = {{ur, -ui}, {ui, ur}};
            for (int s = 0; s < 2; ++s)
                for (int t = 0; t < 2; ++t) {
                    const size_t o = size_t(2 * i + s) * R2 + 2 * j + t;
                    double x = v[s][t];  // part p = RNE(x - parts before it)
                    for (int p = 0; p < 3; ++p) {
                        if (p >= np) {
                            parts[p][o] = 0;
                            continue;
                        }
                        if (fp16) {  // the second part held times 2^11
                            const double f = p ? 2048.0 : 1.0;
                            parts[p][o] = host_f2h(float(x * f));
                            x -= double(host_h2f(parts[p][o])) / f;
                        } else {
                            parts[p][o] = host_f2bf(float(x));
                            x -= double(host_bf2f(parts[p][o]));
                        }
                    }
                }
        }
}

hipError_t launch_mfma_f32(int k, const int *q, const float *d_a, void *psi, int n, hipStream_t st, int tcl,
                           int cap, void *psi2)
{
    if (!mfma_supported(k, n)) return hipErrorInvalidValue;
    if (tcl > n - k) tcl = n - k;
    float *p = static_cast<float *>(psi), *p2 = static_cast<float *>(psi2);
#define SV_F32_CASE(KK, TT) \
    if (k == KK && tcl == TT) return f32_launch<KK, TT>(q, d_a, p, p2, n, st, cap);
    SV_F32_CASE(4, 5) SV_F32_CASE(4, 6) SV_F32_CASE(4, 7)
    SV_F32_CASE(5, 5) SV_F32_CASE(5, 6) SV_F32_CASE(5, 7)
    SV_F32_CASE(6, 5) SV_F32_CASE(6, 6)
#undef SV_F32_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_mfma_split(int k, bool fp16, const int *q, const uint16_t *const *d_parts, void *psi, int n,
                             hipStream_t st, int tcl, int cap)
{
    if (!mfma_supported(k, n)) return hipErrorInvalidValue;
    if (tcl > n - k) tcl = n - k;
    float *p = static_cast<float *>(psi);
#define SV_SPLIT_CASE(KK, TT)                                                                       \
    if (k == KK && tcl == TT)                                                                       \
        return fp16 ? split_launch<KK, TT, true>(q, d_parts, p, n, st, cap)                         \
                    : split_launch<KK, TT, false>(q, d_parts, p, n, st, cap);
    SV_SPLIT_CASE(4, 5) SV_SPLIT_CASE(4, 6) SV_SPLIT_CASE(4, 7)
    SV_SPLIT_CASE(5, 5) SV_SPLIT_CASE(5, 6)
    SV_SPLIT_CASE(6, 5) SV_SPLIT_CASE(6, 6)
#undef SV_SPLIT_CASE
    return hipErrorInvalidValue;
}

}  // namespace dev
}  // namespace sv
