// Multi-block tile passes: several consecutive fused 4-qubit blocks applied
// to a state in ONE read and ONE write of HBM.
//
// The blocks of a pass act on a union U of at most 8 positions.  A tile is
// the 2^TB amplitudes (TB = 13 or 14: 64 or 128 KiB of complex64 in LDS)
// spanned by U plus the lowest TB - |U| positions outside U (tile bit b <->
// position u_b, ascending); at least 5 low positions join, so the tile is
// made of contiguous runs of >= 32 amplitudes (256 B).  For every value of
// the remaining n - TB bits there is one tile; tiles are copied in and out
// with 16-byte accesses along those runs (tile bit 0 is always position 0).
//
// Inside the tile, block s (4 positions at tile bits t_s0 < .. < t_s3) is a
// complex GEMM Y = U_s X with X viewed as 16 rows (the block's tile bits) x
// 2^(TB-4) columns (the other tile bits): one v_mfma_f32_32x32x2f32 chain per
// 32-column block, the real form A' = [[Ur,-Ui],[Ui,Ur]] interleaved by
// (re, im) held in VGPRs (16 per lane per block) for the whole persistent
// kernel, B operands and results addressed in LDS as row_offset(j) +
// column_offset(c) (bit deposits).  Each wave owns whole columns, so blocks
// update the tile in place with one barrier between blocks.
#include <hip/hip_runtime.h>

#include <cstring>

#include "kernels.h"

namespace sv {
namespace dev {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kMaxTileBits = 14;
constexpr int kTileThreads = 512;
constexpr int kTileWaves = kTileThreads / 64;

// Tile of 2^TB amplitudes: 2^TB / 16 columns per 4-qubit block, split over 8 waves.
template <int TB>
struct TileCfg {
    static constexpr int N = 1 << TB;
    static constexpr int COLS = N / 16;
    static constexpr int NB_PER_WAVE = COLS / 32 / kTileWaves;
    static constexpr int CHUNKS = N / 2 / kTileThreads;  // 16-byte copies per thread
};

struct TileArgs {
    uint64_t n_tiles;
    int ubit[kMaxTileBits];            // tile bit -> global position
    int ext_pos[SV_MAX_QUBITS_C64];    // positions outside the tile, ascending
    int n_ext;
    int tbit[kMaxTileSubBlocks][4];    // per block: its tile bits, ascending
};

__device__ __forceinline__ uint32_t deposit(uint32_t v, uint32_t mask)
{
    // scatter the low bits of v into the set bits of mask (ascending)
    uint32_t r = 0;
    for (uint32_t m = mask; m; m &= m - 1) {
        const uint32_t low = m & (~m + 1);
        if (v & 1) r |= low;
        v >>= 1;
    }
    return r;
}

__device__ __forceinline__ uint64_t tile_base(uint64_t T, const TileArgs &a)
{
    // the tile index's bits go to the positions outside the tile, ascending
    uint64_t x = 0;
    for (int i = 0; i < a.n_ext; ++i) x |= ((T >> i) & 1) << a.ext_pos[i];
    return x;
}

template <int TB>
__device__ __forceinline__ uint64_t global_off(uint32_t t, const TileArgs &a)
{
    uint64_t g = 0;
#pragma unroll
    for (int b = 0; b < TB; ++b)
        if ((t >> b) & 1) g += uint64_t(1) << a.ubit[b];
    return g;
}

template <int TB, int NSUB>
__global__ void __launch_bounds__(kTileThreads) k_tile_pass(float *__restrict__ psi, const float *__restrict__ A,
                                                            const TileArgs args)
{
    using C = TileCfg<TB>;
    constexpr int kTileN = C::N;
    constexpr int kNBPerWave = C::NB_PER_WAVE;
    constexpr int kChunks = C::CHUNKS;
    __shared__ float2 X[kTileN];
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int half = lane >> 5, l32 = lane & 31;

    // A' of every block in registers: a[s][j] = A'_s[l32][2j + half]
    float a[NSUB][16];
#pragma unroll
    for (int s = 0; s < NSUB; ++s)
#pragma unroll
        for (int j = 0; j < 16; ++j) a[s][j] = A[s * 1024 + l32 * 32 + 2 * j + half];

    // LDS offsets: row_off[s][j] (uniform) and this lane's column offsets
    uint32_t col_off[NSUB][kNBPerWave];
    uint32_t row_mask[NSUB];
#pragma unroll
    for (int s = 0; s < NSUB; ++s) {
        uint32_t m = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) m |= 1u << args.tbit[s][i];
        row_mask[s] = m;
#pragma unroll
        for (int q = 0; q < kNBPerWave; ++q)
            col_off[s][q] = deposit(uint32_t((w * kNBPerWave + q) * 32 + l32), (kTileN - 1) & ~m);
    }

    // copy offsets: chunk i of this thread covers tile index t = 2*(tid + i*kTileThreads)
    uint64_t g_lo = global_off<TB>(uint32_t(2 * tid), args);
    uint64_t g_hi[kChunks];
#pragma unroll
    for (int i = 0; i < kChunks; ++i) g_hi[i] = global_off<TB>(uint32_t(2 * i * kTileThreads), args);

    uint64_t T = blockIdx.x;
    float4 buf[kChunks];
    if (T < args.n_tiles) {
        const uint64_t base = tile_base(T, args) + g_lo;
#pragma unroll
        for (int i = 0; i < kChunks; ++i) buf[i] = *reinterpret_cast<const float4 *>(psi + 2 * (base + g_hi[i]));
    }
    for (; T < args.n_tiles; T += gridDim.x) {
        const uint64_t base = tile_base(T, args) + g_lo;
#pragma unroll
        for (int i = 0; i < kChunks; ++i)
            reinterpret_cast<float4 *>(X)[tid + i * kTileThreads] = buf[i];
        __syncthreads();
        const uint64_t Tn = T + gridDim.x;
        if (Tn < args.n_tiles) {
            const uint64_t nbase = tile_base(Tn, args) + g_lo;
#pragma unroll
            for (int i = 0; i < kChunks; ++i) buf[i] = *reinterpret_cast<const float4 *>(psi + 2 * (nbase + g_hi[i]));
        }
        const float *Xf = reinterpret_cast<const float *>(X);
#pragma unroll
        for (int s = 0; s < NSUB; ++s) {
            uint32_t row_off[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) row_off[j] = deposit(uint32_t(j), row_mask[s]);
            // the wave's column blocks run as independent MFMA chains (ILP)
            f32x16 acc[kNBPerWave];
#pragma unroll
            for (int q = 0; q < kNBPerWave; ++q)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[q][v] = 0.f;
#pragma unroll
            for (int j = 0; j < 16; ++j)
#pragma unroll
                for (int q = 0; q < kNBPerWave; ++q)
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[s][j], Xf[2 * (row_off[j] + col_off[s][q]) + half],
                                                                  acc[q], 0, 0, 0);
            // D real row = 8*(v/4) + 4*half + v%4; complex row = real row / 2
#pragma unroll
            for (int q = 0; q < kNBPerWave; ++q) {
                const uint32_t co = col_off[s][q];
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int r0 = 4 * g + 2 * half;
                    X[row_off[r0] + co] = make_float2(acc[q][4 * g + 0], acc[q][4 * g + 1]);
                    X[row_off[r0 + 1] + co] = make_float2(acc[q][4 * g + 2], acc[q][4 * g + 3]);
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < kChunks; ++i)
            *reinterpret_cast<float4 *>(psi + 2 * (base + g_hi[i])) = reinterpret_cast<const float4 *>(X)[tid + i * kTileThreads];
        __syncthreads();
    }
}


// Split-BF16 variant: A' = Ah + Al (bf16, from the host), each B operand
// (8 consecutive K values = 4 complex rows of one column) is split while it
// is read from LDS (v_cvt_pk_bf16_f32), and Ah Xh + Ah Xl + Al Xh run on
// v_mfma_f32_32x32x16_bf16 with FP32 accumulation (the Al Xl term, ~2^-16
// relative, is dropped).  Everything else is as in k_tile_pass.
template <int TB, int NSUB>
__global__ void __launch_bounds__(kTileThreads) k_tile_pass_bf16(float *__restrict__ psi,
                                                                 const uint16_t *__restrict__ A,
                                                                 const TileArgs args)
{
    using C = TileCfg<TB>;
    constexpr int kTileN = C::N;
    constexpr int kNBPerWave = C::NB_PER_WAVE;
    constexpr int kChunks = C::CHUNKS;
    __shared__ float2 X[kTileN];
    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int half = lane >> 5, l32 = lane & 31;

    // A' hi / lo: step i (K = 16 i .. 16 i + 15), lane holds A'[l32][16 i + 8 half + e]
    uint4 ah[NSUB][2], al[NSUB][2];
#pragma unroll
    for (int s = 0; s < NSUB; ++s)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int off = s * 2048 + l32 * 32 + 16 * i + 8 * half;
            ah[s][i] = *reinterpret_cast<const uint4 *>(A + off);
            al[s][i] = *reinterpret_cast<const uint4 *>(A + off + 1024);
        }

    uint32_t col_off[NSUB][kNBPerWave];
    uint32_t row_mask[NSUB];
#pragma unroll
    for (int s = 0; s < NSUB; ++s) {
        uint32_t m = 0;
#pragma unroll
        for (int i = 0; i < 4; ++i) m |= 1u << args.tbit[s][i];
        row_mask[s] = m;
#pragma unroll
        for (int q = 0; q < kNBPerWave; ++q)
            col_off[s][q] = deposit(uint32_t((w * kNBPerWave + q) * 32 + l32), (kTileN - 1) & ~m);
    }
    uint64_t g_lo = global_off<TB>(uint32_t(2 * tid), args);
    uint64_t g_hi[kChunks];
#pragma unroll
    for (int i = 0; i < kChunks; ++i) g_hi[i] = global_off<TB>(uint32_t(2 * i * kTileThreads), args);

    uint64_t T = blockIdx.x;
    float4 buf[kChunks];
    if (T < args.n_tiles) {
        const uint64_t base = tile_base(T, args) + g_lo;
#pragma unroll
        for (int i = 0; i < kChunks; ++i) buf[i] = *reinterpret_cast<const float4 *>(psi + 2 * (base + g_hi[i]));
    }
    for (; T < args.n_tiles; T += gridDim.x) {
        const uint64_t base = tile_base(T, args) + g_lo;
#pragma unroll
        for (int i = 0; i < kChunks; ++i)
            reinterpret_cast<float4 *>(X)[tid + i * kTileThreads] = buf[i];
        __syncthreads();
        const uint64_t Tn = T + gridDim.x;
        if (Tn < args.n_tiles) {
            const uint64_t nbase = tile_base(Tn, args) + g_lo;
#pragma unroll
            for (int i = 0; i < kChunks; ++i) buf[i] = *reinterpret_cast<const float4 *>(psi + 2 * (nbase + g_hi[i]));
        }
#pragma unroll
        for (int s = 0; s < NSUB; ++s) {
            uint32_t row_off[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) row_off[j] = deposit(uint32_t(j), row_mask[s]);
            f32x16 acc[kNBPerWave];
#pragma unroll
            for (int q = 0; q < kNBPerWave; ++q)
#pragma unroll
                for (int v = 0; v < 16; ++v) acc[q][v] = 0.f;
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                bf16x8 xah, xal;
                __builtin_memcpy(&xah, &ah[s][i], 16);
                __builtin_memcpy(&xal, &al[s][i], 16);
#pragma unroll
                for (int q = 0; q < kNBPerWave; ++q) {
                    bf16x8 bh, bl;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        // complex row 8 i + 4 half + t of this lane's column
                        const uint32_t r = half ? row_off[8 * i + 4 + t] : row_off[8 * i + t];
                        const float2 v = X[r + col_off[s][q]];
                        const __bf16 hr = (__bf16)v.x, hi = (__bf16)v.y;
                        bh[2 * t] = hr;
                        bh[2 * t + 1] = hi;
                        bl[2 * t] = (__bf16)(v.x - (float)hr);
                        bl[2 * t + 1] = (__bf16)(v.y - (float)hi);
                    }
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xah, bh, acc[q], 0, 0, 0);
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xah, bl, acc[q], 0, 0, 0);
                    acc[q] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xal, bh, acc[q], 0, 0, 0);
                }
            }
            // each wave owns its columns: its reads precede its writes
#pragma unroll
            for (int q = 0; q < kNBPerWave; ++q) {
                const uint32_t co = col_off[s][q];
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int r0 = 4 * g + 2 * half;
                    X[row_off[r0] + co] = make_float2(acc[q][4 * g + 0], acc[q][4 * g + 1]);
                    X[row_off[r0 + 1] + co] = make_float2(acc[q][4 * g + 2], acc[q][4 * g + 3]);
                }
            }
            __syncthreads();
        }
#pragma unroll
        for (int i = 0; i < kChunks; ++i)
            *reinterpret_cast<float4 *>(psi + 2 * (base + g_hi[i])) = reinterpret_cast<const float4 *>(X)[tid + i * kTileThreads];
        __syncthreads();
    }
}

template <int TB, int NSUB>
hipError_t tile_launch(const TileArgs &a, const void *d_a, bool split, float *psi, hipStream_t st, int cap)
{
    uint64_t g = a.n_tiles;
    if (cap > 0 && g > uint64_t(cap)) g = cap;
    if (split)
        hipLaunchKernelGGL((k_tile_pass_bf16<TB, NSUB>), dim3(unsigned(g)), dim3(kTileThreads), 0, st, psi,
                           static_cast<const uint16_t *>(d_a), a);
    else
        hipLaunchKernelGGL((k_tile_pass<TB, NSUB>), dim3(unsigned(g)), dim3(kTileThreads), 0, st, psi,
                           static_cast<const float *>(d_a), a);
    return hipGetLastError();
}

template <int TB>
hipError_t tile_dispatch(int n_sub, const TileArgs &a, const void *d_a, bool split, float *psi, hipStream_t st, int cap)
{
    switch (n_sub) {
    case 1: return tile_launch<TB, 1>(a, d_a, split, psi, st, cap);
    case 2: return tile_launch<TB, 2>(a, d_a, split, psi, st, cap);
    case 3: return tile_launch<TB, 3>(a, d_a, split, psi, st, cap);
    case 4: return tile_launch<TB, 4>(a, d_a, split, psi, st, cap);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

bool tile_supported(int n, int union_bits) { return n >= kMinTileQubits && union_bits <= kMaxTileUnion; }

hipError_t launch_tile_pass(int n_sub, const int (*sub_pos)[4], const void *d_a, bool split_bf16, void *psi, int n,
                            hipStream_t st, int grid_cap, int tile_bits)
{
    const int kTileBits = tile_bits;
    if (tile_bits != 13 && tile_bits != 14) return hipErrorInvalidValue;
    if (n_sub < 1 || n_sub > kMaxTileSubBlocks || n < kTileBits) return hipErrorInvalidValue;
    TileArgs a;
    std::memset(&a, 0, sizeof a);
    uint64_t umask = 0;
    for (int s = 0; s < n_sub; ++s)
        for (int i = 0; i < 4; ++i) umask |= uint64_t(1) << sub_pos[s][i];
    const int nu = __builtin_popcountll(umask);
    if (nu > kMaxTileUnion) return hipErrorInvalidValue;
    // tile positions: the union plus the lowest positions outside it
    uint64_t tmask = umask;
    for (int p = 0; p < n && __builtin_popcountll(tmask) < kTileBits; ++p) tmask |= uint64_t(1) << p;
    int b = 0;
    for (int p = 0; p < n; ++p) {
        if ((tmask >> p) & 1) a.ubit[b++] = p;
        else a.ext_pos[a.n_ext++] = p;
    }
    for (int s = 0; s < n_sub; ++s)
        for (int i = 0; i < 4; ++i) {
            int t = 0;
            while (a.ubit[t] != sub_pos[s][i]) ++t;
            a.tbit[s][i] = t;
        }
    a.n_tiles = uint64_t(1) << (n - kTileBits);
    float *p = static_cast<float *>(psi);
    return tile_bits == 13 ? tile_dispatch<13>(n_sub, a, d_a, split_bf16, p, st, grid_cap)
                           : tile_dispatch<14>(n_sub, a, d_a, split_bf16, p, st, grid_cap);
}

}  // namespace dev
}  // namespace sv
