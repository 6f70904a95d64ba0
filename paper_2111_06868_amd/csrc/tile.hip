// Multi-block tile passes: a sequence of fused blocks of <= 4 qubits applied
// to a state in ONE read and ONE write of HBM.
//
// The blocks of a pass act on a union U of at most TB positions.  A tile is
// the 2^TB amplitudes (TB = 13 or 14: 64 or 128 KiB of complex64 in LDS)
// spanned by U plus the lowest TB - |U| positions outside U (tile bit b <->
// position u_b, ascending), so it is made of contiguous runs of at least
// 2^(TB - |U|) amplitudes, longer when U holds low positions.  For every value of the remaining n - TB bits there
// is one tile; tiles are copied in and out with 16-byte accesses along those
// runs (tile bit 0 is always position 0).
//
// Inside the tile, block s (4 positions at tile bits t_s0 < .. < t_s3) is a
// complex GEMM Y = U_s X with X viewed as 16 rows (the block's tile bits) x
// 2^(TB-4) columns (the other tile bits): one MFMA chain per 32-column block,
// the real form A' = [[Ur,-Ui],[Ui,Ur]] interleaved by (re, im) as the A
// operand.  The operands of all blocks of the pass, expanded into each
// lane's A' fragments, and their column address tables are staged into LDS
// once per workgroup next to the tile.
// B operands and results are addressed in LDS as row(j) XOR column(c) (bit
// deposits, then an XOR swizzle against bank conflicts).  Each wave owns
// whole columns, so blocks update the tile in place with one barrier between
// blocks.
#include <hip/hip_runtime.h>

#include <cstring>
#include <type_traits>

#include "kernels.h"

namespace sv {
namespace dev {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float vf4 __attribute__((ext_vector_type(4)));
typedef float vf2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));

// Arithmetic of a tile pass: FP32 MFMA, or hi + lo split products in BF16 or
// FP16 (FP32 accumulation).
constexpr int kPrecF32 = kTileOperandF32, kPrecBF16 = kTileOperandBF16, kPrecF16 = kTileOperandF16,
              kPrecBF16X3 = kTileOperandBF16X3;

// LDS words per lane of one block's operand (the A' fragments of the 64
// lanes, expanded at staging so that the block loop reads them as they are):
// FP32 16, split 8 per matrix part (FP16: two parts, BF16: three).  The
// smaller FP32 and FP16 operands let more blocks share a launch.
constexpr int lane_words(int prec) { return prec == kPrecBF16 || prec == kPrecBF16X3 ? 24 : 16; }

// 16-byte chunk c of lane L's fragments sits at chunk c ^ frag_swz<LW>(L) of
// its LW words.  With 64-byte lanes (LW = 16) the lanes of one 16-byte LDS
// access (8 over 32 banks, or 16 over 64) would otherwise meet four to a
// bank group; the XOR with lane bits (1 ^ 3, 2) puts them on distinct banks.
// The 96-byte lanes of split BF16 (two to a group) stay in order: the same
// XOR there (lane bits 2 ^ 3) costs those kernels register spills.
template <int LW>
__device__ __forceinline__ uint32_t frag_swz(uint32_t lane)
{
    if constexpr (LW == 16) return (((lane >> 1) ^ (lane >> 3)) & 1u) | ((lane >> 1) & 2u);
    return 0u;
}

// Tile of 2^TB amplitudes held by a workgroup of WAVES waves: 2^TB / 16
// columns per 4-qubit block, in blocks of 32 split evenly over the waves.
// Shapes: (14, 8) and (14, 16) one 128 KiB tile per CU, with 2 or 4 waves
// per SIMD; (13, 4) two 64 KiB workgroups per CU, so one can copy while the
// other computes; (13, 8).  MAX_SUB blocks' operands of LW words per lane
// fit in the LDS left beside the tile.
template <int TB, int WAVES, int LW = 24>
struct TileCfg {
    static constexpr int N = 1 << TB;
    static constexpr int THREADS = 64 * WAVES;
    static constexpr int COLS = N / 16;
    static constexpr int CBLOCKS = COLS / 32;  // 32-column blocks
    static constexpr int NB_PER_WAVE = CBLOCKS / WAVES;
    static constexpr int CHUNKS = N / 2 / THREADS;  // 16-byte copies per thread
    static constexpr int TABLE_WORDS = CBLOCKS + 32;
    // two (13, 4) workgroups share a CU; the others hold the CU alone
    static constexpr int LDS_BUDGET = (TB == 13 && WAVES == 4) ? 160 * 1024 / 2 : 160 * 1024;
    static constexpr int OPERAND_WORDS = 64 * LW;
    static constexpr int FIT = (LDS_BUDGET - N * 8 - 8 * WAVES) / (4 * (OPERAND_WORDS + TABLE_WORDS));
    static constexpr int MAX_SUB = FIT < kMaxTileSubBlocks ? FIT : kMaxTileSubBlocks;
    static_assert(THREADS % 256 == 0 && THREADS <= 1024 && NB_PER_WAVE >= 1, "tile shape");
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

// LDS placement of tile index i: S(i), linear over XOR, with image a.swz[b]
// of tile bit b (chosen per pass on the host, choose_swizzle).  S keeps bit 0,
// so the pair (2t, 2t + 1) stays one aligned 16-byte slot for the HBM copies,
// and permutes the tile's indices.
__device__ __forceinline__ uint32_t swz(uint32_t i, const TileArgs &a)
{
    uint32_t r = 0;
#pragma unroll
    for (int b = 0; b < kMaxTileBits; ++b)
        if ((i >> b) & 1) r ^= a.swz[b];
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

// Swizzled LDS index of complex row j (compile-time after unrolling) of a
// block: the XOR of the per-row-bit values rb[0..3].
__device__ __forceinline__ uint32_t row_of(const uint32_t *rb, int j)
{
    uint32_t r = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b)
        if ((j >> b) & 1) r ^= rb[b];
    return r;
}

// HBM <-> LDS copies of one tile: thread tid moves float4 slots
// tid + i * THREADS, i.e. tile indices 2 * slot and 2 * slot + 1.
template <int TB, int WAVES>
struct TileCopy {
    static constexpr int kChunks = TileCfg<TB, WAVES>::CHUNKS;
    static constexpr int kThreads = TileCfg<TB, WAVES>::THREADS;
    uint64_t g_lo;               // global offset of tile index 2 * tid
    uint64_t g_hi[kChunks];      // uniform: offset of tile index 2 * i * THREADS
    uint32_t lds_slot;           // float4 slot of tile index 2 * tid: S(2 tid) / 2
    uint32_t lds_hi[kChunks];    // uniform: S(2 i THREADS) / 2, XORed onto lds_slot

    __device__ __forceinline__ void init(const TileArgs &args, int tid)
    {
        g_lo = global_off<TB>(uint32_t(2 * tid), args);
#pragma unroll
        for (int i = 0; i < kChunks; ++i) {
            g_hi[i] = global_off<TB>(uint32_t(2 * i * kThreads), args);
            lds_hi[i] = swz(uint32_t(2 * i * kThreads), args) >> 1;
        }
        lds_slot = swz(uint32_t(2 * tid), args) >> 1;
    }
    __device__ __forceinline__ void load(vf4 *buf, const float *psi, uint64_t base) const
    {
#pragma unroll
        for (int i = 0; i < kChunks; ++i) buf[i] = *reinterpret_cast<const vf4 *>(psi + 2 * (base + g_lo + g_hi[i]));
    }
    // The same tile of a basis state, read from nowhere: zeros, and 1 at tile
    // index t when the basis state lies in this tile (`here`).  Thread tid's
    // chunk i holds tile indices 2 (tid + i THREADS) and the next one.
    __device__ __forceinline__ void basis(vf4 *buf, bool here, uint32_t t, int tid) const
    {
        const uint32_t pair = t >> 1;
#pragma unroll
        for (int i = 0; i < kChunks; ++i) {
            buf[i] = vf4{0.f, 0.f, 0.f, 0.f};
            if (here && pair == uint32_t(tid) + uint32_t(i) * kThreads) {
                if (t & 1u)
                    buf[i].z = 1.f;
                else
                    buf[i].x = 1.f;
            }
        }
    }
    // The same with a scale for the values in LDS (exact powers of two): LDS =
    // buf * scale, out = LDS * unscale.
    __device__ __forceinline__ void to_lds_scaled(vf4 *X4, const vf4 *buf, float scale) const
    {
#pragma unroll
        for (int i = 0; i < kChunks; ++i) X4[lds_slot ^ lds_hi[i]] = buf[i] * scale;
    }
    __device__ __forceinline__ void store_scaled(float *psi, uint64_t base, const vf4 *X4, float unscale) const
    {
#pragma unroll
        for (int i = 0; i < kChunks; ++i)
            *reinterpret_cast<vf4 *>(psi + 2 * (base + g_lo + g_hi[i])) = X4[lds_slot ^ lds_hi[i]] * unscale;
    }
    __device__ __forceinline__ void swap_scaled(float *psi, uint64_t base_out, vf4 *X4, const vf4 *buf, float scale,
                                                float unscale) const
    {
#pragma unroll
        for (int i = 0; i < kChunks; ++i) {
            const vf4 o = X4[lds_slot ^ lds_hi[i]];
            X4[lds_slot ^ lds_hi[i]] = buf[i] * scale;
            *reinterpret_cast<vf4 *>(psi + 2 * (base_out + g_lo + g_hi[i])) = o * unscale;
        }
    }
    // sum of the squares of the values in buf
    __device__ __forceinline__ float sum_sq(const vf4 *buf) const
    {
        float a = 0.f;
#pragma unroll
        for (int i = 0; i < kChunks; ++i)
            a += buf[i].x * buf[i].x + buf[i].y * buf[i].y + buf[i].z * buf[i].z + buf[i].w * buf[i].w;
        return a;
    }
    __device__ __forceinline__ void to_lds(vf4 *X4, const vf4 *buf) const
    {
#pragma unroll
        for (int i = 0; i < kChunks; ++i) X4[lds_slot ^ lds_hi[i]] = buf[i];
    }
    __device__ __forceinline__ void store(float *psi, uint64_t base, const vf4 *X4) const
    {
#pragma unroll
        for (int i = 0; i < kChunks; ++i)
            *reinterpret_cast<vf4 *>(psi + 2 * (base + g_lo + g_hi[i])) = X4[lds_slot ^ lds_hi[i]];
    }
    // Each slot: store the finished tile's value (at base_out) and put the
    // next tile's value in its place.  The thread owns its slots, so no
    // barrier is needed between the two.
    __device__ __forceinline__ void swap(float *psi, uint64_t base_out, vf4 *X4, const vf4 *buf) const
    {
#pragma unroll
        for (int i = 0; i < kChunks; ++i) {
            const vf4 o = X4[lds_slot ^ lds_hi[i]];
            X4[lds_slot ^ lds_hi[i]] = buf[i];
            *reinterpret_cast<vf4 *>(psi + 2 * (base_out + g_lo + g_hi[i])) = o;
        }
    }
    // largest magnitude of the values in buf
    __device__ __forceinline__ float max_abs(const vf4 *buf) const
    {
        float a = 0.f;
#pragma unroll
        for (int i = 0; i < kChunks; ++i)
            a = fmaxf(a, fmaxf(fmaxf(fabsf(buf[i].x), fabsf(buf[i].y)), fmaxf(fabsf(buf[i].z), fabsf(buf[i].w))));
        return a;
    }
};

// FP16 passes scale the tile's values by 2^e where they are split, e chosen
// from the tile's largest magnitude m (at copy-in) so that m 2^e lies in
// [2^7, 2^8), and scale the products back by 2^-e (exact powers of two).  The
// blocks act unitarily on the tile, so no value can grow beyond the tile's
// 2-norm, which is at most sqrt(2^15) m: every scaled value stays below
// 2^15.5 < 65504 (the FP16 parts stay finite) while values many binades below
// m stay in FP16's normal range.
__device__ __forceinline__ void tile_scale(float m, float &scale, float &unscale)
{
    scale = unscale = 1.f;
    if (m > 0.f && m <= 3.0e38f) {
        int e;
        frexpf(m, &e);  // m in [2^(e-1), 2^e)
        int s = 8 - e;
        s = s > 120 ? 120 : (s < -120 ? -120 : s);
        scale = ldexpf(1.f, s);
        unscale = ldexpf(1.f, -s);
    }
}

// A scale for a whole pass of FP16 products from the state's 2-norm r (the
// blocks keep it): 2^e with r 2^e in [2^14, 2^15), so that no value, being at
// most r in magnitude, exceeds 2^15 once scaled.  Scale 1 if r is 0 or not
// finite.
__device__ __forceinline__ void norm_scale(double r, float &scale, float &unscale)
{
    scale = unscale = 1.f;
    if (r > 0.0 && r <= 1e300) {
        int e;
        frexp(r, &e);  // r in [2^(e-1), 2^e)
        int s = 15 - e;
        s = s > 120 ? 120 : (s < -120 ? -120 : s);
        scale = ldexpf(1.f, s);
        unscale = ldexpf(1.f, -s);
    }
}

// Per-block data staged in LDS: the A operand and the swizzled column terms
// of lane l32 and column block cb = w NBW + q of wave w: cq[cb] ^ cl[l32].
// Column index c (deposited into the block's column bits, ascending):
// FP32 c = 32 cb + l32; split c = (32 w + l32) NBW + q, which puts q on the
// lowest column bits, so that when tile bit 0 is a column bit the column
// blocks q and q + 1 of a lane share one 16-byte slot.
template <int TB, int WAVES, int LW>
struct TileShared {
    using C = TileCfg<TB, WAVES, LW>;
    vf4 X4[C::N / 2];
    uint32_t op[C::MAX_SUB][C::OPERAND_WORDS];
    uint32_t cq[C::MAX_SUB][C::CBLOCKS];
    uint32_t cl[C::MAX_SUB][32];
    float red[WAVES];  // per-wave partial of the next tile's scale (FP16 passes)
    float nrm[WAVES];  // per-wave sum of squares read so far (FP16 passes that report the norm)
};

// Stage the launch's blocks: each lane's A' fragments, expanded from the
// compact operands (pack_tile_operand) into lane_words(PREC) consecutive
// words per lane, and the column tables.  Lane (half, l32) takes row r = l32 of A' =
// [[Ur,-Ui],[Ui,Ur]] interleaved by (re, im): complex row ci = r / 2, part
// ri = r % 2.
//   FP32: word j < 16 = A'[r][2 j + half], i.e. Ur[ci][j] (ri == half),
//   -Ui[ci][j] (ri = 0, half = 1) or Ui[ci][j] (ri = 1, half = 0).
//   split: word 8 p + 4 i + e (part p = 0..2, step i = 0, 1, e = 0..3) holds
//   the 16-bit pair A'[r][16 i + 8 half + 2 e + {0, 1}] of part p: (Ur, -Ui)
//   for ri = 0, (Ui, Ur) for ri = 1, at complex column j = 8 i + 4 half + e.
template <int TB, int WAVES, int PREC>
__device__ __forceinline__ void stage_blocks(TileShared<TB, WAVES, lane_words(PREC)> &sh, const uint32_t *A,
                                             const TileArgs &args, int tid)
{
    using C = TileCfg<TB, WAVES, lane_words(PREC)>;
    constexpr bool SPLIT = PREC != kPrecF32;
    constexpr int USED = lane_words(PREC);  // every word is read by the block loop
    const int nsub = args.n_sub;
    for (int e = tid; e < nsub * 64 * USED; e += C::THREADS) {
        const int s = e / (64 * USED), r = e % (64 * USED);
        const int lane = r / USED, wd = r % USED;
        const int half = lane >> 5, l32 = lane & 31, ci = l32 >> 1, ri = l32 & 1;
        const uint32_t *cop = A + size_t(s) * kTileOperandWords;
        uint32_t v;
        if (!SPLIT) {
            v = cop[(ri == half ? 0 : 256) + ci * 16 + wd];
            if (ri == 0 && half == 1) v ^= 0x80000000u;
        } else {
            const int part = wd >> 3, i = (wd >> 2) & 1, e4 = wd & 3;
            const uint32_t w = cop[part * 256 + ci * 16 + 8 * i + 4 * half + e4];
            v = ri ? ((w >> 16) | (w << 16)) : (w ^ 0x80000000u);
        }
        const int at = int(((uint32_t(wd) >> 2) ^ frag_swz<USED>(uint32_t(lane))) << 2) | (wd & 3);
        sh.op[s][lane * USED + at] = v;
    }
    for (int e = tid; e < nsub * (C::CBLOCKS + 32); e += C::THREADS) {
        const int s = e / (C::CBLOCKS + 32), r = e % (C::CBLOCKS + 32);
        uint32_t m = 0;
        for (int b = 0; b < 4; ++b) m |= 1u << args.tbit[s][b];
        const uint32_t cmask = ((1u << TB) - 1) & ~m;
        constexpr int NBW = C::NB_PER_WAVE;
        if (r < C::CBLOCKS)
            sh.cq[s][r] = swz(deposit(SPLIT ? uint32_t((r / NBW) * 32 * NBW + r % NBW) : uint32_t(r * 32), cmask),
                              args);
        else
            sh.cl[s][r - C::CBLOCKS] = swz(deposit(uint32_t(r - C::CBLOCKS) * (SPLIT ? NBW : 1), cmask), args);
    }
}

__device__ __forceinline__ void lds_st(char *Xb, uint32_t byte_off, float re, float im)
{
    vf2 v;
    v.x = re;
    v.y = im;
    *reinterpret_cast<vf2 *>(Xb + byte_off) = v;
}

// hi = RNE(v), lo = RNE(v - hi) and, with three parts, lo2 = RNE(v - hi - lo)
// of one (re, im) pair, as packed 16-bit pairs (H2 = bf16x2 or f16x2).  The
// differences are exact in FP32.  FP16 (two parts): lo = RNE(hi * m1 + v)
// with hi read as FP16 and m1 = -1 held in a register (minus_one()), one
// mixed-precision FMA per value (the compiler rounds some of them straight
// to FP16 in the same instruction): the same bits as a conversion back, a
// subtraction and a second conversion.
template <int NS, typename H2>
__device__ __forceinline__ void split_pair(float re, float im, H2 *parts, float m1)
{
    vf2 v;
    v.x = re;
    v.y = im;
    if constexpr (std::is_same<H2, f16x2>::value) {
        static_assert(NS == 2, "FP16 splits in two parts");
        parts[0] = __builtin_convertvector(v, H2);
        parts[1].x = static_cast<_Float16>(__builtin_fmaf(float(parts[0].x), m1, v.x));
        parts[1].y = static_cast<_Float16>(__builtin_fmaf(float(parts[0].y), m1, v.y));
    } else {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
            parts[j] = __builtin_convertvector(v, H2);
            if (j + 1 < NS) v -= __builtin_convertvector(parts[j], vf2);
        }
    }
}

// -1.0f in a scalar register, opaque to the compiler: with the literal it
// folds v + hi * (-1) back into a conversion and a subtraction.
__device__ __forceinline__ float minus_one()
{
    int bits;
    asm volatile("s_mov_b32 %0, 0xbf800000" : "=s"(bits));
    return __builtin_bit_cast(float, bits);
}

// One 32 x 32 x 16 product of 16-bit operands with FP32 accumulation.
__device__ __forceinline__ f32x16 mfma16(bf16x8 a, bf16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x16 mfma16(f16x8 a, f16x8 b, f32x16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ void lds_st4(char *Xb, uint32_t byte_off, float a, float b, float c, float d)
{
    vf4 v;
    v.x = a;
    v.y = b;
    v.z = c;
    v.w = d;
    *reinterpret_cast<vf4 *>(Xb + byte_off) = v;
}

// One block of the pass on the tile in LDS.  D real row = 8 (v / 4) + 4 half
// + v % 4: acc[4 g + 2 e] and acc[4 g + 2 e + 1] are (re, im) of complex row
// 4 g + 2 half + e.  Each wave owns its columns, so its reads of the block
// precede its writes; the caller places the barrier.
//
// FP32: lane (half, l32) reads re (half 0) or im (half 1) of complex row j,
// one 4-byte read per row and column block.  Split: every LDS access moves
// 16 bytes, two complex values that differ in tile bit 0.  If tile bit 0 is
// the block's row bit 0, these are rows (t, t + 1) of one column; otherwise
// tile bit 0 is the lowest column bit, i.e. column blocks (q, q + 1).
template <int TB, int WAVES, int PREC, int SCALE>
__device__ __forceinline__ void apply_block(TileShared<TB, WAVES, lane_words(PREC)> &sh, const TileArgs &args, int s,
                                            int w, int half, int l32, float scale, float unscale)
{
    using C = TileCfg<TB, WAVES, lane_words(PREC)>;
    constexpr bool SPLIT = PREC != kPrecF32;
    using H2 = typename std::conditional<PREC == kPrecF16, f16x2, bf16x2>::type;  // packed 16-bit pair
    using H8 = typename std::conditional<PREC == kPrecF16, f16x8, bf16x8>::type;  // MFMA operand
    constexpr int NBW = C::NB_PER_WAVE;
    static_assert(NBW % 2 == 0, "column blocks come in pairs");
    char *Xb = reinterpret_cast<char *>(sh.X4);
    uint32_t rb[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) rb[b] = args.swz[args.tbit[s][b]];
    const uint32_t cl = sh.cl[s][l32];
    uint32_t lq[NBW], wq[NBW];  // lane byte terms of this lane's column in block q
#pragma unroll
    for (int q = 0; q < NBW; ++q) {
        const uint32_t col = cl ^ sh.cq[s][w * NBW + q];
        // B rows: FP32 2j + half (re | im of complex row j); split 8i + 4 half + t
        lq[q] = SPLIT ? (col ^ (half ? rb[2] : 0u)) << 3 : (col << 3) | uint32_t(half << 2);
        wq[q] = (col ^ (half ? rb[1] : 0u)) << 3;  // complex row bit 1 = half
    }
    f32x16 acc[NBW];
#pragma unroll
    for (int q = 0; q < NBW; ++q)
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[q][v] = 0.f;
    const uint32_t *op = sh.op[s];
    const vf4 *ap = reinterpret_cast<const vf4 *>(op + (half * 32 + l32) * lane_words(PREC));  // staged fragments
    const uint32_t fsw = frag_swz<lane_words(PREC)>(uint32_t(half * 32 + l32));  // their chunk order
    if (!SPLIT) {
        float a[16];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const vf4 v = ap[uint32_t(i) ^ fsw];
            a[4 * i] = v.x;
            a[4 * i + 1] = v.y;
            a[4 * i + 2] = v.z;
            a[4 * i + 3] = v.w;
        }
#pragma unroll
        for (int j = 0; j < 16; ++j)
#pragma unroll
            for (int q = 0; q < NBW; ++q) {
                const float b = *reinterpret_cast<const float *>(Xb + ((row_of(rb, j) << 3) ^ lq[q]));
                acc[q] = __builtin_amdgcn_mfma_f32_32x32x2f32(a[j], b, acc[q], 0, 0, 0);
            }
#pragma unroll
        for (int q = 0; q < NBW; ++q)
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int e = 0; e < 2; ++e)
                    lds_st(Xb, (row_of(rb, 4 * g + e) << 3) ^ wq[q], acc[q][4 * g + 2 * e],
                           acc[q][4 * g + 2 * e + 1]);
        return;
    }
    // split: step i (K = 16 i .. 16 i + 15) with the operand's parts A_p
    // (BF16: three, FP16: two) and the tile values split into NS parts X_s:
    // every A_p X_0, every A_0 X_s, and A_1 X_1 when CROSS, the smaller terms
    // accumulated first.
    // FP16: the values are scaled by `scale` before the split (SCALE 0: one
    // scale per tile; SCALE 1: the tile is held scaled in LDS with one scale
    // per pass), A_1 is held multiplied by 2^11 and meets X_0 2^-11 (so that
    // neither falls below FP16's normal range), and the sums are scaled back
    // by `unscale` (SCALE 0).
    constexpr bool F16 = PREC == kPrecF16;
    constexpr bool SCALE_HERE = F16 && SCALE == 0;
    constexpr int NP = F16 ? 2 : 3;
    constexpr int NS = PREC == kPrecBF16X3 ? 3 : 2;
    constexpr bool CROSS = PREC == kPrecBF16X3;
    auto scaled = [&](vf4 v) { return SCALE_HERE ? v * scale : v; };
    auto out = [&](float v) { return SCALE_HERE ? v * unscale : v; };
    // X_0 2^-11 of a pair's X_0 (FP16 only; exact unless it falls below
    // FP16's normal range, where its product with A_1 is below 2^-35 of m)
    auto low_pair = [&](H2 x0) {
        vf2 c;
        c.x = 0x1p-11f;
        c.y = 0x1p-11f;
        return x0 * __builtin_convertvector(c, H2);  // a packed 16-bit multiply
    };
    const float m1 = F16 ? minus_one() : -1.f;
    auto fragment = [&](int p, int i) {
        H8 h;
        const vf4 f = ap[uint32_t(2 * p + i) ^ fsw];
        __builtin_memcpy(&h, &f, 16);
        return h;
    };
    auto products = [&](f32x16 c, const H8 *xa, const H8 *b) {
#pragma unroll
        for (int d = NP + NS - 2; d >= 0; --d)  // A_p X_s is about 2^(-8 (p + s)) of A X
#pragma unroll
            for (int sp = 0; sp < NS; ++sp) {
                const int p = d - sp;
                if (p >= 0 && p < NP && (sp == 0 || p == 0 || (CROSS && p == 1 && sp == 1)))
                    c = mfma16(xa[p], b[sp], c);
            }
        return c;
    };
    if (args.tbit[s][0] == 0) {  // uniform: rows (t, t + 1) share a slot
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            H8 xa[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) xa[p] = fragment(p, i);
#pragma unroll
            for (int q = 0; q < NBW; ++q) {
                vf4 raw[2];  // rows 8 i + 2 k2 + {0, 1} (plus 4 half)
#pragma unroll
                for (int k2 = 0; k2 < 2; ++k2)
                    raw[k2] = scaled(*reinterpret_cast<const vf4 *>(Xb + ((row_of(rb, 8 * i + 2 * k2) << 3) ^ lq[q])));
                H2 pp[4][NS];
#pragma unroll
                for (int k2 = 0; k2 < 2; ++k2) {
                    split_pair<NS>(raw[k2].x, raw[k2].y, pp[2 * k2], m1);
                    split_pair<NS>(raw[k2].z, raw[k2].w, pp[2 * k2 + 1], m1);
                }
                H8 b[NS];
#pragma unroll
                for (int sp = 0; sp < NS; ++sp) {
                    H2 t[4] = {pp[0][sp], pp[1][sp], pp[2][sp], pp[3][sp]};
                    __builtin_memcpy(&b[sp], t, 16);
                }
                if constexpr (F16) {
                    H2 t[4] = {low_pair(pp[0][0]), low_pair(pp[1][0]), low_pair(pp[2][0]), low_pair(pp[3][0])};
                    H8 bs;
                    __builtin_memcpy(&bs, t, 16);
                    acc[q] = mfma16(xa[0], b[1], acc[q]);
                    acc[q] = mfma16(xa[1], bs, acc[q]);
                    acc[q] = mfma16(xa[0], b[0], acc[q]);
                } else {
                    acc[q] = products(acc[q], xa, b);
                }
            }
        }
        // rows 4 g + 2 half + {0, 1} are acc[4 g .. 4 g + 3]
#pragma unroll
        for (int q = 0; q < NBW; ++q)
#pragma unroll
            for (int g = 0; g < 4; ++g)
                lds_st4(Xb, (row_of(rb, 4 * g) << 3) ^ wq[q], out(acc[q][4 * g]), out(acc[q][4 * g + 1]),
                        out(acc[q][4 * g + 2]), out(acc[q][4 * g + 3]));
    } else {  // column blocks (q, q + 1) share a slot
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            H8 xa[NP];
#pragma unroll
            for (int p = 0; p < NP; ++p) xa[p] = fragment(p, i);
#pragma unroll
            for (int q = 0; q < NBW; q += 2) {
                vf4 raw[4];  // row 8 i + t (plus 4 half): column blocks (q, q + 1)
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    raw[t] = scaled(*reinterpret_cast<const vf4 *>(Xb + ((row_of(rb, 8 * i + t) << 3) ^ lq[q])));
                H2 p0[4][NS], p1[4][NS];
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    split_pair<NS>(raw[t].x, raw[t].y, p0[t], m1);
                    split_pair<NS>(raw[t].z, raw[t].w, p1[t], m1);
                }
                H8 b0[NS], b1[NS];
#pragma unroll
                for (int sp = 0; sp < NS; ++sp) {
                    H2 t0[4] = {p0[0][sp], p0[1][sp], p0[2][sp], p0[3][sp]};
                    H2 t1[4] = {p1[0][sp], p1[1][sp], p1[2][sp], p1[3][sp]};
                    __builtin_memcpy(&b0[sp], t0, 16);
                    __builtin_memcpy(&b1[sp], t1, 16);
                }
                if constexpr (F16) {
                    H2 t0[4], t1[4];
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        t0[t] = low_pair(p0[t][0]);
                        t1[t] = low_pair(p1[t][0]);
                    }
                    H8 bs0, bs1;
                    __builtin_memcpy(&bs0, t0, 16);
                    __builtin_memcpy(&bs1, t1, 16);
                    acc[q] = mfma16(xa[0], b0[1], acc[q]);
                    acc[q + 1] = mfma16(xa[0], b1[1], acc[q + 1]);
                    acc[q] = mfma16(xa[1], bs0, acc[q]);
                    acc[q + 1] = mfma16(xa[1], bs1, acc[q + 1]);
                    acc[q] = mfma16(xa[0], b0[0], acc[q]);
                    acc[q + 1] = mfma16(xa[0], b1[0], acc[q + 1]);
                } else {
                    acc[q] = products(acc[q], xa, b0);
                    acc[q + 1] = products(acc[q + 1], xa, b1);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NBW; q += 2)
#pragma unroll
            for (int g = 0; g < 4; ++g)
#pragma unroll
                for (int e = 0; e < 2; ++e)
                    lds_st4(Xb, (row_of(rb, 4 * g + e) << 3) ^ wq[q], out(acc[q][4 * g + 2 * e]),
                            out(acc[q][4 * g + 2 * e + 1]), out(acc[q + 1][4 * g + 2 * e]),
                            out(acc[q + 1][4 * g + 2 * e + 1]));
    }
}

// The tile loop of one workgroup: tiles T, T + step, .. below T_end of the
// state at psi.  A = the blocks' compact operands (pack_tile_operand), back to
// back.  FP32 (kPrecF32): FP32 MFMA.  Split (kPrecBF16, kPrecBF16X3,
// kPrecF16): the host splits U into 16-bit parts, U = A_0 + A_1 + A_2 for
// BF16 (8 more significand bits each, about FP32's 24 in all) and A_0 + A_1
// for FP16; each B operand (8 consecutive K values = 4 complex rows of one
// column) is split while it is read from LDS, into X_0 + X_1 (kPrecBF16,
// kPrecF16) or X_0 + X_1 + X_2 (kPrecBF16X3), and the products
// sum_p A_p X_0 + sum_s A_0 X_s (plus A_1 X_1 for kPrecBF16X3) run on
// 32 x 32 x 16 MFMA with FP32 accumulation.  The dropped terms are about
// 2^-17 (BF16: the state's third part, A_1 X_1), 2^-22 (FP16) and 2^-25
// (BF16X3) relative to the result.  FP16 passes scale the values per tile
// (tile_scale; SCALE 0, and SCALE 2, which also reports the workgroup's sum
// of squares to norm.out) or per pass from the state's norm (norm_scale;
// SCALE 1, from the sums an earlier pass of the run reported; SCALE 3, the
// same scale with the state already held scaled in HBM, copied as it is).
template <int TB, int WAVES, int PREC, int SCALE>
__device__ __forceinline__ void tile_loop(TileShared<TB, WAVES, lane_words(PREC)> &sh, float *__restrict__ psi,
                                          const uint32_t *__restrict__ A, const TileArgs &args, uint64_t T,
                                          uint64_t T_end, uint64_t step, const TileNorm &norm)
{
    using C = TileCfg<TB, WAVES>;
    constexpr bool F16 = PREC == kPrecF16;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int half = lane >> 5, l32 = lane & 31;

    stage_blocks<TB, WAVES, PREC>(sh, A, args, tid);
    TileCopy<TB, WAVES> cp;
    cp.init(args, tid);
    // the largest magnitude in buf over the workgroup: a wave maximum into
    // sh.red[w]; the caller's next barrier publishes it
    auto wave_max_to_red = [&](const vf4 *buf) {
        // xor butterflies inside each 32-lane half (ds_swizzle in bit-mask
        // mode: no lane-index registers), then the two halves via readlane
        int m = __float_as_int(cp.max_abs(buf));
        m = __float_as_int(fmaxf(__int_as_float(m), __int_as_float(__builtin_amdgcn_ds_swizzle(m, 0x041F))));
        m = __float_as_int(fmaxf(__int_as_float(m), __int_as_float(__builtin_amdgcn_ds_swizzle(m, 0x081F))));
        m = __float_as_int(fmaxf(__int_as_float(m), __int_as_float(__builtin_amdgcn_ds_swizzle(m, 0x101F))));
        m = __float_as_int(fmaxf(__int_as_float(m), __int_as_float(__builtin_amdgcn_ds_swizzle(m, 0x201F))));
        m = __float_as_int(fmaxf(__int_as_float(m), __int_as_float(__builtin_amdgcn_ds_swizzle(m, 0x401F))));
        const float wm = fmaxf(__int_as_float(__builtin_amdgcn_readlane(m, 0)),
                               __int_as_float(__builtin_amdgcn_readlane(m, 32)));
        if (lane == 0) sh.red[w] = wm;
    };
    auto red_max = [&]() {
        float m = 0.f;
#pragma unroll
        for (int i = 0; i < WAVES; ++i) m = fmaxf(m, sh.red[i]);
        // uniform over the workgroup: keep it (and the scales) in scalar registers
        return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, m)));
    };

    // FP16 with SCALE 1: one scale for the pass from the state's norm, the
    // sum of the workgroups' sums of squares that an earlier pass of the run
    // wrote (fixed order; uniform, in scalar registers).  The copy-in
    // multiplies by it unless the state is already held scaled in HBM, and
    // the copy-out divides by it unless the state is to stay scaled.  SCALE 3:
    // the state is held scaled in HBM before and after the pass, so the pass
    // copies it as it is.
    float pscale = 1.f, punscale = 1.f;
    if (F16 && SCALE == 1) {
        double r2 = 0.0;
        for (int i = 0; i < norm.n_in; ++i) r2 += norm.in[i];
        norm_scale(sqrt(r2), pscale, punscale);
        if (norm.in_scaled) pscale = 1.f;
        if (norm.out_scaled) punscale = 1.f;
        pscale = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, pscale)));
        punscale = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, punscale)));
    }
    constexpr bool PER_TILE = F16 && (SCALE == 0 || SCALE == 2);  // scales from each tile's maximum
    // SCALE 2: per-tile scales as SCALE 0, and the workgroup's sum of squares to norm.out
    constexpr bool want_norm = F16 && SCALE == 2;
    if (T >= T_end) {  // uniform over the workgroup
        if (want_norm && tid == 0) norm.out[blockIdx.x] = 0.0;
        return;
    }
    // the wave's sum of squares of what it reads (want_norm), kept in LDS
    auto wave_sum = [&](float v) {
        v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x041F));
        v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x081F));
        v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x101F));
        v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x201F));
        v += __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x401F));
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0)) +
               __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 32));
    };
    if (want_norm && lane == 0) sh.nrm[w] = 0.f;
    // A finished tile is written to HBM at the top of the next round, before
    // that round's prefetch is issued: loads and stores may complete out of
    // order, so any wait for the prefetch also waits for earlier stores, and
    // these were issued a whole round of block work earlier.
    // a pass that starts the state from a basis state reads nothing: the
    // basis state lies in the tile whose outside positions match its bits,
    // at the tile index its tile-position bits form (FP32 and split FP16; in
    // the split BF16 kernels the extra registers made them spill)
    constexpr bool CAN_SYNTH = PREC == kPrecF32 || PREC == kPrecF16;
    const bool synth = CAN_SYNTH && norm.basis >= 0;  // uniform
    uint64_t b_out = 0;
    uint32_t b_t = 0;
    if (synth) {
        const uint64_t b = uint64_t(norm.basis);
        uint64_t in_mask = 0;
        for (int j = 0; j < TB; ++j) {
            b_t |= uint32_t((b >> args.ubit[j]) & 1u) << j;
            in_mask |= uint64_t(1) << args.ubit[j];
        }
        b_out = b & ~in_mask;
    }
    auto fetch = [&](vf4 *into, uint64_t base) {
        if (synth)
            cp.basis(into, base == b_out, b_t, tid);
        else
            cp.load(into, psi, base);
    };
    vf4 buf[C::CHUNKS];
    fetch(buf, tile_base(T, args));
    uint64_t prev = 0;
    for (bool first = true; T < T_end; T += step, first = false) {
        const uint64_t base = tile_base(T, args);
        if (F16 && SCALE == 1) {
            if (first)
                cp.to_lds_scaled(sh.X4, buf, pscale);
            else
                cp.swap_scaled(psi, prev, sh.X4, buf, pscale, punscale);
        } else {
            if (first)
                cp.to_lds(sh.X4, buf);
            else
                cp.swap(psi, prev, sh.X4, buf);
        }
        if (want_norm) {
            const float v = wave_sum(cp.sum_sq(buf));
            if (lane == 0) sh.nrm[w] += v;  // only this wave's lane 0 touches sh.nrm[w]
        }
        if (PER_TILE) wave_max_to_red(buf);  // this tile's largest magnitude, published by the barrier
        __syncthreads();  // the first one also publishes the staged blocks
        float scale = 1.f, unscale = 1.f;
        if (PER_TILE) {
            tile_scale(red_max(), scale, unscale);
            // uniform: held in scalar registers through the block loop
            scale = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, scale)));
            unscale = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, unscale)));
        }
        const uint64_t Tn = T + step;
        const bool more = Tn < T_end;  // uniform
        if (more) {
            // the next tile's loads go out at raised wave priority, ahead of
            // the other waves' block work on the SIMD (2-3 % per pass)
            __builtin_amdgcn_s_setprio(3);
            fetch(buf, tile_base(Tn, args));
            __builtin_amdgcn_s_setprio(0);
        }
        for (int s = 0; s < args.n_sub; ++s) {
            apply_block<TB, WAVES, PREC, F16 && !PER_TILE ? 1 : 0>(sh, args, s, w, half, l32, scale, unscale);
            __syncthreads();
        }
        prev = base;
    }
    // the last tile of this workgroup
    if (F16 && SCALE == 1)
        cp.store_scaled(psi, prev, sh.X4, punscale);
    else
        cp.store(psi, prev, sh.X4);
    if (want_norm) {
        // the workgroup's sum of squares: the wave sums in wave order, in FP64
        // (the norm only has to be right to a factor of two)
        __syncthreads();
        if (tid == 0) {
            double t = 0.0;
            for (int i = 0; i < WAVES; ++i) t += double(sh.nrm[i]);
            norm.out[blockIdx.x] = t;
        }
    }
}

// One pass over one state (gridDim.y = 1) or over psi and psi2 alike
// (gridDim.y = 2): a persistent grid strides over the tiles of its state.
template <int TB, int WAVES, int PREC, int SCALE>
__global__ void __launch_bounds__(64 * WAVES) k_tile_pass(float *__restrict__ psi, const uint32_t *__restrict__ A,
                                                          const TileArgs args, float *__restrict__ psi2,
                                                          const TileNorm norm)
{
    __shared__ TileShared<TB, WAVES, lane_words(PREC)> sh;
    tile_loop<TB, WAVES, PREC, SCALE>(sh, blockIdx.y ? psi2 : psi, A, args, blockIdx.x, args.n_tiles, gridDim.x,
                                      norm);
}

// Passes of many states in one grid: workgroup i takes tiles [t0, t1) of
// the pass units[i] names (states of a batch, each with its own tile layout,
// blocks and operands).
template <int TB, int WAVES, int PREC>
__global__ void __launch_bounds__(64 * WAVES) k_tile_batch(const TileUnit *__restrict__ units,
                                                           const TilePass *__restrict__ passes,
                                                           const uint32_t *__restrict__ pool, float *__restrict__ buf)
{
    __shared__ TileShared<TB, WAVES, lane_words(PREC)> sh;
    const TileUnit u = units[blockIdx.x];
    const TilePass &p = passes[u.pass];
    tile_loop<TB, WAVES, PREC, 0>(sh, buf + 2 * p.state_off, pool + p.op_off, p.args, u.t0, u.t1, 1, TileNorm{});
}

template <int TB, int WAVES>
hipError_t tile_launch(const TileArgs &a, const void *d_a, int prec, float *psi, float *psi2, hipStream_t st,
                       int cap, const TileNorm &norm, int *grid_out)
{
    uint64_t g = a.n_tiles;
    if (cap > 0 && g > uint64_t(cap)) g = cap;
    if (grid_out) *grid_out = int(g);
    const uint32_t *A = static_cast<const uint32_t *>(d_a);
    const dim3 grid(unsigned(g), psi2 ? 2 : 1);
    const dim3 block(64 * WAVES);
    TileNorm plain;  // the variants without the norm take only the basis start
    plain.basis = norm.basis;
    if (prec == kPrecBF16)
        hipLaunchKernelGGL((k_tile_pass<TB, WAVES, kPrecBF16, 0>), grid, block, 0, st, psi, A, a, psi2, plain);
    else if (prec == kPrecBF16X3)
        hipLaunchKernelGGL((k_tile_pass<TB, WAVES, kPrecBF16X3, 0>), grid, block, 0, st, psi, A, a, psi2, plain);
    else if (prec == kPrecF16 && norm.in && norm.in_scaled && norm.out_scaled)
        hipLaunchKernelGGL((k_tile_pass<TB, WAVES, kPrecF16, 3>), grid, block, 0, st, psi, A, a, psi2, norm);
    else if (prec == kPrecF16 && norm.in)
        hipLaunchKernelGGL((k_tile_pass<TB, WAVES, kPrecF16, 1>), grid, block, 0, st, psi, A, a, psi2, norm);
    else if (prec == kPrecF16 && norm.out)
        hipLaunchKernelGGL((k_tile_pass<TB, WAVES, kPrecF16, 2>), grid, block, 0, st, psi, A, a, psi2, norm);
    else if (prec == kPrecF16)
        hipLaunchKernelGGL((k_tile_pass<TB, WAVES, kPrecF16, 0>), grid, block, 0, st, psi, A, a, psi2, plain);
    else
        hipLaunchKernelGGL((k_tile_pass<TB, WAVES, kPrecF32, 0>), grid, block, 0, st, psi, A, a, psi2, plain);
    return hipGetLastError();
}

}  // namespace

bool tile_supported(int n, int union_bits) { return n >= kMinTileQubits && union_bits <= kMaxTileUnion; }

bool tile_shape_supported(int tile_bits, int waves)
{
    return (tile_bits == 14 && (waves == 8 || waves == 16)) || (tile_bits == 13 && (waves == 4 || waves == 8));
}

int tile_wgs_per_cu(int tile_bits, int waves)
{
    // LDS: a 64 KiB tile leaves room for a second workgroup; registers: two
    // 8-wave workgroups would need <= 128 VGPRs per lane
    return tile_bits == 13 && waves == 4 ? 2 : 1;
}

template <int LW>
static int max_blocks_of(int tile_bits, int waves)
{
    if (tile_bits == 14) return waves == 16 ? TileCfg<14, 16, LW>::MAX_SUB : TileCfg<14, 8, LW>::MAX_SUB;
    return waves == 4 ? TileCfg<13, 4, LW>::MAX_SUB : TileCfg<13, 8, LW>::MAX_SUB;
}

int tile_max_blocks(int tile_bits, int waves, int prec)
{
    if (!tile_shape_supported(tile_bits, waves)) return 0;
    return lane_words(prec) == 24 ? max_blocks_of<24>(tile_bits, waves) : max_blocks_of<16>(tile_bits, waves);
}

static uint32_t f2h_rne(float x)
{
    const _Float16 h = static_cast<_Float16>(x);  // round to nearest even
    uint16_t u;
    std::memcpy(&u, &h, 2);
    return u;
}

static float h2f(uint32_t u16)
{
    const uint16_t u = uint16_t(u16);
    _Float16 h;
    std::memcpy(&h, &u, 2);
    return float(h);
}

static uint32_t f2bf_rne(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}

static float bf2f(uint32_t h)
{
    const uint32_t u = h << 16;
    float x;
    std::memcpy(&x, &u, 4);
    return x;
}

void pack_tile_operand(const cd *m, int prec, uint32_t *out)
{
    std::memset(out, 0, sizeof(uint32_t) * kTileOperandWords);
    for (int r = 0; r < 16; ++r)
        for (int c = 0; c < 16; ++c) {
            const double re = m[r * 16 + c].real(), im = m[r * 16 + c].imag();
            if (prec == kTileOperandF32) {
                const float fr = float(re), fi = float(im);
                std::memcpy(&out[r * 16 + c], &fr, 4);
                std::memcpy(&out[256 + r * 16 + c], &fi, 4);
                continue;
            }
            // part p = RNE(x - parts 0..p-1), as (re, im) halves of one word:
            // three BF16 parts, two FP16 parts (the second held times 2^11,
            // which keeps it in FP16's normal range; the kernel pairs it with
            // X_0 2^-11)
            const int parts = prec == kTileOperandF16 ? 2 : 3;
            double xr = re, xi = im;
            for (int p = 0; p < parts; ++p) {
                uint32_t hr, hi;
                if (prec == kTileOperandF16) {
                    const double f = p ? 2048.0 : 1.0;
                    hr = f2h_rne(float(xr * f));
                    hi = f2h_rne(float(xi * f));
                    xr -= double(h2f(hr)) / f;
                    xi -= double(h2f(hi)) / f;
                } else {
                    hr = f2bf_rne(float(xr));
                    hi = f2bf_rne(float(xi));
                    xr -= double(bf2f(hr));
                    xi -= double(bf2f(hi));
                }
                out[256 * p + r * 16 + c] = hr | (hi << 16);
            }
        }
}

hipError_t make_tile_args(int n_sub, const int (*sub_pos)[4], int n, int tile_bits, int waves, int prec,
                          TileArgs *out)
{
    const int kTileBits = tile_bits;
    if ((tile_bits != 13 && tile_bits != 14) || n_sub < 1 || n_sub > kMaxTileSubBlocks || n < kTileBits)
        return hipErrorInvalidValue;
    TileArgs &a = *out;
    std::memset(&a, 0, sizeof a);
    uint64_t umask = 0;
    for (int s = 0; s < n_sub; ++s)
        for (int i = 0; i < 4; ++i) {
            // row bit i of block s is its i-th lowest position
            if (sub_pos[s][i] < 0 || sub_pos[s][i] >= n || (i && sub_pos[s][i] <= sub_pos[s][i - 1]))
                return hipErrorInvalidValue;
            umask |= uint64_t(1) << sub_pos[s][i];
        }
    const int nu = __builtin_popcountll(umask);
    if (nu > kTileBits) return hipErrorInvalidValue;
    // tile positions: the union plus the lowest positions outside it
    uint64_t tmask = umask;
    for (int p = 0; p < n && __builtin_popcountll(tmask) < kTileBits; ++p) tmask |= uint64_t(1) << p;
    if (!(tmask & 1)) return hipErrorInvalidValue;  // unreachable: position 0 always joins
    int b = 0;
    for (int p = 0; p < n; ++p) {
        if ((tmask >> p) & 1) a.ubit[b++] = p;
        else a.ext_pos[a.n_ext++] = p;
    }
    a.n_sub = n_sub;
    for (int s = 0; s < n_sub; ++s)
        for (int i = 0; i < 4; ++i) {
            int t = 0;
            while (a.ubit[t] != sub_pos[s][i]) ++t;
            a.tbit[s][i] = t;
        }
    a.n_tiles = uint64_t(1) << (n - kTileBits);
    // lanes of a wave take columns l32 NBW + q (split) or l32 (FP32), so a
    // lane group's columns differ from column bit log2(NBW) (split) or 0 up
    if (waves <= 0 || (1 << (tile_bits - 9)) % waves) return hipErrorInvalidValue;
    choose_tile_placement(a, tile_bits, waves, prec);
    return hipSuccess;
}

hipError_t launch_tile_pass(int n_sub, const int (*sub_pos)[4], const void *d_a, int prec, void *psi, int n,
                            hipStream_t st, int grid_cap, int tile_bits, int waves, void *psi2, const TileNorm &norm,
                            int *grid_out)
{
    if ((norm.in || norm.out) && (prec != kTileOperandF16 || psi2 || (norm.in && norm.n_in < 1)))
        return hipErrorInvalidValue;
    if ((norm.in_scaled || norm.out_scaled) && !norm.in) return hipErrorInvalidValue;
    if (norm.basis >= 0 && (psi2 || n >= 63 || (uint64_t(norm.basis) >> n) != 0 || norm.in_scaled ||
                            (prec != kTileOperandF32 && prec != kTileOperandF16)))
        return hipErrorInvalidValue;
    if (prec != kTileOperandF32 && prec != kTileOperandBF16 && prec != kTileOperandF16 && prec != kTileOperandBF16X3)
        return hipErrorInvalidValue;
    if (!tile_shape_supported(tile_bits, waves)) return hipErrorInvalidValue;
    if (n_sub < 1 || n_sub > tile_max_blocks(tile_bits, waves, prec)) return hipErrorInvalidValue;
    TileArgs a;
    if (hipError_t e = make_tile_args(n_sub, sub_pos, n, tile_bits, waves, prec, &a)) return e;
    float *p = static_cast<float *>(psi), *p2 = static_cast<float *>(psi2);
    if (tile_bits == 14)
        return waves == 16 ? tile_launch<14, 16>(a, d_a, prec, p, p2, st, grid_cap, norm, grid_out)
                           : tile_launch<14, 8>(a, d_a, prec, p, p2, st, grid_cap, norm, grid_out);
    return waves == 4 ? tile_launch<13, 4>(a, d_a, prec, p, p2, st, grid_cap, norm, grid_out)
                      : tile_launch<13, 8>(a, d_a, prec, p, p2, st, grid_cap, norm, grid_out);
}

hipError_t launch_tile_batch(const TileUnit *units, int n_units, const TilePass *passes, const uint32_t *pool,
                             void *buf, hipStream_t st, int prec)
{
    if (n_units <= 0) return hipSuccess;
    const dim3 grid{unsigned(n_units)}, block{unsigned(64 * kBatchTileWaves)};
    float *b = static_cast<float *>(buf);
    if (prec == kPrecBF16X3)
        hipLaunchKernelGGL((k_tile_batch<kBatchTileBits, kBatchTileWaves, kPrecBF16X3>), grid, block, 0, st, units,
                           passes, pool, b);
    else if (prec == kPrecBF16)
        hipLaunchKernelGGL((k_tile_batch<kBatchTileBits, kBatchTileWaves, kPrecBF16>), grid, block, 0, st, units, passes,
                           pool, b);
    else if (prec == kPrecF16)
        hipLaunchKernelGGL((k_tile_batch<kBatchTileBits, kBatchTileWaves, kPrecF16>), grid, block, 0, st, units, passes,
                           pool, b);
    else
        hipLaunchKernelGGL((k_tile_batch<kBatchTileBits, kBatchTileWaves, kPrecF32>), grid, block, 0, st, units, passes,
                           pool, b);
    return hipGetLastError();
}

}  // namespace dev
}  // namespace sv
