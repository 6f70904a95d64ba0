// LDS placement of a tile pass (host only): the per-pass XOR-linear map from
// tile indices to LDS indices that the tile kernels use (TileArgs::swz),
// chosen so that the 16-byte LDS accesses of every block of the pass hit
// distinct banks.
#include <array>
#include <cstring>
#include <string>
#include <unordered_map>
#include <utility>

#include "kernels.h"

namespace sv {
namespace dev {
namespace {

int gf2_rank(uint32_t *v, int k)
{
    int r = 0;
    for (int bit = 0; bit < 32 && r < k; ++bit) {
        int piv = -1;
        for (int i = r; i < k; ++i)
            if ((v[i] >> bit) & 1) {
                piv = i;
                break;
            }
        if (piv < 0) continue;
        std::swap(v[r], v[piv]);
        for (int i = 0; i < k; ++i)
            if (i != r && ((v[i] >> bit) & 1)) v[i] ^= v[r];
        ++r;
    }
    return r;
}

// Extra LDS cycles of the block loop's 16-byte accesses under the placement
// `img` (image of each tile bit).  Such an access is served a group of lanes
// at a time: 8 lanes over 32 four-byte banks or 16 lanes over 64.  The lanes
// of a group hold columns whose indices differ in 3 (4) consecutive bits
// starting at bit `lane_shift`, the rows being the same; the group is free of
// conflicts when the LDS images of those column bits are independent on LDS
// index bits 1..3 (1..4), and otherwise takes 2^(deficit) cycles.
int placement_conflicts(const uint32_t *img, const TileArgs &a, int tile_bits, int lane_shift)
{
    int c = 0;
    for (int s = 0; s < a.n_sub; ++s) {
        uint32_t m = 0;
        for (int b = 0; b < 4; ++b) m |= 1u << a.tbit[s][b];
        int cpos[kMaxTileBits], nc = 0;
        for (int b = 0; b < tile_bits; ++b)
            if (!((m >> b) & 1)) cpos[nc++] = b;
        uint32_t v3[3], v4[4];
        for (int j = 0; j < 4; ++j) {
            const uint32_t x = img[cpos[lane_shift + j]] >> 1;
            if (j < 3) v3[j] = x & 7u;
            v4[j] = x & 15u;
        }
        c += (1 << (3 - gf2_rank(v3, 3))) - 1 + (1 << (4 - gf2_rank(v4, 4))) - 1;
    }
    return c;
}

// The pass's LDS placement S.  Candidates keep tile bits 0..3 in place and
// add to the image of bit b >= 4 some of LDS bits 1..3 and, for b >= 5, bit 4:
// S is then unit lower triangular over GF(2), a permutation of the tile's
// indices that keeps bit 0.  The first candidate XORs bits 5..8 into bits
// 1..4; while some block still has conflicts, seeded random candidates
// (at most 2048, the same sequence for every pass) are tried and the best kept.
void search_swizzle(TileArgs &a, int tile_bits, int lane_shift)
{
    uint32_t best[kMaxTileBits], cand[kMaxTileBits];
    for (int b = 0; b < tile_bits; ++b) best[b] = (1u << b) ^ (((1u << b) >> 4) & 0x1Eu);
    // FP32 passes (lane_shift < 0: 4-byte accesses, MFMA-bound) keep the first
    int bc = lane_shift < 0 ? 0 : placement_conflicts(best, a, tile_bits, lane_shift);
    uint64_t x = 0x9E3779B97F4A7C15ull;
    for (int t = 0; t < 2048 && bc > 0; ++t) {
        for (int b = 0; b < tile_bits; ++b) {
            cand[b] = 1u << b;
            if (b < 4) continue;
            x ^= x << 13;
            x ^= x >> 7;
            x ^= x << 17;
            cand[b] |= uint32_t(x & 7u) << 1;
            if (b >= 5) cand[b] |= uint32_t((x >> 3) & 1u) << 4;
        }
        const int c = placement_conflicts(cand, a, tile_bits, lane_shift);
        if (c < bc) {
            bc = c;
            std::memcpy(best, cand, sizeof(uint32_t) * size_t(tile_bits));
        }
    }
    for (int b = 0; b < kMaxTileBits; ++b) a.swz[b] = b < tile_bits ? best[b] : 0u;
}

// The search depends only on the blocks' tile bits, the tile size and the lane
// shift, and a plan's passes recur on every run (and in the adjoint sweep), so
// each host thread remembers its results (at most 4096 layouts, then it
// starts over).
void choose_swizzle(TileArgs &a, int tile_bits, int lane_shift)
{
    std::string k;
    k.reserve(3 + 4 * size_t(a.n_sub));
    k.push_back(char(tile_bits));
    k.push_back(char(lane_shift + 1));
    k.push_back(char(a.n_sub));
    for (int s = 0; s < a.n_sub; ++s)
        for (int j = 0; j < 4; ++j) k.push_back(char(a.tbit[s][j]));
    thread_local std::unordered_map<std::string, std::array<uint32_t, kMaxTileBits>> memo;
    const auto it = memo.find(k);
    if (it != memo.end()) {
        std::memcpy(a.swz, it->second.data(), sizeof a.swz);
        return;
    }
    search_swizzle(a, tile_bits, lane_shift);
    if (memo.size() >= 4096) memo.clear();
    std::array<uint32_t, kMaxTileBits> v;
    std::memcpy(v.data(), a.swz, sizeof a.swz);
    memo.emplace(k, v);
}

}  // namespace

// Lanes of a wave take columns l32 NBW + q (split) or l32 (FP32), so a lane
// group's columns differ from column bit log2(NBW) (split) or 0 up.  FP32
// passes (4-byte accesses, MFMA-bound) keep the first candidate.
void choose_tile_placement(TileArgs &a, int tile_bits, int waves, int prec)
{
    const int nbw = (1 << (tile_bits - 9)) / waves;
    choose_swizzle(a, tile_bits, prec == kTileOperandF32 ? -1 : __builtin_ctz(unsigned(nbw)));
}

int tile_placement_conflicts(const TileArgs &a, int tile_bits, int waves, int prec)
{
    if (prec == kTileOperandF32 || waves <= 0) return 0;
    return placement_conflicts(a.swz, a, tile_bits, __builtin_ctz(unsigned((1 << (tile_bits - 9)) / waves)));
}

}  // namespace dev
}  // namespace sv
