// Runtime: buffers, launch timing, kernel-path choice, operand packing and
// launch sequencing for fused plans.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>

#include "runtime.h"

namespace sv {

// ---------------------------------------------------------------- buffers
hipError_t DevBuf::ensure(size_t bytes)
{
    if (bytes <= cap) return hipSuccess;
    release();
    size_t want = std::max(bytes, size_t(4096));
    hipError_t e = hipMalloc(&p, want);
    if (e != hipSuccess) {
        p = nullptr;
        return e;
    }
    cap = want;
    return hipSuccess;
}

void DevBuf::release()
{
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
}

hipError_t PinBuf::ensure(size_t bytes)
{
    if (bytes <= cap) return hipSuccess;
    release();
    size_t want = std::max(bytes, size_t(4096));
    hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e != hipSuccess) {
        p = nullptr;
        return e;
    }
    cap = want;
    return hipSuccess;
}

void PinBuf::release()
{
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
}

// ---------------------------------------------------------------- timing
namespace {
struct Pending {
    int cls;
    hipEvent_t a, b;
};
struct StatsState {
    std::mutex mu;
    bool on = false;
    bool suspended = false;
    std::vector<Pending> pending;
    std::vector<hipEvent_t> free_events;
    std::map<int, std::pair<int64_t, double>> totals;
};
StatsState &stats()
{
    static StatsState s;
    return s;
}
hipEvent_t take_event(StatsState &s)
{
    if (!s.free_events.empty()) {
        hipEvent_t e = s.free_events.back();
        s.free_events.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
// Fold pending launches into the totals (synchronises on their events).
int drain(StatsState &s)
{
    int rc = SV_OK;
    for (auto &p : s.pending) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(p.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.a, p.b);
        if (e != hipSuccess) {
            rc = fail(SV_ERR_HIP, "launch timing: %s", hipGetErrorString(e));
        } else {
            auto &t = s.totals[p.cls];
            t.first += 1;
            t.second += ms;
        }
        s.free_events.push_back(p.a);
        s.free_events.push_back(p.b);
    }
    s.pending.clear();
    return rc;
}
}  // namespace

LaunchTimer::LaunchTimer(int cls, hipStream_t st) : cls_(cls), st_(st)
{
    auto &s = stats();
    std::lock_guard<std::mutex> lk(s.mu);
    if (!s.on || s.suspended) return;
    a_ = take_event(s);
    b_ = take_event(s);
    if (a_ && b_) (void)hipEventRecord(a_, st_);
}

LaunchTimer::~LaunchTimer()
{
    if (!a_ || !b_) return;
    auto &s = stats();
    std::lock_guard<std::mutex> lk(s.mu);
    (void)hipEventRecord(b_, st_);
    s.pending.push_back({cls_, a_, b_});
    if (s.pending.size() > 4096) drain(s);
}

void timing_suspend(bool on)
{
    auto &s = stats();
    std::lock_guard<std::mutex> lk(s.mu);
    s.suspended = on;
}

int stats_enable(int on)
{
    auto &s = stats();
    std::lock_guard<std::mutex> lk(s.mu);
    s.on = on != 0;
    return SV_OK;
}

int stats_reset()
{
    auto &s = stats();
    std::lock_guard<std::mutex> lk(s.mu);
    int rc = drain(s);
    s.totals.clear();
    return rc;
}

int stats_query(int cls, int64_t *launches, double *total_ms)
{
    auto &s = stats();
    std::lock_guard<std::mutex> lk(s.mu);
    int rc = drain(s);
    auto it = s.totals.find(cls);
    *launches = it == s.totals.end() ? 0 : it->second.first;
    *total_ms = it == s.totals.end() ? 0.0 : it->second.second;
    return rc;
}

// ---------------------------------------------------------------- paths
Tuning &tuning()
{
    static Tuning t = [] {
        Tuning x;
        for (int k = 0; k <= SV_MAX_K; ++k) {
            x.reg_grid_cap[k] = 8192;
            x.mfma_tc_log[k] = 6;
            x.mfma_grid_cap[k] = 2048;
            x.split_tc_log[k] = 6;
        }
        x.mfma_tc_log[4] = 7;
        x.split_tc_log[4] = 7;
        x.mfma_tc_log[6] = 5;
        x.split_tc_log[6] = 5;
        x.k4_reg = false;
        x.tile_grid_cap = 256;
        x.tile_bits = 14;
        x.tile_waves = 16;
        if (const char *e = std::getenv("SV_TILE_BITS")) x.tile_bits = std::atoi(e) == 13 ? 13 : 14;
        if (const char *e = std::getenv("SV_TILE_WAVES")) x.tile_waves = std::atoi(e);
        if (!dev::tile_shape_supported(x.tile_bits, x.tile_waves)) x.tile_waves = x.tile_bits == 14 ? 16 : 4;
        if (const char *e = std::getenv("SV_TILE_GRID")) x.tile_grid_cap = std::max(1, std::atoi(e));
        return x;
    }();
    return t;
}

int tile_pass_bits() { return tuning().tile_bits; }

int tile_pass_capacity(int precision)
{
    const Tuning &t = tuning();
    const int prec = precision < 0 ? dev::kTileOperandBF16 : tile_operand_prec(tile_path(precision));
    return dev::tile_max_blocks(t.tile_bits, t.tile_waves, prec);
}

Path choose_path(int dtype, int precision, int k, const int *q, int n)
{
    if (dtype == SV_C128) return dev::reg_supported(dtype, k, q, n) ? PATH_REG : PATH_GENERIC;
    if (k >= 4 && dev::mfma_supported(k, n)) {
        if (precision == SV_PREC_SPLIT_BF16) return PATH_SPLIT_BF16;
        if (precision == SV_PREC_SPLIT_FP16) return PATH_SPLIT_FP16;
        if (!(k == 4 && tuning().k4_reg && dev::reg_supported(dtype, k, q, n))) return PATH_MFMA32;
    }
    if (dev::reg_supported(dtype, k, q, n)) return PATH_REG;
    return PATH_GENERIC;
}

int path_family(Path p)
{
    switch (p) {
    case PATH_REG: return FAM_REG;
    case PATH_GENERIC: return FAM_GENERIC;
    case PATH_MFMA32: return FAM_MFMA32;
    case PATH_SPLIT_BF16: return FAM_SPLIT_BF16;
    case PATH_TILE: return FAM_TILE;
    case PATH_TILE_BF16: return FAM_TILE_BF16;
    case PATH_TILE_FP16: return FAM_TILE_FP16;
    case PATH_TILE_BF16X3: return FAM_TILE_BF16X3;
    default: return FAM_SPLIT_FP16;
    }
}

static size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t pack_operands(std::vector<Launch> &launches, int dtype, PinBuf &stage)
{
    // pass 1: sizes
    size_t total = 0;
    for (auto &L : launches) {
        const int D = 1 << L.k;
        switch (L.path) {
        case PATH_REG: break;
        case PATH_GENERIC:
            L.arena_off = total;
            total = align256(total + size_t(D) * D * 2 * (dtype == SV_C64 ? 4 : 8));
            break;
        case PATH_MFMA32:
            L.arena_off = total;
            total = align256(total + dev::real_form_elems(L.k) * 4);
            break;
        case PATH_TILE:
        case PATH_TILE_BF16:
        case PATH_TILE_FP16:
        case PATH_TILE_BF16X3:
            L.arena_off = total;
            total = align256(total + size_t(L.k) * dev::kTileOperandWords * 4);
            break;
        default:
            L.arena_off = total;
            total = align256(total + dev::real_form_elems(L.k) * 2);
            L.arena_off2 = total;
            total = align256(total + dev::real_form_elems(L.k) * 2);
            L.arena_off3 = total;
            total = align256(total + dev::real_form_elems(L.k) * 2);
            break;
        }
    }
    // one region for the norm partials of the run's split-FP16 tile passes
    bool fp16_tiles = false;
    for (const auto &L : launches) fp16_tiles = fp16_tiles || L.path == PATH_TILE_FP16;
    if (fp16_tiles) {
        for (auto &L : launches)
            if (L.path == PATH_TILE_FP16) L.norm_off = total;
        total = align256(total + sizeof(double) * kTileNormSlots);
    }
    if (total == 0) return 0;
    if (stage.ensure(total) != hipSuccess) return size_t(-1);
    char *h = static_cast<char *>(stage.p);
    for (auto &L : launches) {
        const int D = 1 << L.k;
        switch (L.path) {
        case PATH_REG: break;
        case PATH_GENERIC:
            if (dtype == SV_C64) {
                float *f = reinterpret_cast<float *>(h + L.arena_off);
                for (int i = 0; i < D * D; ++i) {
                    f[2 * i] = float(L.m[i].real());
                    f[2 * i + 1] = float(L.m[i].imag());
                }
            } else {
                double *f = reinterpret_cast<double *>(h + L.arena_off);
                for (int i = 0; i < D * D; ++i) {
                    f[2 * i] = L.m[i].real();
                    f[2 * i + 1] = L.m[i].imag();
                }
            }
            break;
        case PATH_MFMA32:
            dev::pack_real_form_f32(L.m.data(), L.k, reinterpret_cast<float *>(h + L.arena_off));
            break;
        case PATH_TILE:
        case PATH_TILE_BF16:
        case PATH_TILE_FP16:
        case PATH_TILE_BF16X3:
            for (int sb = 0; sb < L.k; ++sb)
                dev::pack_tile_operand(L.m.data() + 256 * sb, tile_operand_prec(L.path),
                                       reinterpret_cast<uint32_t *>(h + L.arena_off) + dev::kTileOperandWords * sb);
            break;
        default: {
            uint16_t *const parts[3] = {reinterpret_cast<uint16_t *>(h + L.arena_off),
                                        reinterpret_cast<uint16_t *>(h + L.arena_off2),
                                        reinterpret_cast<uint16_t *>(h + L.arena_off3)};
            dev::pack_real_form_split(L.m.data(), L.k, L.path == PATH_SPLIT_FP16, parts);
            break;
        }
        }
    }
    return total;
}

// Canonical 16 x 16 matrix of a block on positions q[0..k-1] (ascending)
// padded with identity on the extra positions of p4 (ascending, 4 entries).
static void pad_to_four(const Block &b, const int *p4, std::vector<cd> &out)
{
    int where[4];  // for each of the 4 padded bits: index in b.q, or -1
    for (int j = 0; j < 4; ++j) {
        where[j] = -1;
        for (int i = 0; i < b.k; ++i)
            if (b.q[i] == p4[j]) where[j] = i;
    }
    const int D = 1 << b.k;
    out.assign(256, cd(0));
    for (int r = 0; r < 16; ++r)
        for (int c = 0; c < 16; ++c) {
            int rr = 0, cc = 0;
            bool same = true;
            for (int j = 0; j < 4; ++j) {
                const int rb = (r >> j) & 1, cb = (c >> j) & 1;
                if (where[j] >= 0) {
                    rr |= rb << where[j];
                    cc |= cb << where[j];
                } else if (rb != cb) {
                    same = false;
                }
            }
            if (same) out[size_t(r) * 16 + c] = b.m[size_t(rr) * D + cc];
        }
}

static uint64_t mask_of(const Block &b)
{
    uint64_t m = 0;
    for (int j = 0; j < b.k; ++j) m |= uint64_t(1) << b.q[j];
    return m;
}

Path tile_path(int precision)
{
    if (precision == SV_PREC_SPLIT_BF16) return PATH_TILE_BF16;
    if (precision == SV_PREC_SPLIT_FP16) return PATH_TILE_FP16;
    if (precision == SV_PREC_SPLIT_BF16X3) return PATH_TILE_BF16X3;
    return PATH_TILE;
}

int tile_operand_prec(int path)
{
    return path == PATH_TILE_BF16     ? dev::kTileOperandBF16
           : path == PATH_TILE_FP16   ? dev::kTileOperandF16
           : path == PATH_TILE_BF16X3 ? dev::kTileOperandBF16X3
                                      : dev::kTileOperandF32;
}

void tile_pass_blocks(const Block *const *blocks, int count, int n, int (*sub_pos)[4], std::vector<cd> &mats)
{
    uint64_t um = 0;
    for (int i = 0; i < count; ++i) um |= mask_of(*blocks[i]);
    // the union gets at least 4 positions (lowest free ones)
    for (int p = 0; p < n && __builtin_popcountll(um) < 4; ++p) um |= uint64_t(1) << p;
    mats.clear();
    for (int sb = 0; sb < count; ++sb) {
        const Block &b = *blocks[sb];
        uint64_t pm = mask_of(b);
        for (int p = 0; p < 64 && __builtin_popcountll(pm) < 4; ++p)
            if (((um >> p) & 1) && !((pm >> p) & 1)) pm |= uint64_t(1) << p;
        int c = 0;
        for (int p = 0; p < 64; ++p)
            if ((pm >> p) & 1) sub_pos[sb][c++] = p;
        std::vector<cd> m4;
        pad_to_four(b, sub_pos[sb], m4);
        mats.insert(mats.end(), m4.begin(), m4.end());
    }
}

void group_tile_passes(const std::vector<Block> &blocks, int n, int precision, std::vector<Launch> &out)
{
    out.clear();
    const CostTable cost = lookup_costs(n, precision, nullptr);
    for (const auto &grp : tile_groups(blocks, n)) {
        // a block alone: its own dense launch, or a tile pass of one block
        // where that is priced lower
        const Block &b0 = blocks[grp[0]];
        if (grp.size() == 1 && !(b0.k <= 4 && dev::tile_supported(n, 4) && cost.tile[1] < cost.ms[b0.k])) {
            const Block &b = b0;
            Launch L;
            L.k = b.k;
            std::copy(b.q, b.q + SV_MAX_K, L.q);
            L.path = choose_path(SV_C64, precision, b.k, b.q, n);
            L.m = b.m;
            out.push_back(std::move(L));
            continue;
        }
        Launch L;
        L.path = tile_path(precision);
        L.k = int(grp.size());
        std::fill(L.q, L.q + SV_MAX_K, 0);
        std::vector<const Block *> bp;
        for (size_t b : grp) bp.push_back(&blocks[b]);
        tile_pass_blocks(bp.data(), L.k, n, L.sub_pos, L.m);
        out.push_back(std::move(L));
    }
}

int enqueue(const std::vector<Launch> &launches, int dtype, void *psi, int n, const void *arena, hipStream_t st)
{
    return enqueue(launches.data(), launches.size(), dtype, psi, n, arena, st);
}

int enqueue(const Launch *first, size_t count, int dtype, void *psi, int n, const void *arena, hipStream_t st,
            void *psi2)
{
    const char *A = static_cast<const char *>(arena);
    const Tuning &T = tuning();
    // split-FP16 tile passes of one state: the first writes the norm partials,
    // the later ones take their scale from them (unitary blocks keep the norm,
    // so it is one scale for all of them), and from the second of them to the
    // last the state stays in HBM times that scale: the second scales it at
    // copy-in, the last unscales it at copy-out, the ones between copy it as
    // it is.  Launches in between act on it linearly; the state is plain again
    // when this call's launches end.
    const uint64_t norm_tiles = n >= T.tile_bits ? uint64_t(1) << (n - T.tile_bits) : 0;  // no tile passes below
    const int norm_grid_cap = T.tile_grid_cap * dev::tile_wgs_per_cu(T.tile_bits, T.tile_waves);
    const uint64_t norm_grid_size =
        norm_grid_cap > 0 && norm_tiles > uint64_t(norm_grid_cap) ? uint64_t(norm_grid_cap) : norm_tiles;
    int norm_launches = 0;  // split-FP16 tile launches of this call that take part
    if (!psi2 && norm_grid_size <= uint64_t(kTileNormSlots))
        for (const Launch *it = first; it != first + count; ++it)
            if (it->path == PATH_TILE_FP16) {
                const int cap = dev::tile_max_blocks(T.tile_bits, T.tile_waves, dev::kTileOperandF16);
                norm_launches += (it->k + cap - 1) / cap;
            }
    int norm_grid = 0, norm_done = 0;
    for (const Launch *it = first; it != first + count; ++it) {
        const Launch &L = *it;
        if (psi2 && L.path != PATH_REG && L.path != PATH_GENERIC && L.path != PATH_MFMA32 && !is_tile_path(L.path)) {
            // paths without a second-state launch: one launch per state
            if (int rc = enqueue(it, 1, dtype, psi, n, arena, st)) return rc;
            if (int rc = enqueue(it, 1, dtype, psi2, n, arena, st)) return rc;
            continue;
        }
        if (is_tile_path(L.path)) {
            // one launch per chunk of blocks whose operands fit the shape's LDS
            const int cap = dev::tile_max_blocks(T.tile_bits, T.tile_waves, tile_operand_prec(L.path));
            const size_t op_bytes = 4 * dev::kTileOperandWords;
            const int grid_cap = T.tile_grid_cap * dev::tile_wgs_per_cu(T.tile_bits, T.tile_waves);
            const uint64_t n_tiles = uint64_t(1) << (n - T.tile_bits);
            const uint64_t grid = grid_cap > 0 && n_tiles > uint64_t(grid_cap) ? uint64_t(grid_cap) : n_tiles;
            const bool use_norm = L.path == PATH_TILE_FP16 && !psi2 && grid <= uint64_t(kTileNormSlots);
            for (int c = 0; c < L.k; c += cap) {
                const int m = std::min(cap, L.k - c);
                dev::TileNorm norm;
                int launched = 0;
                if (use_norm) {
                    double *part = reinterpret_cast<double *>(const_cast<char *>(A) + L.norm_off);
                    if (norm_grid > 0) {
                        norm.in = part;
                        norm.n_in = norm_grid;
                        norm.in_scaled = norm_done >= 2;
                        norm.out_scaled = norm_done + 1 < norm_launches;
                    } else {
                        norm.out = part;
                    }
                }
                if (c == 0 && L.basis >= 0) norm.basis = L.basis;  // reads nothing: the state starts here
                LaunchTimer timer(stat_class(path_family(L.path), m), st);
                hipError_t e = dev::launch_tile_pass(m, L.sub_pos + c, A + L.arena_off + c * op_bytes,
                                                     tile_operand_prec(L.path), psi, n, st, grid_cap, T.tile_bits,
                                                     T.tile_waves, psi2, norm, &launched);
                if (e != hipSuccess)
                    return fail(SV_ERR_HIP, "tile pass launch (%d blocks): %s", m, hipGetErrorString(e));
                if (norm.out) norm_grid = launched;
                if (use_norm) ++norm_done;
            }
            continue;
        }
        LaunchTimer timer(stat_class(path_family(L.path), L.k), st);
        hipError_t e = hipSuccess;
        switch (L.path) {
        case PATH_REG: e = dev::launch_reg(dtype, L.k, L.q, L.m.data(), psi, n, st, T.reg_grid_cap[L.k], psi2); break;
        case PATH_GENERIC: e = dev::launch_generic(dtype, L.k, L.q, A + L.arena_off, psi, n, st, psi2); break;
        case PATH_MFMA32:
            e = dev::launch_mfma_f32(L.k, L.q, reinterpret_cast<const float *>(A + L.arena_off), psi, n, st,
                                     T.mfma_tc_log[L.k], T.mfma_grid_cap[L.k], psi2);
            break;
        default: {
            const uint16_t *const parts[3] = {reinterpret_cast<const uint16_t *>(A + L.arena_off),
                                              reinterpret_cast<const uint16_t *>(A + L.arena_off2),
                                              reinterpret_cast<const uint16_t *>(A + L.arena_off3)};
            e = dev::launch_mfma_split(L.k, L.path == PATH_SPLIT_FP16, L.q, parts, psi, n, st,
                                       T.split_tc_log[L.k], T.mfma_grid_cap[L.k]);
            break;
        }
        }
        if (e != hipSuccess) return fail(SV_ERR_HIP, "kernel launch (path %d, k=%d): %s", int(L.path), L.k, hipGetErrorString(e));
    }
    return SV_OK;
}

}  // namespace sv
