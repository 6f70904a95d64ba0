// Autotuner: times the block kernels on the caller's scratch state and keeps
// the fastest launch shape per block size k; the per-k times form the cost
// table that fusion (max_k = -1, enhanced merging) optimises against.
//
// Candidates per k (complex64):
//   k <= 3 : register kernel, grid caps {2048, 4096, 8192, 16384, unbounded};
//   k = 4  : register kernel (same caps) and the MFMA kernel;
//   k >= 4 : MFMA kernel, column tiles 2^5..2^7 (where the tile fits) x grid
//            caps {1024, 2048, 4096} (split kernels for SPLIT_* precisions).
// Complex128 (FP64) times the register kernel for k <= 3 and the generic
// kernel above.  Each candidate is timed on three position sets (lowest k
// positions, highest k, and a spread set) and the mean is kept.  For
// complex64 states of >= 14 qubits the tile passes holding 1..4 blocks are
// timed too (FP32, or split BF16 for the split precisions), so SV_RULE_AUTO
// can price tiled plans against plain fused ones.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include <unistd.h>

#include "runtime.h"

using namespace sv;

namespace {

std::vector<cd> dft_matrix(int k)
{
    const int D = 1 << k;
    std::vector<cd> m(size_t(D) * D);
    const double s = 1.0 / std::sqrt(double(D));
    for (int r = 0; r < D; ++r)
        for (int c = 0; c < D; ++c) m[size_t(r) * D + c] = std::polar(s, 2.0 * M_PI * r * c / D);
    return m;
}

std::vector<std::vector<int>> position_sets(int n, int k)
{
    std::vector<std::vector<int>> sets;
    std::vector<int> lo, hi, spread;
    for (int j = 0; j < k; ++j) {
        lo.push_back(j);
        hi.push_back(n - k + j);
        spread.push_back(int(std::lround(double(j) * (n - 1) / std::max(k - 1, 1))));
    }
    std::sort(spread.begin(), spread.end());
    spread.erase(std::unique(spread.begin(), spread.end()), spread.end());
    sets.push_back(lo);
    sets.push_back(hi);
    if (int(spread.size()) == k) sets.push_back(spread);
    return sets;
}

struct Cand {
    Path path;
    int grid_cap;
    int tc_log;
};

// Mean milliseconds per application over the position sets (reps each).
int time_candidate(sv_state *s, int k, const Cand &c, int reps, double *ms_out)
{
    Tuning saved = tuning();
    Tuning &T = tuning();
    T.reg_grid_cap[k] = c.grid_cap;
    T.mfma_grid_cap[k] = c.grid_cap;
    if (c.path == PATH_MFMA32) T.mfma_tc_log[k] = c.tc_log;
    if (c.path == PATH_SPLIT_BF16 || c.path == PATH_SPLIT_FP16) T.split_tc_log[k] = c.tc_log;
    hipEvent_t a, b;
    SV_HIP(hipEventCreate(&a));
    SV_HIP(hipEventCreate(&b));
    double total = 0;
    int count = 0;
    int rc = SV_OK;
    const std::vector<cd> m = dft_matrix(k);
    for (const auto &pos : position_sets(s->n, k)) {
        std::vector<Launch> L(1);
        L[0].path = c.path;
        L[0].k = k;
        std::fill(L[0].q, L[0].q + SV_MAX_K, 0);
        std::copy(pos.begin(), pos.end(), L[0].q);
        L[0].m = m;
        if (c.path == PATH_REG && !dev::reg_supported(s->dtype, k, L[0].q, s->n)) continue;
        if (c.path != PATH_REG && c.path != PATH_GENERIC && !dev::mfma_supported(k, s->n)) continue;
        SV_HIP(hipEventSynchronize(s->arena_free));
        const size_t bytes = pack_operands(L, s->dtype, s->stage);
        if (bytes) {
            SV_HIP(s->arena.ensure(bytes));
            SV_HIP(hipMemcpyAsync(s->arena.p, s->stage.p, bytes, hipMemcpyHostToDevice, s->stream));
        }
        rc = enqueue(L, s->dtype, s->buf, s->n, s->arena.p, s->stream);  // warm-up
        if (rc) break;
        SV_HIP(hipEventRecord(a, s->stream));
        for (int r = 0; r < reps && !rc; ++r) rc = enqueue(L, s->dtype, s->buf, s->n, s->arena.p, s->stream);
        SV_HIP(hipEventRecord(b, s->stream));
        SV_HIP(hipEventRecord(s->arena_free, s->stream));
        SV_HIP(hipEventSynchronize(b));
        float ms = 0;
        SV_HIP(hipEventElapsedTime(&ms, a, b));
        total += ms / reps;
        ++count;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    tuning() = saved;
    if (rc) return rc;
    *ms_out = count ? total / count : 1e30;
    return SV_OK;
}

// Mean milliseconds of one tile pass holding nsub 4-qubit blocks, over two
// union layouts (8 positions spread over the state, and the lowest 8).
int time_tile(sv_state *s, Path path, int nsub, int reps, double *ms_out)
{
    hipEvent_t a, b;
    SV_HIP(hipEventCreate(&a));
    SV_HIP(hipEventCreate(&b));
    const std::vector<cd> m4 = dft_matrix(4);
    double total = 0;
    int count = 0, rc = SV_OK;
    for (int layout = 0; layout < 2 && !rc; ++layout) {
        int u[8];
        for (int i = 0; i < 8; ++i) u[i] = layout ? i : int(std::lround(double(i) * (s->n - 1) / 7));
        std::vector<Launch> L(1);
        L[0].path = path;
        L[0].k = nsub;
        std::fill(L[0].q, L[0].q + SV_MAX_K, 0);
        for (int sb = 0; sb < nsub; ++sb) {
            int pos[4];
            for (int t = 0; t < 4; ++t) pos[t] = u[(2 * sb + t) % 8];
            std::sort(pos, pos + 4);
            std::copy(pos, pos + 4, L[0].sub_pos[sb]);
            L[0].m.insert(L[0].m.end(), m4.begin(), m4.end());
        }
        SV_HIP(hipEventSynchronize(s->arena_free));
        const size_t bytes = pack_operands(L, s->dtype, s->stage);
        if (bytes) {
            SV_HIP(s->arena.ensure(bytes));
            SV_HIP(hipMemcpyAsync(s->arena.p, s->stage.p, bytes, hipMemcpyHostToDevice, s->stream));
        }
        rc = enqueue(L, s->dtype, s->buf, s->n, s->arena.p, s->stream);  // warm-up
        if (rc) break;
        SV_HIP(hipEventRecord(a, s->stream));
        for (int r = 0; r < reps && !rc; ++r) rc = enqueue(L, s->dtype, s->buf, s->n, s->arena.p, s->stream);
        SV_HIP(hipEventRecord(b, s->stream));
        SV_HIP(hipEventRecord(s->arena_free, s->stream));
        SV_HIP(hipEventSynchronize(b));
        float ms = 0;
        SV_HIP(hipEventElapsedTime(&ms, a, b));
        total += ms / reps;
        ++count;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc) return rc;
    *ms_out = count ? total / count : 1e30;
    return SV_OK;
}

// ------------------------------------------------------------ tuning cache
// One text line per (architecture, n, precision):
//   sv-tune-1 <arch> <n> <precision> <ms[1..6]> <tile[1..16]> <launch shapes>
// with the launch shapes as reg_grid_cap[0..6] mfma_tc_log[0..6]
// mfma_grid_cap[0..6] split_tc_log[0..6] k4_reg tile_grid_cap tile_bits
// tile_waves.  Saving replaces the line of the same key.
constexpr const char *kTuneTag = "sv-tune-1";
std::mutex g_cache_mu;

int device_arch(int device, std::string &arch)
{
    hipDeviceProp_t prop;
    SV_HIP(hipGetDeviceProperties(&prop, device));
    arch = prop.gcnArchName;
    const size_t colon = arch.find(':');  // drop feature flags (gfx950:sramecc+:xnack-)
    if (colon != std::string::npos) arch.resize(colon);
    return SV_OK;
}

std::string tuning_line(const std::string &arch, int n, int precision, const CostTable &c, const Tuning &t)
{
    std::ostringstream o;
    o.precision(17);
    o << kTuneTag << ' ' << arch << ' ' << n << ' ' << precision;
    for (int k = 1; k <= SV_MAX_K; ++k) o << ' ' << c.ms[k];
    for (int b = 1; b <= kTilePassMaxBlocks; ++b) o << ' ' << c.tile[b];
    for (int k = 0; k <= SV_MAX_K; ++k) o << ' ' << t.reg_grid_cap[k];
    for (int k = 0; k <= SV_MAX_K; ++k) o << ' ' << t.mfma_tc_log[k];
    for (int k = 0; k <= SV_MAX_K; ++k) o << ' ' << t.mfma_grid_cap[k];
    for (int k = 0; k <= SV_MAX_K; ++k) o << ' ' << t.split_tc_log[k];
    o << ' ' << int(t.k4_reg) << ' ' << t.tile_grid_cap << ' ' << t.tile_bits << ' ' << t.tile_waves;
    return o.str();
}

// Parse one line: false for other tags, architectures or malformed lines.
bool parse_tuning_line(const std::string &line, const std::string &arch, int &n, int &precision, double *ms,
                       double *tile, Tuning &t)
{
    std::istringstream in(line);
    std::string tag, a;
    if (!(in >> tag >> a >> n >> precision) || tag != kTuneTag || a != arch) return false;
    if (n < 1 || n > SV_MAX_QUBITS_C64 || precision < SV_PREC_FP32 || precision > SV_PREC_SPLIT_BF16X3) return false;
    ms[0] = tile[0] = 0;
    for (int k = 1; k <= SV_MAX_K; ++k)
        if (!(in >> ms[k]) || !(ms[k] > 0) || !std::isfinite(ms[k])) return false;
    for (int b = 1; b <= kTilePassMaxBlocks; ++b)
        if (!(in >> tile[b]) || !(tile[b] >= 0) || !std::isfinite(tile[b])) return false;
    int k4 = 0;
    for (int k = 0; k <= SV_MAX_K; ++k) in >> t.reg_grid_cap[k];
    for (int k = 0; k <= SV_MAX_K; ++k) in >> t.mfma_tc_log[k];
    for (int k = 0; k <= SV_MAX_K; ++k) in >> t.mfma_grid_cap[k];
    for (int k = 0; k <= SV_MAX_K; ++k) in >> t.split_tc_log[k];
    if (!(in >> k4 >> t.tile_grid_cap >> t.tile_bits >> t.tile_waves)) return false;
    t.k4_reg = k4 != 0;
    for (int k = 0; k <= SV_MAX_K; ++k)
        if (t.reg_grid_cap[k] < 0 || t.mfma_grid_cap[k] < 0 || t.mfma_tc_log[k] < 5 || t.mfma_tc_log[k] > 7 ||
            t.split_tc_log[k] < 5 || t.split_tc_log[k] > 7)
            return false;
    return t.tile_grid_cap >= 1 && dev::tile_shape_supported(t.tile_bits, t.tile_waves);
}

int save_tuning(const char *path, int device, int n, int precision)
{
    std::string arch;
    if (int rc = device_arch(device, arch)) return rc;
    bool found = false;
    const CostTable c = lookup_costs(n, precision, &found);
    if (!found) return fail(SV_ERR_ARG, "no cost table for n = %d, precision %d", n, precision);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    std::vector<std::string> keep;
    {
        std::ifstream in(path);
        std::string line;
        while (std::getline(in, line)) {
            std::istringstream f(line);
            std::string tag, a;
            int ln = -1, lp = -1;
            f >> tag >> a >> ln >> lp;
            if (tag == kTuneTag && a == arch && ln == n && lp == precision) continue;  // replaced below
            if (!line.empty()) keep.push_back(line);
        }
    }
    keep.push_back(tuning_line(arch, n, precision, c, tuning()));
    const std::string tmp = std::string(path) + ".tmp" + std::to_string(::getpid());
    {
        std::ofstream out(tmp);
        for (const auto &l : keep) out << l << '\n';
        if (!out) return fail(SV_ERR_ARG, "cannot write the tuning cache %s", tmp.c_str());
    }
    if (std::rename(tmp.c_str(), path) != 0) {
        std::remove(tmp.c_str());
        return fail(SV_ERR_ARG, "cannot replace the tuning cache %s", path);
    }
    return SV_OK;
}

}  // namespace

namespace sv {

// Install the cost tables of `path` recorded for the device's architecture;
// the launch shapes come from the last such line.  Returns the count.
int load_tuning(const char *path, int device, int *loaded)
{
    std::string arch;
    if (int rc = device_arch(device, arch)) return rc;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    std::ifstream in(path);
    if (!in) return fail(SV_ERR_ARG, "cannot read the tuning cache %s", path);
    std::string line;
    int count = 0;
    Tuning last = tuning();
    while (std::getline(in, line)) {
        int n = 0, precision = 0;
        double ms[SV_MAX_K + 1], tile[kTilePassMaxBlocks + 1];
        Tuning t = tuning();
        if (!parse_tuning_line(line, arch, n, precision, ms, tile, t)) continue;
        store_costs(n, precision, ms, tile);
        last = t;
        ++count;
    }
    if (count) tuning() = last;
    if (loaded) *loaded = count;
    return SV_OK;
}

}  // namespace sv

extern "C" int sv_tune_cache_load(const char *path, int *loaded)
{
    clear_error();
    if (!path) path = std::getenv("SV_TUNE_CACHE");
    if (!path || !*path) return fail(SV_ERR_ARG, "no path given and SV_TUNE_CACHE is not set");
    int device = 0;
    SV_HIP(hipGetDevice(&device));
    return sv::load_tuning(path, device, loaded);
}

extern "C" int sv_autotune(sv_state *s, int precision, double *cost_ms)
{
    clear_error();
    if (!s || !cost_ms) return fail(SV_ERR_ARG, "NULL argument");
    if (precision < SV_PREC_FP32 || precision > SV_PREC_SPLIT_BF16X3) return fail(SV_ERR_ARG, "precision %d", precision);
    if ((s->dtype == SV_C128) != (precision == SV_PREC_FP64))
        return fail(SV_ERR_ARG, "precision %d does not match the state's amplitude type", precision);
    SV_HIP(hipSetDevice(s->device));
    // timing runs must not be recorded by the launch statistics
    timing_suspend(true);
    int rc = SV_OK;
    {
        double amps[4 * SV_MAX_QUBITS_C64];
        for (int p = 0; p < s->n; ++p) {
            amps[4 * p] = amps[4 * p + 2] = 0.70710678118654752440;
            amps[4 * p + 1] = amps[4 * p + 3] = 0.0;
        }
        hipError_t e = dev::launch_product(s->dtype, s->buf, s->n, amps, s->stream);
        if (e != hipSuccess) rc = fail(SV_ERR_HIP, "autotune init: %s", hipGetErrorString(e));
    }
    const int reps = s->n >= 26 ? 3 : 10;
    const int caps[] = {2048, 4096, 8192, 16384, 0};
    const int mcaps[] = {1024, 2048, 4096};
    cost_ms[0] = 0;
    Tuning best_tuning = tuning();
    for (int k = 1; k <= SV_MAX_K && !rc; ++k) {
        std::vector<Cand> cands;
        if (s->dtype == SV_C128) {
            if (k <= 3)
                for (int c : caps) cands.push_back({PATH_REG, c, 0});
            else
                cands.push_back({PATH_GENERIC, 0, 0});
        } else {
            if (k <= 4)
                for (int c : caps) cands.push_back({PATH_REG, c, 0});
            if (k >= 4 && dev::mfma_supported(k, s->n)) {
                Path p = precision == SV_PREC_SPLIT_BF16 ? PATH_SPLIT_BF16
                         : precision == SV_PREC_SPLIT_FP16 ? PATH_SPLIT_FP16 : PATH_MFMA32;
                const bool split = p != PATH_MFMA32;
                for (int tcl = 5; tcl <= 7; ++tcl) {
                    if (k == 6 && tcl > (split ? 5 : 6)) continue;
                    if (split && k == 5 && tcl > 6) continue;
                    if (tcl > s->n - k) continue;
                    for (int c : mcaps) cands.push_back({p, c, tcl});
                }
            }
            if (cands.empty()) cands.push_back({PATH_GENERIC, 0, 0});
        }
        double best = 1e30;
        Cand bc = cands[0];
        for (const auto &c : cands) {
            double ms = 0;
            rc = time_candidate(s, k, c, reps, &ms);
            if (rc) break;
            if (ms < best) {
                best = ms;
                bc = c;
            }
        }
        if (rc) break;
        cost_ms[k] = best;
        if (bc.path == PATH_REG) best_tuning.reg_grid_cap[k] = bc.grid_cap;
        if (bc.path == PATH_MFMA32) {
            best_tuning.mfma_tc_log[k] = bc.tc_log;
            best_tuning.mfma_grid_cap[k] = bc.grid_cap;
        }
        if (bc.path == PATH_SPLIT_BF16 || bc.path == PATH_SPLIT_FP16) {
            best_tuning.split_tc_log[k] = bc.tc_log;
            best_tuning.mfma_grid_cap[k] = bc.grid_cap;
        }
        if (k == 4 && s->dtype == SV_C64 && precision == SV_PREC_FP32) best_tuning.k4_reg = bc.path == PATH_REG;
    }
    double tile_ms[kTilePassMaxBlocks + 1] = {0};
    const bool tiles = !rc && s->dtype == SV_C64 && dev::tile_supported(s->n, 8);
    if (tiles) {
        tuning() = best_tuning;
        const Path tp = tile_path(precision);
        // tile shape: the fastest pass of 4 blocks
        const int shapes[][2] = {{14, 8}, {14, 16}, {13, 4}, {13, 8}};
        double best_shape = 1e30;
        for (const auto &sh : shapes) {
            if (rc || !dev::tile_shape_supported(sh[0], sh[1]) || s->n < sh[0]) continue;
            tuning().tile_bits = sh[0];
            tuning().tile_waves = sh[1];
            double ms = 0;
            rc = time_tile(s, tp, 4, reps, &ms);
            if (!rc && ms < best_shape) {
                best_shape = ms;
                best_tuning.tile_bits = sh[0];
                best_tuning.tile_waves = sh[1];
            }
        }
        tuning() = best_tuning;
        for (int nsub = 1; nsub <= dev::kMaxTileSubBlocks && !rc; ++nsub) rc = time_tile(s, tp, nsub, reps, &tile_ms[nsub]);
    }
    timing_suspend(false);
    if (rc) return rc;
    tuning() = best_tuning;
    store_costs(s->n, precision, cost_ms, tiles ? tile_ms : nullptr);
    if (const char *path = std::getenv("SV_TUNE_CACHE"))
        if (*path) return save_tuning(path, s->device, s->n, precision);
    return SV_OK;
}

extern "C" int sv_set_cost_table(int n, int precision, const double *cost_ms)
{
    clear_error();
    if (n < 1 || n > SV_MAX_QUBITS_C64) return fail(SV_ERR_ARG, "n = %d", n);
    if (precision < SV_PREC_FP32 || precision > SV_PREC_SPLIT_BF16X3) return fail(SV_ERR_ARG, "precision %d", precision);
    if (!cost_ms) return fail(SV_ERR_ARG, "NULL cost table");
    for (int k = 1; k <= SV_MAX_K; ++k)
        if (!(cost_ms[k] > 0) || !std::isfinite(cost_ms[k])) return fail(SV_ERR_ARG, "cost_ms[%d] must be positive", k);
    store_costs(n, precision, cost_ms);
    return SV_OK;
}

extern "C" int sv_set_tile_shape(int tile_bits, int waves)
{
    clear_error();
    if (!dev::tile_shape_supported(tile_bits, waves))
        return fail(SV_ERR_ARG, "tile shape (%d bits, %d waves) is not one of (14, 8), (14, 16), (13, 4), (13, 8)",
                    tile_bits, waves);
    tuning().tile_bits = tile_bits;
    tuning().tile_waves = waves;
    return SV_OK;
}

extern "C" int sv_get_tile_shape(int *tile_bits, int *waves, int *max_blocks)
{
    clear_error();
    const Tuning &t = tuning();
    if (tile_bits) *tile_bits = t.tile_bits;
    if (waves) *waves = t.tile_waves;
    if (max_blocks) *max_blocks = dev::tile_max_blocks(t.tile_bits, t.tile_waves, dev::kTileOperandBF16);
    return SV_OK;
}

extern "C" int sv_tile_placement(int n_sub, const int32_t *sub_pos, int n, int tile_bits, int waves, int precision,
                                 int32_t *tile_pos, uint32_t *lds_image, int32_t *conflicts)
{
    clear_error();
    if (!sub_pos || !tile_pos || !lds_image) return fail(SV_ERR_ARG, "NULL argument");
    if (!dev::tile_shape_supported(tile_bits, waves))
        return fail(SV_ERR_ARG, "tile shape (%d bits, %d waves) is not supported", tile_bits, waves);
    if (precision < SV_PREC_FP32 || precision > SV_PREC_SPLIT_BF16X3 || precision == SV_PREC_FP64)
        return fail(SV_ERR_ARG, "precision %d has no tile passes", precision);
    if (n_sub < 1 || n_sub > dev::kMaxTileSubBlocks) return fail(SV_ERR_ARG, "n_sub = %d", n_sub);
    if (n < tile_bits || n > SV_MAX_QUBITS_C64) return fail(SV_ERR_ARG, "n = %d", n);
    int pos[dev::kMaxTileSubBlocks][4];
    for (int s = 0; s < n_sub; ++s)
        for (int i = 0; i < 4; ++i) pos[s][i] = sub_pos[4 * s + i];
    dev::TileArgs a;
    const int tprec = tile_operand_prec(tile_path(precision));
    if (dev::make_tile_args(n_sub, pos, n, tile_bits, waves, tprec, &a) != hipSuccess)
        return fail(SV_ERR_ARG, "blocks need 4 ascending positions below n, with a union of at most %d",
                    tile_bits);
    for (int b = 0; b < tile_bits; ++b) {
        tile_pos[b] = a.ubit[b];
        lds_image[b] = a.swz[b];
    }
    if (conflicts) *conflicts = dev::tile_placement_conflicts(a, tile_bits, waves, tprec);
    return SV_OK;
}

extern "C" int sv_set_tile_union(int max_positions)
{
    clear_error();
    if (max_positions < 8 || max_positions > kTilePassMaxUnion)
        return fail(SV_ERR_ARG, "tile union %d outside 8..%d", max_positions, kTilePassMaxUnion);
    set_tile_union_limit(max_positions);
    return SV_OK;
}
